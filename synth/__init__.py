"""Seeded synthetic linear systems with outlying singular values / eigenvalues.

This module only draws inputs.  It holds none of the solver's arithmetic and is
the one piece of code shared by the CPU oracle (``oracle/``), the tests and the
benchmark.  Every system is consistent (b = A x*), as the convergence theory of
the paper assumes (Section 2, Theorem 2.1).

Recipes (all seeded; numpy ``default_rng(seed)`` on the CPU, a seeded
``torch.Generator`` when a torch device is requested for the large sizes):

* Haar-random orthonormal columns: QR of a standard Gaussian matrix with the
  signs of R's diagonal moved into Q (Mezzadri's fix), so the result is
  Haar-distributed.
* General systems (Kaczmarz++): A = U diag(sigma) V^T with U (m x r) and
  V (n x r) Haar columns, r = min(m, n).  x* ~ N(0, I) (over-determined) or
  x* = V g, g ~ N(0, I_r) (under-determined, so x* is the minimum-norm
  solution).  b = A x*.
* PSD systems (CD++): A = Q diag(lambda) Q^T, symmetrised as (A + A^T)/2,
  x* ~ N(0, I), b = A x*.

* Kernel systems (the setting of the paper's FLOP comparison, Section 6.3):
  n points phi_i ~ N(0, I_d), A = K + phi I with K_ij = exp(-gamma ||phi_i -
  phi_j||^2) (Gaussian) or exp(-gamma ||phi_i - phi_j||) (Laplacian),
  b ~ N(0, I).  A is positive definite, so the system is consistent, but x* is
  not planted (xstar is None).

The spectra follow the paper's experimental premise (Section 6): a few large
outliers over a flat or decaying bulk.  The paper's own matrices (the
scikit-learn low-rank generator and four ML data sets, Section 6.1) are not
available; these seeded systems stand in for them.

Draw order inside one recipe is fixed: spectrum bulk, then U (or Q), then V,
then x* -- so a change to one size never silently reshuffles another.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "System",
    "haar_columns",
    "svd_system",
    "psd_system",
    "spectrum_c1",
    "spectrum_c2",
    "spectrum_c3",
    "spectrum_c4",
    "config",
    "CONFIGS",
    "tiny_system",
    "serving_workload",
    "kernel_system",
]


@dataclasses.dataclass
class System:
    """A consistent system A x = b with its planted solution and metadata."""

    A: object          # numpy (m, n) float64, or a torch tensor on `device`
    b: object          # (m,)
    xstar: object      # (n,)
    kind: str          # "general" (Kaczmarz++) or "psd" (CD++)
    name: str
    spectrum: np.ndarray
    params: dict

    @property
    def shape(self):
        return tuple(self.A.shape)


# ----------------------------------------------------------------------------
# spectra (numpy, always on the CPU: they are small)
# ----------------------------------------------------------------------------

def spectrum_c1(rng: np.random.Generator, n: int = 200, n_out: int = 10) -> np.ndarray:
    """10 outliers log-spaced in [1e2, 1e3], the rest i.i.d. U[1, 2]."""
    bulk = rng.uniform(1.0, 2.0, size=n - n_out)
    return np.concatenate([np.geomspace(1e2, 1e3, n_out), bulk])


def spectrum_c2(rng: np.random.Generator, n: int = 4096, n_out: int = 32) -> np.ndarray:
    """Eigenvalues: 32 outliers log-spaced in [1e3, 1e5], the rest U[1, 10]."""
    bulk = rng.uniform(1.0, 10.0, size=n - n_out)
    return np.concatenate([np.geomspace(1e3, 1e5, n_out), bulk])


def spectrum_c3(rng: np.random.Generator, r: int = 2048, n_out: int = 50) -> np.ndarray:
    """50 outliers log-spaced in [1e2, 1e4], the rest 1/(1 + 0.01 i), i = 0.."""
    del rng  # deterministic spectrum
    tail = 1.0 / (1.0 + 0.01 * np.arange(r - n_out))
    return np.concatenate([np.geomspace(1e2, 1e4, n_out), tail])


def spectrum_c4(rng: np.random.Generator, r: int = 2048, n_out: int = 20) -> np.ndarray:
    """20 outliers log-spaced in [1e3, 1e4], the rest i.i.d. U[0.5, 1]."""
    bulk = rng.uniform(0.5, 1.0, size=r - n_out)
    return np.concatenate([np.geomspace(1e3, 1e4, n_out), bulk])


# ----------------------------------------------------------------------------
# random orthonormal factors
# ----------------------------------------------------------------------------

def haar_columns(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """n x k matrix with Haar-distributed orthonormal columns (k <= n)."""
    g = rng.standard_normal((n, k))
    q, r = np.linalg.qr(g, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def _torch_haar_columns(gen, n: int, k: int, device):
    import torch

    g = torch.randn((n, k), dtype=torch.float64, device=device, generator=gen)
    q, r = torch.linalg.qr(g, mode="reduced")
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1.0
    return q * d


# ----------------------------------------------------------------------------
# systems
# ----------------------------------------------------------------------------

def svd_system(m: int, n: int, sigma_fn, seed: int, *, x_in_rowspace: bool = False,
               device: Optional[str] = None, name: str = "svd") -> System:
    """A = U diag(sigma) V^T (m x n, rank r = min(m, n)), b = A x*."""
    r = min(m, n)
    rng = np.random.default_rng(seed)
    sigma = np.asarray(sigma_fn(rng, r), dtype=np.float64)
    assert sigma.shape == (r,)
    if device is None:
        U = haar_columns(rng, m, r)
        V = haar_columns(rng, n, r)
        A = (U * sigma) @ V.T
        if x_in_rowspace:
            xstar = V @ rng.standard_normal(r)
        else:
            xstar = rng.standard_normal(n)
        b = A @ xstar
    else:
        import torch

        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed))
        U = _torch_haar_columns(gen, m, r, device)
        V = _torch_haar_columns(gen, n, r, device)
        sig = torch.as_tensor(sigma, device=device)
        A = ((U * sig) @ V.T).contiguous()
        del U
        if x_in_rowspace:
            xstar = V @ torch.randn(r, dtype=torch.float64, device=device, generator=gen)
        else:
            xstar = torch.randn(n, dtype=torch.float64, device=device, generator=gen)
        del V
        b = A @ xstar
    return System(A=A, b=b, xstar=xstar, kind="general", name=name, spectrum=sigma,
                  params=dict(m=m, n=n, seed=seed, x_in_rowspace=x_in_rowspace))


def psd_system(n: int, eig_fn, seed: int, *, device: Optional[str] = None,
               name: str = "psd") -> System:
    """A = Q diag(lambda) Q^T symmetrised, b = A x*, x* ~ N(0, I)."""
    rng = np.random.default_rng(seed)
    lam = np.asarray(eig_fn(rng, n), dtype=np.float64)
    assert lam.shape == (n,)
    if device is None:
        Q = haar_columns(rng, n, n)
        A = (Q * lam) @ Q.T
        A = 0.5 * (A + A.T)
        xstar = rng.standard_normal(n)
        b = A @ xstar
    else:
        import torch

        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed))
        Q = _torch_haar_columns(gen, n, n, device)
        A = (Q * torch.as_tensor(lam, device=device)) @ Q.T
        A = (0.5 * (A + A.T)).contiguous()
        del Q
        xstar = torch.randn(n, dtype=torch.float64, device=device, generator=gen)
        b = A @ xstar
    return System(A=A, b=b, xstar=xstar, kind="psd", name=name, spectrum=lam,
                  params=dict(n=n, seed=seed))


def kernel_system(kernel: str, n: int, gamma: float, *, d: int = 8, phi: float = 1e-3, seed: int = 0,
                  device: Optional[str] = None) -> System:
    """Kernel matrix plus phi I on n seeded Gaussian points in d dimensions
    (Section 6.1, "Kernel Matrices from Machine Learning", with synthetic
    features in place of the data sets); b ~ N(0, I)."""
    if kernel not in ("gaussian", "laplacian"):
        raise ValueError("kernel must be gaussian or laplacian")
    if device is None:
        rng = np.random.default_rng(seed)
        F = rng.standard_normal((n, d))
        sq = np.maximum((F * F).sum(1)[:, None] + (F * F).sum(1)[None, :] - 2.0 * F @ F.T, 0.0)
        np.fill_diagonal(sq, 0.0)
        K = np.exp(-gamma * sq) if kernel == "gaussian" else np.exp(-gamma * np.sqrt(sq))
        A = 0.5 * (K + K.T) + phi * np.eye(n)
        b = rng.standard_normal(n)
    else:
        import torch

        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed))
        F = torch.randn((n, d), dtype=torch.float64, device=device, generator=gen)
        nrm = (F * F).sum(1)
        sq = torch.clamp(nrm[:, None] + nrm[None, :] - 2.0 * (F @ F.T), min=0.0)
        sq.fill_diagonal_(0.0)
        K = torch.exp(-gamma * sq) if kernel == "gaussian" else torch.exp(-gamma * torch.sqrt(sq))
        del sq
        A = (0.5 * (K + K.T)).contiguous()
        del K
        A.diagonal().add_(phi)
        b = torch.randn(n, dtype=torch.float64, device=device, generator=gen)
    return System(A=A, b=b, xstar=None, kind="psd", name=f"{kernel}_g{gamma:g}_n{n}", spectrum=np.zeros(0),
                  params=dict(n=n, d=d, gamma=gamma, phi=phi, seed=seed))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
# Each entry: builder + the solver parameters the workload is run with.
# "scale" variants keep the spectrum's shape (same outlier count and ranges)
# at sizes the CPU oracle finishes in seconds.

CONFIGS = {
    # dense consistent 1000 x 200, Kaczmarz++, block 20, lambda 1e-3, online memo
    "c1": dict(kind="general", m=1000, n=200, spectrum=spectrum_c1, seed=1,
               s=20, lam=1e-3, memo="online", schedule_seed=101, eta=None),
    # SPD n = 4096, CD++, block 128, fixed partition into 32 blocks, lambda 1e-8
    "c2": dict(kind="psd", n=4096, spectrum=spectrum_c2, seed=2,
               s=128, lam=1e-8, memo="fixed", partition=True, schedule_seed=202, eta=None),
    # over-determined 65536 x 2048, Kaczmarz++, block 256, fixed partition (256 blocks)
    "c3": dict(kind="general", m=65536, n=2048, spectrum=spectrum_c3, seed=3,
               s=256, lam=1e-8, memo="fixed", partition=True, schedule_seed=303, eta=None),
    # under-determined 2048 x 32768, Kaczmarz++, block 128, lambda 1e-4, online memo
    "c4": dict(kind="general", m=2048, n=32768, spectrum=spectrum_c4, seed=4,
               s=128, lam=1e-4, memo="online", schedule_seed=404, eta=None, x_in_rowspace=True),
    # reduced sizes with the same spectral shape (parity cases the oracle runs in seconds);
    # sizes chosen so blocks and tiles have ragged tails
    "c2_small": dict(kind="psd", n=1000, spectrum=spectrum_c2, seed=12,
                     s=128, lam=1e-8, memo="fixed", partition=True, schedule_seed=212, eta=None),
    "c3_small": dict(kind="general", m=6000, n=700, spectrum=spectrum_c3, seed=13,
                     s=256, lam=1e-8, memo="fixed", partition=True, schedule_seed=313, eta=None),
    "c4_small": dict(kind="general", m=300, n=5000, spectrum=spectrum_c4, seed=14,
                     s=64, lam=1e-4, memo="online", schedule_seed=414, eta=None, x_in_rowspace=True),
}


def config(name: str, device: Optional[str] = None) -> System:
    """Build the named workload (see CONFIGS)."""
    c = CONFIGS[name]
    if c["kind"] == "psd":
        n_out = 32
        fn = lambda rng, n: c["spectrum"](rng, n, n_out)  # noqa: E731
        sysm = psd_system(c["n"], fn, c["seed"], device=device, name=name)
    else:
        sysm = svd_system(c["m"], c["n"], c["spectrum"], c["seed"],
                          x_in_rowspace=c.get("x_in_rowspace", False),
                          device=device, name=name)
    sysm.params.update({k: v for k, v in c.items() if k not in ("spectrum",)})
    return sysm


def tiny_system(kind: str, m: int, n: int, seed: int, cond: float = 10.0,
                x_in_rowspace: Optional[bool] = None) -> System:
    """Small well-conditioned system (kappa(A) <= cond) for exact-arithmetic pins.

    Singular values (or eigenvalues) are log-spaced in [1, cond].
    """
    if kind == "psd":
        assert m == n
        fn = lambda rng, r: np.geomspace(1.0, cond, r)  # noqa: E731
        return psd_system(n, fn, seed, name=f"tiny_psd_{n}")
    if x_in_rowspace is None:
        x_in_rowspace = m < n
    fn = lambda rng, r: np.geomspace(1.0, cond, r)  # noqa: E731
    return svd_system(m, n, fn, seed, x_in_rowspace=x_in_rowspace,
                      name=f"tiny_general_{m}x{n}")


def serving_workload(num_requests: int = 512, rate_per_s: float = 200.0, seed: int = 5,
                     sizes=(512, 1024, 2048, 4096, 8192), tols=(1e-6, 1e-10),
                     pool_per_size: int = 8):
    """Arrival process for the serving workload.

    Returns a list of dicts {arrival_s, n, pool_index, tol, x_seed}: Poisson
    arrivals (exponential gaps of mean 1/rate), sizes and tolerances uniform
    over the given sets, each request pointing at one of `pool_per_size`
    distinct PSD matrices of its size (spectrum as in the n = 4096 CD++
    workload: 32 outliers in [1e3, 1e5], bulk U[1, 10]).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=num_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = rng.choice(np.asarray(sizes), size=num_requests)
    pools = rng.integers(0, pool_per_size, size=num_requests)
    tl = rng.choice(np.asarray(tols), size=num_requests)
    return [dict(arrival_s=float(arrivals[i]), n=int(ns[i]), pool_index=int(pools[i]),
                 tol=float(tl[i]), x_seed=int(seed * 100003 + i))
            for i in range(num_requests)]


def serving_matrix(n: int, pool_index: int, device: Optional[str] = None) -> System:
    """The pool_index-th PSD matrix of size n used by the serving workload."""
    fn = lambda rng, nn: spectrum_c2(rng, nn, 32)  # noqa: E731
    return psd_system(n, fn, seed=50_000 + 97 * n + pool_index, device=device,
                      name=f"serve_{n}_{pool_index}")


# ----------------------------------------------------------------------------
# sparse systems (compressed sparse rows)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class SparseSystem:
    """A consistent sparse system in CSR form: int64 row pointers, int32
    column indices (strictly increasing within each row), float64 values."""

    rp: np.ndarray
    ci: np.ndarray
    cv: np.ndarray
    b: np.ndarray
    xstar: np.ndarray
    m: int
    n: int
    kind: str          # "general" (Kaczmarz++) or "psd" (CD++)
    name: str
    params: dict

    @property
    def shape(self):
        return (self.m, self.n)

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    def dense(self) -> np.ndarray:
        A = np.zeros((self.m, self.n))
        rows = np.repeat(np.arange(self.m), np.diff(self.rp))
        A[rows, self.ci] = self.cv
        return A

    def to(self, device):
        """(rp, ci, cv, b) as torch tensors on `device`."""
        import torch

        return (torch.from_numpy(self.rp).to(device), torch.from_numpy(self.ci).to(device),
                torch.from_numpy(self.cv).to(device), torch.from_numpy(self.b).to(device))


def _csr_from_coo(m: int, n: int, r: np.ndarray, c: np.ndarray, v: np.ndarray):
    import scipy.sparse as sp

    A = sp.coo_matrix((v, (r, c)), shape=(m, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64), A


def sparse_general(m: int, n: int, per_row: int, seed: int, *, outlier_frac: float = 0.02,
                   outlier_scale: float = 10.0, empty_every: int = 0,
                   x_in_rowspace: Optional[bool] = None, name: str = "") -> SparseSystem:
    """Kaczmarz++ input: every row holds `per_row` draws of a uniform column
    (duplicates merged, so a row may hold fewer) with N(0, 1) values; a
    fraction `outlier_frac` of the rows (chosen uniformly) is scaled by
    `outlier_scale`, which puts a few large outlying singular values over the
    bulk; with empty_every = k > 0, rows k-1, 2k-1, ... are empty.  x* ~ N(0, I)
    (over-determined) or x* = A^T g, g ~ N(0, I) (under-determined: the
    minimum-norm solution); b = A x*.  Draw order: columns, values, outlier
    rows, x*."""
    rng = np.random.default_rng(seed)
    cols = rng.integers(0, n, size=(m, per_row))
    vals = rng.standard_normal((m, per_row))
    scale = np.ones(m)
    n_out = int(round(outlier_frac * m))
    if n_out:
        scale[rng.choice(m, size=n_out, replace=False)] = outlier_scale
    vals *= scale[:, None]
    keep = np.ones((m, per_row), dtype=bool)
    if empty_every > 0:
        keep[empty_every - 1::empty_every, :] = False
    r = np.repeat(np.arange(m), per_row).reshape(m, per_row)
    rp, ci, cv, A = _csr_from_coo(m, n, r[keep], cols[keep], vals[keep])
    if x_in_rowspace is None:
        x_in_rowspace = m < n
    if x_in_rowspace:
        xs = np.asarray(A.T @ rng.standard_normal(m)).ravel()
    else:
        xs = rng.standard_normal(n)
    b = np.asarray(A @ xs).ravel()
    return SparseSystem(rp, ci, cv, b, xs, m, n, "general", name or f"sparse_general_{m}x{n}",
                        dict(per_row=per_row, seed=seed, outlier_frac=outlier_frac,
                             outlier_scale=outlier_scale, empty_every=empty_every))


def sparse_psd(n: int, degree: int, seed: int, *, hubs: int = 4, hub_degree: int = 0, phi: float = 0.1,
               name: str = "") -> SparseSystem:
    """CD++ input: A = L + phi I with L the Laplacian of a random weighted
    graph.  Every node links to `degree` uniform partners (weights U(0.5,
    1.5), links made symmetric, repeats merged); `hubs` nodes (chosen
    uniformly) link to `hub_degree` more (default 20 * degree), which gives a
    few large outlying eigenvalues over the bulk.  A is symmetric positive
    definite (eigenvalues >= phi).  x* ~ N(0, I), b = A x*.  Draw order:
    partners, weights, hubs, hub partners, hub weights, x*."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    src = np.repeat(np.arange(n), degree)
    dst = rng.integers(0, n, size=n * degree)
    w = rng.uniform(0.5, 1.5, size=n * degree)
    hd = hub_degree or 20 * degree
    if hubs:
        hub = rng.choice(n, size=hubs, replace=False)
        hs = np.repeat(hub, hd)
        ht = rng.integers(0, n, size=hubs * hd)
        hw = rng.uniform(0.5, 1.5, size=hubs * hd)
        src, dst, w = np.concatenate([src, hs]), np.concatenate([dst, ht]), np.concatenate([w, hw])
    off = src != dst
    src, dst, w = src[off], dst[off], w[off]
    W = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([src, dst]), np.concatenate([dst, src]))),
                      shape=(n, n)).tocsr()
    W.sum_duplicates()
    deg = np.asarray(W.sum(axis=1)).ravel()
    A = (sp.diags(deg + phi) - W).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    xs = rng.standard_normal(n)
    b = np.asarray(A @ xs).ravel()
    return SparseSystem(A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64), b, xs,
                        n, n, "psd", name or f"sparse_psd_{n}",
                        dict(degree=degree, seed=seed, hubs=hubs, hub_degree=hd, phi=phi))
