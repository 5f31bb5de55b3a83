"""Oracle: plain FP64 Kaczmarz++ (exact Cholesky projection) and CD++ (no RHT).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Each function follows one passage of the paper and is written for a reader to
check by eye; nothing is blocked, fused or reordered beyond what that passage
states.  numpy's matmul, Cholesky and scipy's triangular solve serve as library
steps.

Notation: A (m x n), b (m), block S (sorted row indices), s = |S|, lambda >= 0,
x the iterate, mom the momentum vector m_t, rho, eta the acceleration
parameters.

Readings of the paper taken here (each listed in the design notes):
  * eta defaults to s / (2 min(m, n)) for Kaczmarz++ and s / (2 n) for CD++
    (Section 5.4 derives eta ~ s/n from nu = O~(n/s); for a wide Kaczmarz++
    system the variance parameter scales with the rank min(m, n)).
  * The two window sums of Algorithms 2 and 5 are read as: step t adds ||r_t||^2
    to E0 when (t mod 2 zeta) < zeta, else to E1; the checkpoint is the step
    with (t mod 2 zeta) == 2 zeta - 1.  zeta = ceil(m / s) (Kaczmarz++,
    Algorithm 5) or ceil(n / s) (CD++, Algorithm 2).
  * The weighted average of eq. (weighted): checkpoint i = 0, 1, ... takes the
    first ratio as is, then r_hat_i = w_i r_hat_{i-1} + (1 - w_i) q_i with
    w_i = a(i-1) / a(i), a(j) = (j + 1)^{ln(j + 1)}.
  * rho = 1 - r_hat^(1/zeta), clamped to [0, 1] (rho lies in [0, 1] in eq.
    (momentum)); a checkpoint whose first window sum E0 is zero leaves rho
    and r_hat unchanged.
  * A candidate stop (E1 <= eps^2 ||b||^2, Algorithms 2 and 5) is confirmed
    with the true residual ||A x - b|| <= eps ||b|| (eq. (residual-error));
    if that fails the run continues and the checkpoint updates rho as usual.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg

from .schedule import Schedule

# ----------------------------------------------------------------------------
# one block step, piece by piece
# ----------------------------------------------------------------------------


def block_residual(A: np.ndarray, b: np.ndarray, S: np.ndarray, x: np.ndarray,
                   reverse: bool = False) -> np.ndarray:
    """r = A_S x - b_S  (Algorithm 5 / Algorithm 2: "r_t <- A_S x_t - b_S").

    reverse=True sums over the columns in the opposite order (same value in
    exact arithmetic); used only to measure the FP64 rounding noise floor."""
    if reverse:
        return A[S, ::-1] @ x[::-1] - b[S]
    return A[S, :] @ x - b[S]


def regularized_gram(A: np.ndarray, S: np.ndarray, lam: float, kind: str,
                     reverse: bool = False) -> np.ndarray:
    """G = A_S A_S^T + lam I (eq. (bk)), or A_{S,S} + lam I for CD++ (eq. (cd-update))."""
    if kind == "psd":
        G = A[np.ix_(S, S)].copy()
    else:
        AS = A[S, ::-1] if reverse else A[S, :]
        G = AS @ AS.T
    G[np.diag_indices_from(G)] += lam
    return G


class NotSPD(ArithmeticError):
    """The regularized block Gram has no Cholesky factor."""


def cholesky_lower(G: np.ndarray) -> np.ndarray:
    """L with L L^T = G (the memoized factor R[S] of Algorithms 1 and 2)."""
    try:
        return np.linalg.cholesky(G)
    except np.linalg.LinAlgError as e:  # pragma: no cover - exercised by tests
        raise NotSPD(str(e)) from e


def projection_solve(L: np.ndarray, r: np.ndarray) -> np.ndarray:
    """y = (L L^T)^{-1} r by a forward then a backward triangular solve."""
    z = scipy.linalg.solve_triangular(L, r, lower=True)
    return scipy.linalg.solve_triangular(L.T, z, lower=False)


def direction(A: np.ndarray, S: np.ndarray, y: np.ndarray, kind: str,
              reverse: bool = False) -> np.ndarray:
    """w = A_S^T y (eq. (bk)) or w = I_S^T y (eq. (cd-update))."""
    if kind == "psd":
        w = np.zeros(A.shape[1])
        w[S] = y
        return w
    if reverse:
        return A[S[::-1], :].T @ y[::-1]
    return A[S, :].T @ y


def momentum_update(x: np.ndarray, mom: np.ndarray, w: np.ndarray, rho: float, eta: float):
    """m <- (1-rho)/(1+rho) (m - w);  x <- x - w + eta m   (eq. (momentum), Alg. 1)."""
    c = (1.0 - rho) / (1.0 + rho)
    mom_new = c * (mom - w)
    x_new = x - w + eta * mom_new
    return x_new, mom_new


def regularized_projection(A, b, S, x, lam, kind="general"):
    """w_t of eq. (bk) / eq. (cd-update) in one call (unmemoized)."""
    r = block_residual(A, b, S, x)
    L = cholesky_lower(regularized_gram(A, S, lam, kind))
    return direction(A, S, projection_solve(L, r), kind)


# ----------------------------------------------------------------------------
# adaptive acceleration (Section 5.4)
# ----------------------------------------------------------------------------


def averaging_weight(i: int) -> float:
    """w_i = a(i-1)/a(i) with a(j) = (j+1)^{ln(j+1)}; w_0 = 0 (eq. (weighted))."""
    if i <= 0:
        return 0.0
    return math.exp(math.log(i) ** 2 - math.log(i + 1) ** 2)


def rho_from_rate(r_hat: float, zeta: int) -> float:
    """rho = 1 - r_hat^(1/zeta), clamped to [0, 1] (Algorithm 2, Section 5.4)."""
    if not (r_hat < 1.0):
        return 0.0
    return min(1.0, max(0.0, 1.0 - r_hat ** (1.0 / zeta)))


def default_eta(kind: str, m: int, n: int, s: int) -> float:
    if kind == "psd":
        return s / (2.0 * n)
    return s / (2.0 * min(m, n))


def default_zeta(kind: str, m: int, n: int, s: int) -> int:
    return -(-(n if kind == "psd" else m) // s)


# ----------------------------------------------------------------------------
# the solver loop
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Params:
    s: int
    lam: float = 1e-8
    tol: float = 1e-10
    max_iters: int = 100_000
    eta: Optional[float] = None       # None -> default_eta
    accel: bool = True                # False: eta = 0 ("without acceleration")
    adaptive_rho: bool = True
    rho0: float = 0.0
    memo: bool = True                 # False: refactor at every step
    confirm_true_residual: bool = True
    reverse_sums: bool = False        # noise-floor probe: every sum in the opposite order


@dataclasses.dataclass
class Result:
    x: np.ndarray
    iters: int
    converged: bool
    rho_final: float
    est_rel_res: float
    true_rel_res: float
    factorizations: int
    memo_hits: int
    flops: float
    checkpoints: List[dict]
    snapshots: Dict[int, np.ndarray]


def solve(A: np.ndarray, b: np.ndarray, kind: str, params: Params, schedule: Schedule,
          x0: Optional[np.ndarray] = None, snapshot_steps=(), record_checkpoint_x=False,
          proj=None) -> Result:
    """Kaczmarz++ (Algorithm 5, exact projection) or CD++ (Algorithm 2, no RHT).

    `snapshot_steps`: step counts t at which x_t (the iterate after t steps)
    is stored in Result.snapshots.  `proj`: another projection for
    Kaczmarz++ (an object with factor(A, S), direction(A, S, F, r),
    factor_flops(sb, n) and step_flops(sb, n); the inexact Proj of Algorithm 5
    in oracle/lsqr.py); None is the exact memoized Cholesky projection.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    if kind == "psd" and m != n:
        raise ValueError("CD++ needs a square matrix")
    s = params.s
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    mom = np.zeros(n)
    eta = default_eta(kind, m, n, s) if params.eta is None else float(params.eta)
    if not params.accel:
        eta = 0.0
    zeta = default_zeta(kind, m, n, s)
    rho = float(params.rho0)
    r_hat = None
    ckpt = 0
    E0 = E1 = 0.0
    bb = float(b @ b)
    thr = params.tol ** 2 * bb
    factors: Dict[int, np.ndarray] = {}
    nfact = hits = 0
    flops = 0.0
    checkpoints: List[dict] = []
    snaps: Dict[int, np.ndarray] = {}
    snap_set = set(int(t) for t in snapshot_steps)
    if 0 in snap_set:
        snaps[0] = x.copy()
    converged = False
    true_rel = math.nan
    est_rel = math.nan
    t = 0
    for t in range(params.max_iters):
        bid = int(schedule.step_block[t])
        S = schedule.blocks[bid]
        sb = len(S)
        rev = params.reverse_sums
        r = block_residual(A, b, S, x, reverse=rev)
        if params.memo and bid in factors:
            L = factors[bid]
            hits += 1
        else:
            if proj is not None:
                L = proj.factor(A, S)
                flops += proj.factor_flops(sb, n)
            else:
                L = cholesky_lower(regularized_gram(A, S, params.lam, kind, reverse=rev))
                flops += sb ** 3 / 3.0 + (sb * sb * n if kind != "psd" else 0.0)
            nfact += 1
            if params.memo:
                factors[bid] = L
        if proj is not None:
            w = proj.direction(A, S, L, r)
            flops += proj.step_flops(sb, n)
        else:
            y = projection_solve(L, r)
            w = direction(A, S, y, kind, reverse=rev)
            flops += 2.0 * sb * n + 2.0 * sb * sb + (2.0 * sb * n if kind != "psd" else 0.0) + 5.0 * n
        x, mom = momentum_update(x, mom, w, rho, eta)
        if t + 1 in snap_set:
            snaps[t + 1] = x.copy()
        rr = float(r @ r)
        phase = t % (2 * zeta)
        if phase < zeta:
            E0 += rr
        else:
            E1 += rr
        if phase == 2 * zeta - 1:
            rec = dict(t=t, E0=E0, E1=E1, rho_used=rho)
            est_rel = math.sqrt(E1 / bb) if bb > 0 else math.sqrt(E1)
            if E1 <= thr:
                if params.confirm_true_residual:
                    res = float(np.linalg.norm(A @ x - b))
                    true_rel = res / math.sqrt(bb) if bb > 0 else res
                    rec["true_rel"] = true_rel
                    if res <= params.tol * math.sqrt(bb):
                        converged = True
                else:
                    converged = True
            if not converged and params.adaptive_rho and E0 > 0.0:
                q = E1 / E0
                wgt = averaging_weight(ckpt)
                r_hat = q if r_hat is None else wgt * r_hat + (1.0 - wgt) * q
                ckpt += 1
                rho = rho_from_rate(r_hat, zeta)
            rec["rho_next"] = rho
            if record_checkpoint_x:
                rec["x"] = x.copy()
            checkpoints.append(rec)
            E0 = E1 = 0.0
            if converged:
                break
    iters = t + 1 if params.max_iters > 0 else 0
    if not converged or math.isnan(true_rel):
        res = float(np.linalg.norm(A @ x - b))
        true_rel = res / math.sqrt(bb) if bb > 0 else res
    return Result(x=x, iters=iters, converged=converged, rho_final=rho, est_rel_res=est_rel,
                  true_rel_res=true_rel, factorizations=nfact, memo_hits=hits, flops=flops,
                  checkpoints=checkpoints, snapshots=snaps)


# ----------------------------------------------------------------------------
# mixed-precision iterative refinement (outer loop in FP64)
# ----------------------------------------------------------------------------


def refine(A, b, kind, inner_solve, tol=1e-10, max_rounds=20, x0=None):
    """x <- x + d, with d an approximate solution of A d = b - A x, until
    ||b - A x|| <= tol ||b||.  `inner_solve(rhs)` returns d.  Residual and
    accumulation are FP64 (classical iterative refinement)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(A.shape[1]) if x0 is None else np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    hist = []
    for k in range(max_rounds):
        res = b - A @ x
        rel = float(np.linalg.norm(res)) / (nb if nb > 0 else 1.0)
        hist.append(rel)
        if rel <= tol:
            return x, hist, True
        x = x + inner_solve(res)
    res = b - A @ x
    hist.append(float(np.linalg.norm(res)) / (nb if nb > 0 else 1.0))
    return x, hist, hist[-1] <= tol
