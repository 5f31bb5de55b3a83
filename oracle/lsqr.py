"""Oracle sketch-preconditioned LSQR projection: the inexact Proj of
Kaczmarz++ (Section 4.1, "Computing the Projection Step"; the Proj routine
called by Algorithm 5).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What is computed
  * On a block S not yet in the collection: the sketch A_hat = A_S Pi^T with
    Pi the subsampled randomized Hadamard transform sqrt(N / tau) I_T H D of
    Lemma l:inner (D = diag(d) / sqrt(N) with Rademacher signs, T a uniformly
    random tau-subset of the N rows of H), and the Cholesky factor of
    A_hat A_hat^T + lambda I, saved for S.  With L that lower factor the
    paper's R is L^T, so R^{-T} = L^{-1}.
  * Every step: the first n entries of LSQR run for t_max iterations from zero
    on min || M z - L^{-1} r ||, M = L^{-1} [A_S, sqrt(lambda) I] (eq. (lsqr)).
    With t_max at least the rank, LSQR reaches the minimum-norm solution,
    whose first n entries are the exact projection A_S^T (A_S A_S^T +
    lambda I)^{-1} r whatever the preconditioner.
  * LSQR is Paige and Saunders' algorithm (ACM TOMS 8, 1982): Golub-Kahan
    bidiagonalization of M started from the right-hand side, with the
    QR factorization of the bidiagonal matrix updated by one plane rotation
    per iteration.  Written here from that published description.

Readings (listed in the design notes)
  * n is padded with zero columns to N, the next power of two, for the
    Hadamard transform; the scale is sqrt(N / tau) so that E[Pi^T Pi] = I_N.
  * tau defaults to 2 s (Section 6.2 uses tau = 2 s), capped at N;
    t_max defaults to 8 (Appendix F.1 finds 8 enough).
  * The draws come from SplitMix64(sketch_seed), apart from the schedule's
    generator: first the N signs (top bit 0: +1), then, for each block at its
    first use in step order, T as the sorted first tau entries of a partial
    Fisher-Yates shuffle of 0..N-1 (the schedule's subset draw).
  * LSQR stops early only when a rotation would divide by zero (rho = 0:
    the right-hand side or the Krylov space is exhausted exactly).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import scipy.linalg

from .rht import fht, next_pow2
from .schedule import SplitMix64, random_subset


def lsqr(M: np.ndarray, rhs: np.ndarray, iters: int) -> np.ndarray:
    """iters iterations of LSQR from z = 0 on min || M z - rhs ||."""
    z = np.zeros(M.shape[1])
    beta = float(np.linalg.norm(rhs))
    if beta == 0.0:
        return z
    u = rhs / beta
    v = M.T @ u
    alpha = float(np.linalg.norm(v))
    if alpha == 0.0:
        return z
    v = v / alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    for _ in range(iters):
        u = M @ v - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0.0:
            u = u / beta
        v = M.T @ u - beta * v
        alpha = float(np.linalg.norm(v))
        if alpha > 0.0:
            v = v / alpha
        rho = math.hypot(rhobar, beta)
        if rho == 0.0:
            break
        c, sn = rhobar / rho, beta / rho
        theta = sn * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = sn * phibar
        z = z + (phi / rho) * w
        w = v - (theta / rho) * w
    return z


def srht_sketch(AS: np.ndarray, d: np.ndarray, T: np.ndarray) -> np.ndarray:
    """A_S Pi^T = sqrt(N / tau) (H D [A_S, 0]^T)[T, :]^T (Lemma l:inner)."""
    s, n = AS.shape
    N = len(d)
    tau = len(T)
    X = np.zeros((N, s))
    X[:n] = AS.T
    HX = fht((np.asarray(d, dtype=np.float64) / math.sqrt(N))[:, None] * X)
    return math.sqrt(N / tau) * HX[np.asarray(T)].T


class LsqrProj:
    """The inexact projection of Algorithm 5 for one solve (holds the draws)."""

    def __init__(self, n: int, s: int, lam: float, sketch_seed: int, tau: Optional[int] = None,
                 iters: int = 8):
        self.n = n
        self.N = next_pow2(n)
        self.lam = float(lam)
        self.tau = min(2 * s if tau is None else int(tau), self.N)
        self.iters = int(iters)
        self.gen = SplitMix64(sketch_seed)
        self.d = np.array([1.0 if (self.gen.next() >> 63) == 0 else -1.0 for _ in range(self.N)])

    def factor(self, A: np.ndarray, S: np.ndarray) -> np.ndarray:
        """L, lower, with L L^T = A_hat A_hat^T + lambda I for a new block."""
        T = random_subset(self.gen, self.N, self.tau)
        Ah = srht_sketch(A[S, :], self.d, T)
        G = Ah @ Ah.T
        G[np.diag_indices_from(G)] += self.lam
        return np.linalg.cholesky(G)

    def direction(self, A: np.ndarray, S: np.ndarray, L: np.ndarray, r: np.ndarray) -> np.ndarray:
        AS = A[S, :]
        sb = len(S)
        M = scipy.linalg.solve_triangular(L, np.hstack([AS, math.sqrt(self.lam) * np.eye(sb)]), lower=True)
        rhs = scipy.linalg.solve_triangular(L, r, lower=True)
        return lsqr(M, rhs, self.iters)[:self.n]

    def factor_flops(self, sb: int, n: int) -> float:
        """Sketch (an FHT of the s padded rows), its Gram, Cholesky and the
        triangular inverse the GPU keeps."""
        return sb * self.N * math.log2(self.N) + sb * sb * self.tau + 2.0 * sb ** 3 / 3.0

    def step_flops(self, sb: int, n: int) -> float:
        """r and w (2 s n each), the momentum update (5 n), L^{-1} r, and per
        LSQR iteration one product with A_S and one with A_S^T (4 s n), their
        norms and two triangular products with L^{-1} (2 s^2 each)."""
        return 4.0 * sb * n + 5.0 * n + sb * sb + self.iters * (4.0 * sb * n + 2.0 * n + 4.0 * sb * sb)
