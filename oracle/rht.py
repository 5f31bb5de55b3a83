"""Oracle randomized Hadamard preprocessing: FHT, SymFHT and the RHT of the
two solvers.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What is computed
  * H_n, the Hadamard matrix of the Appendix on SymFHT (Definition "Hadamard
    matrix"): H_1 = 1 and H_2k = [[H_k, H_k], [H_k, -H_k]] (Sylvester order).
  * FHT(X) = H_n X for an n x d matrix, by the recursion of Algorithm 4: each
    column splits into halves a_1, a_2 and the result stacks the transforms of
    a_1 + a_2 and of a_1 - a_2.  The printed recursion forms the second half
    from a_2 - a_1, which contradicts the definition of H_n; this follows the
    definition.
  * SymFHT(A) = H_n A H_n for symmetric A (Algorithm 3, Theorem t:symFHT),
    derived here from the Sylvester definition: with h = n/2, H = H_h and A
    split into h x h blocks [[A11, A12], [A12^T, A22]],
        H_n A H_n = [[P + Q + (R + R^T),  (P - Q) - (R - R^T)],
                     [(P - Q) + (R - R^T), P + Q - (R + R^T)]]
    where P = H A11 H and Q = H A22 H (the same transform, recursively, on the
    symmetric diagonal blocks) and R = H A12 H (two FHTs); H A12^T H = R^T.
    The lower-left block is the transpose of the upper-right one.  The
    additions this takes are counted; Theorem t:symFHT bounds them by
    n^2 (2.5 + log2 n).
  * The RHT Q = H D (Definition d:rht), D = diag(d_1, ..., d_N) / sqrt(N) with
    Rademacher signs d_i.  Kaczmarz++ (Algorithm 5) solves (Q A) x = Q b, the
    same x.  CD++ (Algorithm 2; Section 5.3, symmetric RHT) solves
    (Q A Q^T) xbar = Q b and returns x = Q^T xbar = D FHT(xbar).

Readings (each listed in the design notes)
  * Sizes that are not a power of two are zero-padded to the next one
    (Appendix, experiments on synthetic low-rank matrices): the rows of A and
    b for Kaczmarz++, rows and columns of A and the entries of b for CD++;
    the result is truncated back.  The padded system has the same solutions
    (restricted to the original unknowns) and the same residual norm, since Q
    is orthogonal and the padded rows are zero.
  * The solver then runs on the transformed padded system, so every default
    that depends on the shape (zeta, eta, the online sampling rate) uses the
    padded row count.
  * The signs come from SplitMix64 seeded with the RHT seed: d_i = +1 when
    the top bit of the i-th output is 0, -1 otherwise (the paper only asks
    for independent Rademacher signs).
  * An initial iterate x0 of CD++ enters as xbar0 = Q [x0; 0] (Algorithm 2
    starts from the transformed iterate; it does not spell the mapping out).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from .kpp import Params, Result, solve
from .schedule import Schedule, SplitMix64


class OpCount:
    """Counts scalar additions and subtractions done by fht / symfht."""

    def __init__(self):
        self.adds = 0


def next_pow2(k: int) -> int:
    p = 1
    while p < k:
        p *= 2
    return p


def fht(X: np.ndarray, ops: Optional[OpCount] = None) -> np.ndarray:
    """H_n X (Algorithm 4, with the halves combined as the definition of H_n
    says).  X is n x d (or a length-n vector); n must be a power of two."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if n & (n - 1) or n == 0:
        raise ValueError("FHT needs a power-of-two length, got %d" % n)
    if n == 1:
        return X.copy()
    half = n // 2
    a1, a2 = X[:half], X[half:]
    if ops is not None:
        ops.adds += 2 * a1.size
    top = fht(a1 + a2, ops)
    bottom = fht(a1 - a2, ops)
    return np.concatenate([top, bottom], axis=0)


def symfht(A: np.ndarray, ops: Optional[OpCount] = None) -> np.ndarray:
    """H_n A H_n for symmetric A (Theorem t:symFHT), from the block form of
    H_n = [[H, H], [H, -H]] given in the module docstring.  1 x 1: A itself."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if A.shape != (n, n) or n & (n - 1) or n == 0:
        raise ValueError("SymFHT needs a square power-of-two matrix")
    if n == 1:
        return A.copy()
    h = n // 2
    P = symfht(A[:h, :h], ops)              # H A11 H
    Q = symfht(A[h:, h:], ops)              # H A22 H
    R = fht(fht(A[:h, h:], ops).T, ops).T   # H A12 H (H is symmetric)
    diag_sum = P + Q
    diag_diff = P - Q
    cross_sym = R + R.T
    cross_skew = R - R.T
    out = np.empty((n, n))
    out[:h, :h] = diag_sum + cross_sym
    out[h:, h:] = diag_sum - cross_sym
    out[:h, h:] = diag_diff - cross_skew
    out[h:, :h] = out[:h, h:].T
    if ops is not None:
        ops.adds += 7 * h * h   # four block sums/differences, then three output blocks
    return out


def rademacher(seed: int, N: int) -> np.ndarray:
    """N signs +-1 from SplitMix64(seed): + when the output's top bit is 0."""
    g = SplitMix64(seed)
    return np.array([1.0 if (g.next() >> 63) == 0 else -1.0 for _ in range(N)])


def rht_general(A: np.ndarray, b: np.ndarray, d: np.ndarray):
    """Kaczmarz++ preprocessing (Algorithm 5): A <- FHT(D A), b <- FHT(D b),
    with A, b zero-padded to M = len(d) rows (a power of two >= m)."""
    m, n = A.shape
    M = len(d)
    if M != next_pow2(M) or M < m:
        raise ValueError("need len(d) a power of two >= m")
    Ap = np.zeros((M, n))
    Ap[:m] = A
    bp = np.zeros(M)
    bp[:m] = b
    scale = np.asarray(d, dtype=np.float64) / math.sqrt(M)
    return fht(scale[:, None] * Ap), fht(scale * bp)


def rht_psd(A: np.ndarray, b: np.ndarray, d: np.ndarray):
    """CD++ preprocessing (Algorithm 2): A <- SymFHT(D A D), b <- FHT(D b),
    with A zero-padded to N x N and b to N entries (N = len(d))."""
    n = A.shape[0]
    N = len(d)
    if N != next_pow2(N) or N < n:
        raise ValueError("need len(d) a power of two >= n")
    Ap = np.zeros((N, N))
    Ap[:n, :n] = A
    bp = np.zeros(N)
    bp[:n] = b
    D = np.asarray(d, dtype=np.float64) / math.sqrt(N)
    return symfht(D[:, None] * Ap * D[None, :]), fht(D * bp)


def rht_forward(x: np.ndarray, d: np.ndarray) -> np.ndarray:
    """xbar = Q [x; 0] = FHT(D [x; 0])."""
    N = len(d)
    xp = np.zeros(N)
    xp[:len(x)] = x
    return fht(np.asarray(d, dtype=np.float64) / math.sqrt(N) * xp)


def rht_back(xbar: np.ndarray, d: np.ndarray, n: int) -> np.ndarray:
    """x = Q^T xbar = D FHT(xbar), truncated to the first n entries (the
    return line of Algorithm 2)."""
    N = len(d)
    return (np.asarray(d, dtype=np.float64) / math.sqrt(N) * fht(xbar))[:n]


def solve_rht(A: np.ndarray, b: np.ndarray, kind: str, params: Params, schedule: Schedule,
              d: np.ndarray, x0: Optional[np.ndarray] = None, **kw) -> Result:
    """Algorithm 5 (kind "general") or Algorithm 2 (kind "psd") with the RHT
    lines: transform, run the solver on the transformed padded system (the
    schedule draws from its rows), map the iterate back.  Result.x is the
    solution of the original system."""
    if kind == "psd":
        At, bt = rht_psd(A, b, d)
        xb0 = None if x0 is None else rht_forward(x0, d)
        res = solve(At, bt, kind, params, schedule, x0=xb0, **kw)
        res.x = rht_back(res.x, d, A.shape[0])
        res.snapshots = {t: rht_back(v, d, A.shape[0]) for t, v in res.snapshots.items()}
        return res
    At, bt = rht_general(A, b, d)
    return solve(At, bt, kind, params, schedule, x0=x0, **kw)
