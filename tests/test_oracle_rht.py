"""Pins of the oracle's randomized Hadamard preprocessing (oracle/rht.py)
against what the paper and the mathematics fix:

* the Sylvester Hadamard matrix of the Appendix's definition, which
  scipy.linalg.hadamard also builds (a library routine, not the oracle's
  recursion): FHT(X) = H X and SymFHT(A) = H A H exactly on integer inputs;
* H^T H = n I (Section 2, after Definition d:rht);
* SymFHT(A) = FHT(FHT(A)^T) for symmetric A (Section 5.3);
* Theorem t:symFHT's cost bound n^2 (2.5 + log2 n), and the ~2.4e8 it gives
  at n = 4096 (Appendix, effect of RHT);
* the RHT keeps the solution of both systems (Q is orthogonal), with and
  without zero padding;
* the sign draw against the published SplitMix64 vectors.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import rht
from oracle import kpp as okpp
from oracle import schedule as osch
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [1, 2, 4, 8, 32, 128])
def test_fht_is_the_sylvester_hadamard_matrix(n):
    H = scipy.linalg.hadamard(n).astype(np.float64)
    assert np.array_equal(rht.fht(np.eye(n)), H)
    X = np.random.default_rng(n).integers(-9, 10, size=(n, 5)).astype(np.float64)
    assert np.array_equal(rht.fht(X), H @ X)
    assert np.array_equal(rht.fht(X[:, 0]), H @ X[:, 0])


def test_fht_halves_follow_the_definition():
    # H_2 = [[1, 1], [1, -1]]: the second half is a_1 - a_2, not a_2 - a_1
    assert np.array_equal(rht.fht(np.array([0.0, 1.0])), [1.0, -1.0])
    assert np.array_equal(rht.fht(np.array([0.0, 0.0, 1.0, 0.0])), [1.0, 1.0, -1.0, -1.0])


@pytest.mark.parametrize("n", [2, 16, 256])
def test_hadamard_is_scaled_orthogonal(n):
    H = rht.fht(np.eye(n))
    assert np.array_equal(H.T @ H, n * np.eye(n))
    assert np.array_equal(rht.fht(rht.fht(np.eye(n))), n * np.eye(n))


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 64, 128])
def test_symfht_is_H_A_H(n):
    rng = np.random.default_rng(100 + n)
    X = rng.integers(-5, 6, size=(n, n)).astype(np.float64)
    A = X + X.T
    H = scipy.linalg.hadamard(n).astype(np.float64)
    got = rht.symfht(A)
    assert np.array_equal(got, H @ A @ H)
    assert np.array_equal(got, rht.fht(rht.fht(A).T))   # the two-FHT form of Section 5.3
    assert np.array_equal(got, got.T)


@pytest.mark.parametrize("n", [4, 16, 256, 4096])
def test_symfht_operation_count(n):
    ops = rht.OpCount()
    rht.symfht(np.zeros((n, n)), ops)
    bound = n * n * (2.5 + math.log2(n))
    assert ops.adds <= bound
    # the naive two-FHT route costs 2 n^2 log2 n; for large n SymFHT saves close to half
    if n >= 256:
        assert ops.adds < 0.6 * 2 * n * n * math.log2(n)
    if n == 4096:
        assert 2.2e8 <= ops.adds <= 2.45e8      # "approximately 2.4e8 FLOPs"


def test_fht_operation_count():
    ops = rht.OpCount()
    rht.fht(np.zeros((64, 3)), ops)
    assert ops.adds == 64 * 3 * 6               # n d log2 n (Appendix, Algorithm 4 cost)


def test_rademacher_signs_follow_splitmix64_vectors():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "splitmix64_vectors.txt"))
            if ln.strip() and not ln.startswith("#")]
    seed = int(rows[0][0])
    outs = [int(r[2]) for r in rows if int(r[0]) == seed]
    want = [1.0 if o < 2 ** 63 else -1.0 for o in outs]
    assert rht.rademacher(seed, len(outs)).tolist() == want
    d = rht.rademacher(9, 4096)
    assert set(np.unique(d)) == {-1.0, 1.0}
    assert abs(d.mean()) < 0.06


@pytest.mark.parametrize("m,n", [(64, 16), (1000, 200), (37, 50)])
def test_rht_general_keeps_the_solution(m, n):
    sysm = synth.tiny_system("general", m, n, seed=m + n, cond=30.0)
    M = rht.next_pow2(m)
    d = rht.rademacher(5, M)
    At, bt = rht.rht_general(sysm.A, sysm.b, d)
    assert At.shape == (M, n) and bt.shape == (M,)
    # Q is orthogonal: residual norms and the Gram matrix are preserved
    x = np.random.default_rng(1).standard_normal(n)
    assert math.isclose(np.linalg.norm(At @ x - bt), np.linalg.norm(sysm.A @ x - sysm.b), rel_tol=1e-12)
    assert np.allclose(At.T @ At, sysm.A.T @ sysm.A, rtol=0, atol=1e-12 * np.abs(sysm.A.T @ sysm.A).max())
    # the same (minimum-norm) solution
    xs = np.linalg.lstsq(At, bt, rcond=None)[0]
    assert np.linalg.norm(xs - sysm.xstar) <= 1e-10 * np.linalg.norm(sysm.xstar)
    # against the explicit Q = H D on the padded system
    Q = scipy.linalg.hadamard(M) * (d / math.sqrt(M))[None, :]
    Ap = np.zeros((M, n))
    Ap[:m] = sysm.A
    assert np.allclose(At, Q @ Ap, rtol=0, atol=1e-13 * np.abs(Q @ Ap).max() * M)


@pytest.mark.parametrize("n", [64, 100])
def test_rht_psd_keeps_the_solution(n):
    sysm = synth.tiny_system("psd", n, n, seed=n, cond=50.0)
    N = rht.next_pow2(n)
    d = rht.rademacher(11, N)
    At, bt = rht.rht_psd(sysm.A, sysm.b, d)
    assert At.shape == (N, N)
    assert np.allclose(At, At.T, rtol=0, atol=1e-13 * np.abs(At).max())
    # same spectrum (plus N - n zero eigenvalues from the padding)
    ev = np.sort(np.linalg.eigvalsh(At))
    want = np.sort(np.concatenate([np.linalg.eigvalsh(sysm.A), np.zeros(N - n)]))
    assert np.allclose(ev, want, rtol=0, atol=1e-11 * want.max())
    # Q A Q^T (Q x*) = Q b, and x* comes back through D FHT(.)
    xbar = rht.rht_forward(sysm.xstar, d)
    assert np.linalg.norm(At @ xbar - bt) <= 1e-11 * np.linalg.norm(bt)
    assert np.allclose(rht.rht_back(xbar, d, n), sysm.xstar, rtol=0, atol=1e-12 * np.abs(sysm.xstar).max())
    # against the explicit Q = H D
    Q = scipy.linalg.hadamard(N) * (d / math.sqrt(N))[None, :]
    Ap = np.zeros((N, N))
    Ap[:n, :n] = sysm.A
    assert np.allclose(At, Q @ Ap @ Q.T, rtol=0, atol=1e-12 * np.abs(At).max())


def test_rht_rejects_bad_sizes():
    with pytest.raises(ValueError):
        rht.fht(np.zeros(6))
    with pytest.raises(ValueError):
        rht.rht_general(np.zeros((5, 2)), np.zeros(5), np.ones(4))
    with pytest.raises(ValueError):
        rht.rht_psd(np.zeros((3, 3)), np.zeros(3), np.ones(6))


@pytest.mark.parametrize("kind,m,n,s", [("general", 200, 40, 8), ("psd", 96, 96, 16)])
def test_solvers_with_rht_converge_to_the_planted_solution(kind, m, n, s):
    sysm = synth.tiny_system(kind, m, n, seed=7, cond=20.0)
    R = rht.next_pow2(m)
    d = rht.rademacher(3, R)
    p = okpp.Params(s=s, lam=1e-10, tol=1e-11, max_iters=20000)
    B0 = osch.online_rate(kind, R, R if kind == "psd" else n, s)
    schd = osch.make_schedule("online", R, s, 20000, 17, B0=B0)
    x0 = np.random.default_rng(2).standard_normal(n) if kind == "psd" else None
    res = rht.solve_rht(sysm.A, sysm.b, kind, p, schd, d, x0=x0)
    assert res.converged
    assert np.linalg.norm(sysm.A @ res.x - sysm.b) <= 1e-10 * np.linalg.norm(sysm.b)
    assert np.linalg.norm(res.x - sysm.xstar) <= 1e-7 * np.linalg.norm(sysm.xstar)
