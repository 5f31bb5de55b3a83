"""Pins of the oracle's sketch-preconditioned LSQR projection (oracle/lsqr.py)
against what the paper and the mathematics fix:

* LSQR's iterates against scipy.sparse.linalg.lsqr (a library routine) on
  the same preconditioned system;
* with enough iterations the inexact projection equals the exact regularized
  projection A_S^T (A_S A_S^T + lambda I)^{-1} r whatever the preconditioner
  (eq. (lsqr) has that minimum-norm solution);
* the sketch with T = all N rows is an orthogonal transform (A_hat A_hat^T =
  A_S A_S^T), and kappa of the preconditioned system falls towards 1 as tau
  grows (Lemma l:inner);
* Kaczmarz++ with this projection converges to the planted solution.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg as spl

import synth
from oracle import kpp as okpp
from oracle import lsqr as ol
from oracle import schedule as osch


def _block(seed, s=30, n=200):
    rng = np.random.default_rng(seed)
    AS = rng.standard_normal((s, n)) * np.geomspace(1.0, 100.0, n)[None, :]
    return AS, rng.standard_normal(s)


def _precond(AS, L, lam):
    s = AS.shape[0]
    return scipy.linalg.solve_triangular(L, np.hstack([AS, math.sqrt(lam) * np.eye(s)]), lower=True)


@pytest.mark.parametrize("iters", [1, 2, 5, 8])
def test_lsqr_matches_scipy(iters):
    AS, r = _block(1)
    lam = 1e-3
    P = ol.LsqrProj(AS.shape[1], AS.shape[0], lam, 7)
    L = P.factor(AS, np.arange(AS.shape[0]))
    M = _precond(AS, L, lam)
    rhs = scipy.linalg.solve_triangular(L, r, lower=True)
    z = ol.lsqr(M, rhs, iters)
    ref = spl.lsqr(M, rhs, damp=0.0, atol=0.0, btol=0.0, conlim=1e300, iter_lim=iters)[0]
    assert np.linalg.norm(z - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("lam", [1e-8, 1e-3, 1.0])
def test_enough_iterations_give_the_exact_projection(lam):
    AS, r = _block(2, s=24, n=150)
    s, n = AS.shape
    P = ol.LsqrProj(n, s, lam, 3, iters=60)
    L = P.factor(AS, np.arange(s))
    w = P.direction(AS, np.arange(s), L, r)
    exact = AS.T @ np.linalg.solve(AS @ AS.T + lam * np.eye(s), r)
    assert np.linalg.norm(w - exact) <= 1e-10 * np.linalg.norm(exact)
    # few iterations are only approximate, and improve with more
    P.iters = 2
    e2 = np.linalg.norm(P.direction(AS, np.arange(s), L, r) - exact)
    P.iters = 8
    e8 = np.linalg.norm(P.direction(AS, np.arange(s), L, r) - exact)
    assert e8 < e2


def test_full_sketch_is_orthogonal_and_kappa_falls_with_tau():
    AS, _ = _block(3, s=20, n=100)
    s, n = AS.shape
    N = 128
    d = np.where(np.random.default_rng(0).standard_normal(N) > 0, 1.0, -1.0)
    Ah = ol.srht_sketch(AS, d, np.arange(N))
    assert np.allclose(Ah @ Ah.T, AS @ AS.T, rtol=0, atol=1e-10 * np.abs(AS @ AS.T).max())
    lam = 1e-6
    kap = []
    for tau in (2 * s, 4 * s, 6 * s):
        P = ol.LsqrProj(n, s, lam, 11, tau=tau)
        sv = np.linalg.svd(_precond(AS, P.factor(AS, np.arange(s)), lam), compute_uv=False)
        kap.append(sv[0] / sv[-1])
    assert kap[0] > kap[1] > kap[2] and kap[2] < 2.0


def test_draws_are_reproducible():
    a, b = ol.LsqrProj(100, 10, 1e-3, 42), ol.LsqrProj(100, 10, 1e-3, 42)
    assert np.array_equal(a.d, b.d) and len(a.d) == 128 and a.tau == 20
    AS, _ = _block(4, s=10, n=100)
    assert np.array_equal(a.factor(AS, np.arange(10)), b.factor(AS, np.arange(10)))


def test_kaczmarz_with_lsqr_projection_converges():
    sysm = synth.tiny_system("general", 300, 60, seed=9, cond=20.0)
    m, n = sysm.A.shape
    s = 12
    T = 20000
    schd = osch.make_schedule("online", m, s, T, 5, B0=osch.online_rate("general", m, n, s))
    P = ol.LsqrProj(n, s, 1e-8, 17)
    res = okpp.solve(sysm.A, sysm.b, "general", okpp.Params(s=s, lam=1e-8, tol=1e-10, max_iters=T), schd, proj=P)
    assert res.converged
    assert np.linalg.norm(res.x - sysm.xstar) <= 1e-6 * np.linalg.norm(sysm.xstar)
