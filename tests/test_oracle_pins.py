"""Pins for the CPU oracle: each test fixes part of the oracle to something other
than the oracle itself -- a textbook routine, a closed form, an identity the
paper proves, an invariant, brute force on tiny inputs, or a published test
vector.  The mutation tests at the end plant plausible mistakes in the oracle
and check that these pins catch them.
"""
import itertools
import math
import os

import numpy as np
import pytest

import synth
from oracle import kpp
from oracle import schedule as sch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def tiny_general(m, n, seed, cond=10.0):
    return synth.tiny_system("general", m, n, seed, cond=cond)


# ---------------------------------------------------------------------------
# random numbers and the block schedule (Section 5.2; Algorithms 1, 2, 5)
# ---------------------------------------------------------------------------

def test_splitmix64_published_vectors():
    """Generator output equals the published SplitMix64 reference outputs."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "splitmix64_vectors.txt"))
            if ln.strip() and not ln.startswith("#")]
    by_seed = {}
    for seed, idx, out in rows:
        by_seed.setdefault(int(seed), []).append((int(idx), int(out)))
    for seed, pairs in by_seed.items():
        g = sch.SplitMix64(seed)
        outs = [g.next() for _ in range(max(i for i, _ in pairs) + 1)]
        for i, o in pairs:
            assert outs[i] == o


def test_bounded_and_subset_are_uniform():
    g = sch.SplitMix64(7)
    k = 7
    counts = np.bincount([g.bounded(k) for _ in range(70_000)], minlength=k)
    chi2 = float(((counts - 10_000.0) ** 2 / 10_000.0).sum())
    assert chi2 < 30.0  # 6 dof, p ~ 4e-5
    # all C(5, 2) = 10 subsets equally likely
    g = sch.SplitMix64(11)
    cnt = {}
    for _ in range(20_000):
        S = tuple(sch.random_subset(g, 5, 2).tolist())
        assert list(S) == sorted(set(S)) and len(S) == 2
        cnt[S] = cnt.get(S, 0) + 1
    assert len(cnt) == 10
    e = 2000.0
    chi2 = sum((c - e) ** 2 / e for c in cnt.values())
    assert chi2 < 35.0  # 9 dof


def test_partition_schedule_covers_rows_once():
    s_ = sch.make_schedule("fixed", 1000, 128, 50, seed=3, partition=True)
    assert len(s_.blocks) == 8
    allrows = np.concatenate(s_.blocks)
    assert np.array_equal(np.sort(allrows), np.arange(1000))
    assert [len(b) for b in s_.blocks] == [128] * 7 + [104]
    assert s_.step_block.min() >= 0 and s_.step_block.max() < 8


def test_online_schedule_rate_matches_bernoulli_expectation():
    """Number of new blocks after T steps has mean 1 + sum_{t>=1} min(1, B0/t)
    (Section 5.2), which is about B0 (1 + ln(T/B0))."""
    N, s, T = 400, 20, 3000
    B0 = sch.online_rate("psd", N, N, s)
    expect = 1.0 + sum(min(1.0, B0 / t) for t in range(1, T))
    var = sum(min(1.0, B0 / t) * (1 - min(1.0, B0 / t)) for t in range(1, T))
    got = [len(sch.make_schedule("online", N, s, T, seed=sd, B0=B0).blocks) for sd in range(20)]
    assert abs(np.mean(got) - expect) < 4.0 * math.sqrt(var / 20.0) + 1e-9
    assert abs(expect - B0 * (1 + math.log(T / B0))) < 0.1 * expect
    # the first ceil(B0) steps always draw new blocks
    s_ = sch.make_schedule("online", N, s, T, seed=1, B0=B0)
    assert s_.new_block[: int(math.floor(B0))].all()
    # reuse picks are uniform over the collection so far
    assert all(s_.step_block[t] < len(s_.blocks) for t in range(T))


def test_online_rate_values_from_section_5_2():
    """B0 of the new-block rule, evaluated by hand at the workloads' shapes.
    Section 5.2 and Algorithm 2: min(1, (1/t) (n/s) log n) for CD++;
    Algorithm 5: min(1, (1/t) (m/s) log m, (1/t) (n/s) log m) for Kaczmarz++,
    i.e. (min(m, n)/s) log m.  Natural log (the paper states no base).
      n = 4096, s = 128 (CD++):          32 ln 4096  = 266.1685...
      1000 x 200, s = 20:                10 ln 1000  = 69.0776...
      65536 x 2048, s = 256 (tall):       8 ln 65536 = 88.7228...
      2048 x 32768, s = 128 (wide):      16 ln 2048  = 121.9939...
    A swapped n and s, a base-2 log, m in place of min(m, n) or log n in
    place of log m each move at least one of these."""
    assert sch.online_rate("psd", 4096, 4096, 128) == pytest.approx(266.168517335019, rel=1e-12)
    assert sch.online_rate("general", 1000, 200, 20) == pytest.approx(69.07755278982137, rel=1e-12)
    assert sch.online_rate("general", 65536, 2048, 256) == pytest.approx(88.722839111673, rel=1e-12)
    assert sch.online_rate("general", 2048, 32768, 128) == pytest.approx(121.99390377855038, rel=1e-12)


def test_online_block_count_follows_section_5_2():
    """Section 5.2: the first B = (n/s) log n steps all draw new blocks, and T
    steps collect about B + sum_{t=B}^{T} B/t = B (1 + log(T/B)) blocks.  B is
    the hand value for 1000 x 200 with s = 20 (not taken from online_rate)."""
    B = 69.07755278982137
    T = 2000
    expect = 1.0 + sum(min(1.0, B / t) for t in range(1, T))   # 302.05 (Bernoulli means)
    assert abs(expect - B * (1.0 + math.log(T / B))) < 1.0
    var = sum(min(1.0, B / t) * (1.0 - min(1.0, B / t)) for t in range(1, T))
    rate = sch.online_rate("general", 1000, 200, 20)
    counts = []
    for sd in range(16):
        s_ = sch.make_schedule("online", 1000, 20, T, seed=sd, B0=rate)
        assert s_.new_block[:69].all()
        counts.append(len(s_.blocks))
    assert abs(np.mean(counts) - expect) < 4.0 * math.sqrt(var / 16.0)


def test_default_eta_values():
    """eta = s/(2n) (Section 5.4; Algorithm 2; Algorithm 5 for tall systems),
    evaluated by hand: 1000 x 200, s = 20 -> 0.05; n = 4096 CD++, s = 128 ->
    0.015625; 65536 x 2048, s = 256 -> 0.0625.  Wide Kaczmarz++ takes the rank
    min(m, n) in place of n (the variance parameter nu scales with the rank,
    Section 5.4): 2048 x 32768, s = 128 -> 0.03125 (the literal s/(2n) would be
    0.001953125)."""
    assert kpp.default_eta("general", 1000, 200, 20) == 0.05
    assert kpp.default_eta("psd", 4096, 4096, 128) == 0.015625
    assert kpp.default_eta("general", 65536, 2048, 256) == 0.0625
    assert kpp.default_eta("general", 2048, 32768, 128) == 0.03125


def test_refinement_with_half_exact_inner_solve():
    """Classical iterative refinement, closed form: an inner solve returning
    exactly half of the correction leaves r_k = 2^-k r_0, so the relative
    residual history is 1, 1/2, 1/4, ... and 1e-6 is reached after
    ceil(log2(1e6)) = 20 corrections; x_k = (1 - 2^-k) x*."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((12, 12)) + 6.0 * np.eye(12)
    xs = rng.standard_normal(12)
    b = A @ xs
    x, hist, ok = kpp.refine(A, b, "general", lambda r: 0.5 * np.linalg.solve(A, r), tol=1e-6,
                             max_rounds=20)
    assert ok and len(hist) == 21
    for k, h in enumerate(hist):
        assert h == pytest.approx(2.0 ** -k, rel=1e-9)
    assert relerr(x, (1.0 - 2.0 ** -20) * xs) < 1e-12
    # one round fewer does not reach the tolerance
    _, hist19, ok19 = kpp.refine(A, b, "general", lambda r: 0.5 * np.linalg.solve(A, r), tol=1e-6,
                                 max_rounds=19)
    assert not ok19 and hist19[-1] == pytest.approx(2.0 ** -19, rel=1e-9)


def test_refinement_with_perturbed_inner_solve_contracts():
    """An inner solve with a relative error e (here the exact solve of a
    perturbed matrix) contracts the residual by about e per round: reaching
    1e-10 from 1 takes about log(1e-10)/log(e) rounds (Section 2: inexact
    projections within a bound proportional to the error still converge)."""
    rng = np.random.default_rng(8)
    n = 30
    A = rng.standard_normal((n, n)) + 8.0 * np.eye(n)
    xs = rng.standard_normal(n)
    b = A @ xs
    E = rng.standard_normal((n, n))
    E *= 1e-2 * np.linalg.norm(A, 2) / np.linalg.norm(E, 2)
    Ap = A + E
    x, hist, ok = kpp.refine(A, b, "general", lambda r: np.linalg.solve(Ap, r), tol=1e-10, max_rounds=40)
    assert ok
    e = np.linalg.norm(np.eye(n) - A @ np.linalg.inv(Ap), 2)   # residual contraction bound
    assert e < 0.2
    assert len(hist) - 1 <= math.ceil(math.log(1e-10) / math.log(e)) + 1
    for k in range(1, len(hist)):
        assert hist[k] <= e * hist[k - 1] * (1 + 1e-6) + 1e-15
    assert relerr(x, xs) < 1e-8


# ---------------------------------------------------------------------------
# the regularized projection (eq. (bk), eq. (cd-update), Theorem 5.1 proof)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,s,lam", [(12, 7, 5, 0.3), (9, 20, 6, 1e-3), (30, 30, 30, 2.0)])
def test_projection_is_regularized_least_squares(m, n, s, lam):
    """x_t - w_t = argmin ||A_S x - b_S||^2 + lam ||x - x_t||^2 (eq. (bk)),
    checked with lstsq on the stacked system [A_S; sqrt(lam) I]."""
    rng = np.random.default_rng(m * 100 + n)
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    x = rng.standard_normal(n)
    S = np.sort(rng.choice(m, size=s, replace=False))
    w = kpp.regularized_projection(A, b, S, x, lam)
    M = np.vstack([A[S], math.sqrt(lam) * np.eye(n)])
    rhs = np.concatenate([b[S], math.sqrt(lam) * x])
    xnew = np.linalg.lstsq(M, rhs, rcond=None)[0]
    assert relerr(x - w, xnew) < 1e-11
    # push-through form: w = (A_S^T A_S + lam I)^{-1} A_S^T r
    r = A[S] @ x - b[S]
    w2 = np.linalg.solve(A[S].T @ A[S] + lam * np.eye(n), A[S].T @ r)
    assert relerr(w, w2) < 1e-10
    # dense LU of the regularized Gram
    w3 = A[S].T @ np.linalg.solve(A[S] @ A[S].T + lam * np.eye(s), r)
    assert relerr(w, w3) < 1e-11


def test_lambda_zero_projection_is_exact():
    """lam = 0 recovers the block Kaczmarz projection: A_S (x - w) = b_S."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((20, 12))
    b = rng.standard_normal(20)
    x = rng.standard_normal(12)
    S = np.array([1, 4, 5, 9, 13, 17])
    w = kpp.regularized_projection(A, b, S, x, 0.0)
    assert np.linalg.norm(A[S] @ (x - w) - b[S]) < 1e-12 * np.linalg.norm(b[S])
    # CD++ at lam = 0 zeroes the residual on the block: (A(x - w) - b)_S = 0
    P = synth.tiny_system("psd", 15, 15, seed=2).A
    bp = rng.standard_normal(15)
    xp = rng.standard_normal(15)
    Sp = np.array([0, 3, 7, 8, 14])
    wp = kpp.regularized_projection(P, bp, Sp, xp, 0.0, kind="psd")
    assert np.linalg.norm((P @ (xp - wp) - bp)[Sp]) < 1e-12 * np.linalg.norm(bp)
    assert np.count_nonzero(wp) == len(Sp)


def test_lambda_zero_rank_deficient_block_raises():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((6, 3))
    A[4] = A[1]  # duplicate row: singular Gram at lam = 0
    with pytest.raises(kpp.NotSPD):
        kpp.regularized_projection(A, np.ones(6), np.array([1, 2, 4, 5]), np.zeros(3), 0.0)


def test_cd_projection_is_kaczmarz_projection_on_a_factor():
    """eq. (implicit): Phi_S^T (Phi_S Phi_S^T + lam I)^{-1} (Phi_S z - b_S)
    = Phi^T I_S^T (A_SS + lam I)^{-1} (A_S x - b_S) with A = Phi Phi^T, z = Phi^T x."""
    rng = np.random.default_rng(9)
    Phi = rng.standard_normal((10, 10))
    A = Phi @ Phi.T
    b = rng.standard_normal(10)
    x = rng.standard_normal(10)
    S = np.array([0, 2, 3, 7])
    lam = 0.05
    wz = kpp.regularized_projection(Phi, b, S, Phi.T @ x, lam)
    wx = kpp.regularized_projection(A, b, S, x, lam, kind="psd")
    assert relerr(Phi.T @ wx, wz) < 1e-11


# ---------------------------------------------------------------------------
# momentum (eq. (momentum); Lemma 2.3 and its proof, eq. (para_rho))
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rho,eta", [(0.3, 0.2), (0.05, 0.01), (0.9, 0.5)])
def test_momentum_equals_three_sequence_form(rho, eta):
    """With beta = 1 - rho, gamma = 1 + eta/rho - eta, alpha = rho/(1+rho),
    v0 = y0 = x0, the (x, y, v) recursion reproduces x_{t+1} = x_t - w_t + eta m_{t+1}."""
    rng = np.random.default_rng(1)
    n = 6
    x0 = rng.standard_normal(n)
    ws = rng.standard_normal((25, n))
    beta, gamma, alpha = 1 - rho, 1 + eta / rho - eta, rho / (1 + rho)
    x, mom = x0.copy(), np.zeros(n)
    y, v = x0.copy(), x0.copy()
    for w in ws:
        x, mom = kpp.momentum_update(x, mom, w, rho, eta)
        xt = alpha * v + (1 - alpha) * y
        y_new = xt - w
        v = beta * v + (1 - beta) * xt - gamma * w
        y = y_new
        x3 = alpha * v + (1 - alpha) * y
        assert relerr(x, x3) < 1e-12


# ---------------------------------------------------------------------------
# the solver loop
# ---------------------------------------------------------------------------

def run(A, b, kind, s, T, mode="online", seed=5, **kw):
    m, n = A.shape
    N = n if kind == "psd" else m
    if mode == "online":
        schd = sch.make_schedule("online", N, s, T, seed, B0=sch.online_rate(kind, m, n, s))
    elif mode == "fixed":
        schd = sch.make_schedule("fixed", N, s, T, seed, num_blocks=kw.pop("num_blocks", 0),
                                 partition=kw.pop("partition", True))
    else:
        schd = sch.make_schedule("off", N, s, T, seed)
    snaps = kw.pop("snapshot_steps", ())
    x0 = kw.pop("x0", None)
    p = kpp.Params(s=s, max_iters=T, **kw)
    return kpp.solve(A, b, kind, p, schd, x0=x0, snapshot_steps=snaps), schd


def test_cdpp_is_implicit_kaczmarzpp_on_factor():
    """Theorem 5.1 proof: CD++ on A = Phi Phi^T and Kaczmarz++ on Phi z = b with
    the same block sequence satisfy z_t = Phi^T x_t at every step (the block
    residuals coincide, so the window sums and rho coincide too)."""
    sysm = synth.tiny_system("psd", 48, 48, seed=4, cond=30.0)
    A, b = sysm.A, sysm.b
    Phi = np.linalg.cholesky(A)
    T = 300
    steps = list(range(0, T + 1, 25))
    rx, _ = run(A, b, "psd", 6, T, seed=8, lam=1e-3, tol=0.0, snapshot_steps=steps)
    rz, _ = run(Phi, b, "general", 6, T, seed=8, lam=1e-3, tol=0.0, snapshot_steps=steps)
    for t in steps:
        assert relerr(Phi.T @ rx.snapshots[t], rz.snapshots[t]) < 1e-10, t
    assert [c["rho_next"] for c in rx.checkpoints] == pytest.approx(
        [c["rho_next"] for c in rz.checkpoints], rel=1e-9, abs=1e-12)


def test_planted_solution_is_a_fixed_point():
    sysm = tiny_general(40, 15, seed=3)
    res, _ = run(sysm.A, sysm.b, "general", 5, 200, x0=sysm.xstar, tol=0.0, lam=1e-2)
    assert relerr(res.x, sysm.xstar) < 1e-13


@pytest.mark.parametrize("case", ["over", "under", "psd"])
def test_converges_to_dense_normal_equations(case):
    """Consistent system: the iterate converges to the minimum-norm solution
    (Theorem 2.1), which a dense normal-equations solve gives on tiny inputs."""
    if case == "over":
        sysm = tiny_general(60, 20, seed=21)
        A, b = sysm.A, sysm.b
        ref = np.linalg.solve(A.T @ A, A.T @ b)
        kind, s = "general", 8
    elif case == "under":
        sysm = tiny_general(20, 60, seed=22)
        A, b = sysm.A, sysm.b
        ref = A.T @ np.linalg.solve(A @ A.T, b)
        kind, s = "general", 6
    else:
        sysm = synth.tiny_system("psd", 40, 40, seed=23)
        A, b = sysm.A, sysm.b
        ref = np.linalg.solve(A, b)
        kind, s = "psd", 8
    res, _ = run(A, b, kind, s, 20_000, lam=1e-8, tol=1e-12)
    assert res.converged
    assert relerr(res.x, ref) < 1e-10
    assert relerr(res.x, sysm.xstar) < 1e-10


@pytest.mark.parametrize("accel", [True, False])
@pytest.mark.parametrize("mode", ["online", "fixed", "off"])
def test_momentum_and_memo_do_not_move_the_fixed_point(accel, mode):
    sysm = tiny_general(50, 16, seed=31)
    kw = dict(num_blocks=30, partition=False) if mode == "fixed" else {}
    res, _ = run(sysm.A, sysm.b, "general", 6, 30_000, mode=mode, accel=accel,
                 memo=(mode != "off"), lam=1e-6, tol=1e-12, **kw)
    assert res.converged
    assert relerr(res.x, sysm.xstar) < 1e-10


def test_underdetermined_iterates_stay_in_row_space():
    """Every update lies in range(A_S^T) (eq. (bk)), so from x0 = 0 the
    iterates never leave the row space of A."""
    sysm = tiny_general(15, 50, seed=41)
    A = sysm.A
    Q, _ = np.linalg.qr(A.T)
    steps = list(range(0, 401, 20))
    res, _ = run(A, sysm.b, "general", 5, 400, tol=0.0, lam=1e-4, snapshot_steps=steps)
    for t in steps[1:]:
        xt = res.snapshots[t]
        assert np.linalg.norm(xt - Q @ (Q.T @ xt)) <= 1e-12 * np.linalg.norm(xt)


def test_block_residual_estimator_is_unbiased():
    """eq. (residual): averaged over all s-subsets, (m/s) ||A_S x - b_S||^2
    equals ||A x - b||^2."""
    rng = np.random.default_rng(3)
    m, n, s = 8, 5, 3
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    x = rng.standard_normal(n)
    tot = [(m / s) * float(np.sum(kpp.block_residual(A, b, np.array(S), x) ** 2))
           for S in itertools.combinations(range(m), s)]
    full = float(np.sum((A @ x - b) ** 2))
    assert abs(np.mean(tot) - full) < 1e-12 * full


def test_mu_nu_bounds_by_brute_force():
    """Lemma 2.2: 1 <= nu <= 1/mu for the uniform distribution over all subsets."""
    rng = np.random.default_rng(12)
    m, n, s, lam = 7, 4, 3, 0.1
    A = rng.standard_normal((m, n))
    Ps = []
    for S in itertools.combinations(range(m), s):
        S = np.array(S)
        L = kpp.cholesky_lower(kpp.regularized_gram(A, S, lam, "general"))
        # P = A_S^T G^{-1} A_S, one column of A_S at a time through the projection solve
        GinvAS = np.column_stack([kpp.projection_solve(L, A[S][:, j]) for j in range(n)])
        Ps.append(A[S].T @ GinvAS)
    Pbar = np.mean(Ps, axis=0)
    ev, U = np.linalg.eigh(Pbar)
    mu = ev[ev > 1e-12].min()
    Ph = U @ np.diag([e ** -0.5 if e > 1e-12 else 0.0 for e in ev]) @ U.T
    nu = np.linalg.eigvalsh(np.mean([(Ph @ P @ Ph) @ (Ph @ P @ Ph) for P in Ps], axis=0)).max()
    assert 1.0 - 1e-10 <= nu <= 1.0 / mu + 1e-10
    # and each P is a contraction (0 <= P <= I): regularized projections shrink
    for P in Ps:
        e = np.linalg.eigvalsh(0.5 * (P + P.T))
        assert e.min() > -1e-12 and e.max() < 1.0


# ---------------------------------------------------------------------------
# adaptive rho (Section 5.4, eq. (weighted))
# ---------------------------------------------------------------------------

def test_averaging_weights_closed_form():
    """a(j) = (j+1)^{ln(j+1)}: w_1 = 1/a(1) = 2^{-ln 2}, w_2 = a(1)/a(2) = 2^{ln 2}/3^{ln 3}."""
    assert kpp.averaging_weight(0) == 0.0
    assert kpp.averaging_weight(1) == pytest.approx(2.0 ** (-math.log(2.0)), rel=1e-14)
    assert kpp.averaging_weight(2) == pytest.approx(2.0 ** math.log(2.0) / 3.0 ** math.log(3.0),
                                                    rel=1e-14)
    assert kpp.averaging_weight(9) == pytest.approx(9.0 ** math.log(9.0) / 10.0 ** math.log(10.0),
                                                    rel=1e-13)
    # weights approach 1 (old estimates dominate eventually)
    assert 0.9 < kpp.averaging_weight(100) < 1.0


def test_rho_from_rate():
    assert kpp.rho_from_rate(0.25, 2) == pytest.approx(0.5)
    assert kpp.rho_from_rate(0.5 ** 8, 8) == pytest.approx(0.5)
    assert kpp.rho_from_rate(1.0, 4) == 0.0
    assert kpp.rho_from_rate(3.0, 4) == 0.0
    assert kpp.rho_from_rate(0.0, 4) == 1.0


def test_checkpoint_windows_and_flop_counter():
    """Window sums follow (t mod 2 zeta) < zeta (E0) vs the rest (E1); every new
    factor costs s^3/3 flops (Appendix F.2 accounting)."""
    sysm = synth.tiny_system("psd", 40, 40, seed=51)
    T = 160
    res, schd = run(sysm.A, sysm.b, "psd", 8, T, mode="fixed", partition=True, tol=0.0,
                    lam=1e-6)
    zeta = 5
    assert [c["t"] for c in res.checkpoints] == list(range(2 * zeta - 1, T, 2 * zeta))
    # recompute E0/E1 of the first window from the block residual pieces
    x = np.zeros(40)
    used = set(schd.step_block[:T].tolist())
    assert res.factorizations == len(used) == 5
    assert res.memo_hits == T - 5
    expect_fact = 5 * 8 ** 3 / 3.0
    per_step = T * (2.0 * 8 * 40 + 2.0 * 64 + 5.0 * 40)
    assert res.flops == pytest.approx(expect_fact + per_step)
    del x


# ---------------------------------------------------------------------------
# mutation tests: plausible mistakes planted in the oracle must fail a pin
# ---------------------------------------------------------------------------

def _bad_momentum_sign(x, mom, w, rho, eta):
    c = (1.0 - rho) / (1.0 + rho)
    mom_new = c * (mom + w)
    return x - w + eta * mom_new, mom_new


def _bad_momentum_c(x, mom, w, rho, eta):
    c = (1.0 + rho) / (1.0 - rho)
    mom_new = c * (mom - w)
    return x - w + eta * mom_new, mom_new


def _bad_gram_no_lambda(A, S, lam, kind, reverse=False):
    if kind == "psd":
        return A[np.ix_(S, S)].copy()
    return A[S] @ A[S].T


def _bad_direction_transposed(A, S, y, kind, reverse=False):
    if kind == "psd":
        w = np.zeros(A.shape[1])
        w[S[::-1]] = y
        return w
    return A[S, :].T @ y[::-1]


def _bad_rate_n_s_swapped(kind, m, n, s):
    if kind == "psd":
        return (float(s) / float(n)) * math.log(float(n))
    return (float(s) / float(min(m, n))) * math.log(float(m))


def _bad_rate_log2(kind, m, n, s):
    if kind == "psd":
        return (float(n) / float(s)) * math.log2(float(n))
    return (float(min(m, n)) / float(s)) * math.log2(float(m))


def _bad_rate_m_not_min(kind, m, n, s):
    if kind == "psd":
        return (float(n) / float(s)) * math.log(float(n))
    return (float(m) / float(s)) * math.log(float(m))


def _bad_eta_no_half(kind, m, n, s):
    return s / float(n if kind == "psd" else min(m, n))


def _bad_eta_max(kind, m, n, s):
    return s / (2.0 * (n if kind == "psd" else max(m, n)))


def _bad_refine_sign(A, b, kind, inner_solve, tol=1e-10, max_rounds=20, x0=None):
    A = np.asarray(A, dtype=np.float64)
    x = np.zeros(A.shape[1]) if x0 is None else np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    hist = []
    for _ in range(max_rounds):
        res = b - A @ x
        rel = float(np.linalg.norm(res)) / nb
        hist.append(rel)
        if rel <= tol:
            return x, hist, True
        x = x - inner_solve(res)
    hist.append(float(np.linalg.norm(b - A @ x)) / nb)
    return x, hist, hist[-1] <= tol


@pytest.mark.parametrize("mutant,target", [
    (_bad_momentum_sign, "momentum_update"),
    (_bad_momentum_c, "momentum_update"),
    (_bad_gram_no_lambda, "regularized_gram"),
    (_bad_direction_transposed, "direction"),
    (_bad_rate_n_s_swapped, "schedule.online_rate"),
    (_bad_rate_log2, "schedule.online_rate"),
    (_bad_rate_m_not_min, "schedule.online_rate"),
    (_bad_eta_no_half, "default_eta"),
    (_bad_eta_max, "default_eta"),
    (_bad_refine_sign, "refine"),
])
def test_planted_mistakes_are_caught(monkeypatch, mutant, target):
    if target.startswith("schedule."):
        monkeypatch.setattr(sch, target.split(".", 1)[1], mutant)
    else:
        monkeypatch.setattr(kpp, target, mutant)
    caught = []
    for fn in (lambda: test_momentum_equals_three_sequence_form(0.3, 0.2),
               lambda: test_projection_is_regularized_least_squares(12, 7, 5, 0.3),
               lambda: test_cdpp_is_implicit_kaczmarzpp_on_factor(),
               lambda: test_converges_to_dense_normal_equations("psd"),
               lambda: test_online_rate_values_from_section_5_2(),
               lambda: test_default_eta_values(),
               lambda: test_refinement_with_half_exact_inner_solve()):
        try:
            fn()
        except (AssertionError, ValueError, ArithmeticError, np.linalg.LinAlgError):
            caught.append(True)
    assert caught, f"no pin caught the planted mistake in {target}"
