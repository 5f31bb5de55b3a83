"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on the
same seeded inputs and the same seeded block schedule.

Bar (FP64): iterates agree to 1e-10 relative after the same number of block
steps; factors of well-conditioned blocks agree to 1e-12 relative.  Floating
point never decides an integer here except the stop step, so iterate
comparisons use fixed step counts (tol = 0) and convergence is checked as a
property (true residual, distance to the planted solution).
"""
import math

import numpy as np
import pytest

import synth
from oracle import kpp as okpp
from oracle import schedule as osch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2501_11673_amd as kpp

    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    ctx = kpp.kpp_context_create(0, torch.cuda.current_stream(dev).cuda_stream)
    yield kpp, torch, dev, ctx
    kpp.kpp_context_destroy(ctx)


def relerr(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / (nb if nb > 0 else 1.0)


MODES = {"online": 1, "fixed": 2, "off": 0}


def gpu_solve(env, A, b, kind, s, *, lam, T, tol=0.0, mode="online", seed=7, num_blocks=0,
              partition=True, accel=True, eta=None, x0=None, adaptive=True, keep_memo=False,
              engine=0, team_groups=0):
    kpp, torch, dev, ctx = env
    m, n = A.shape
    ck = kpp.KPP_CD_PSD if kind == "psd" else kpp.KPP_KACZMARZ
    p = kpp.kpp_params_default(ck)
    p.block_size = s
    p.lambda_ = lam
    p.tol = tol
    p.max_iters = T
    p.seed = seed
    p.memo = MODES[mode]
    p.num_blocks = num_blocks
    p.fixed_partition = 1 if partition else 0
    p.accel = 1 if accel else 0
    p.adaptive_rho = 1 if adaptive else 0
    p.keep_memo = 1 if keep_memo else 0
    p.engine = engine
    p.team_groups = team_groups
    if eta is not None:
        p.eta = eta
    Ad = A if hasattr(A, "data_ptr") else torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    bd = b if hasattr(b, "data_ptr") else torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    if x0 is None:
        xd = torch.zeros(n, dtype=torch.float64, device=dev)
    else:
        xd = torch.from_numpy(np.array(x0, dtype=np.float64)).to(dev)
    h = kpp.kpp_system_create(ctx, ck, m, n, Ad.data_ptr(), n, bd.data_ptr())
    try:
        st, res = kpp.kpp_solve(h, p, xd.data_ptr())
    finally:
        kpp.kpp_system_destroy(h)
    return xd.cpu().numpy(), st, res


def oracle_solve(A, b, kind, s, *, lam, T, tol=0.0, mode="online", seed=7, num_blocks=0,
                 partition=True, accel=True, eta=None, x0=None, adaptive=True, snapshot_steps=(),
                 reverse_sums=False):
    m, n = A.shape
    N = n if kind == "psd" else m
    schd = osch.make_schedule(mode, N, s, T, seed, B0=osch.online_rate(kind, m, n, s),
                              num_blocks=num_blocks, partition=partition)
    p = okpp.Params(s=s, lam=lam, tol=tol, max_iters=T, accel=accel, eta=eta,
                    adaptive_rho=adaptive, memo=(mode != "off"), reverse_sums=reverse_sums)
    return okpp.solve(A, b, kind, p, schd, x0=x0, snapshot_steps=snapshot_steps)


def parity_bound(A, b, kind, s, ref, **kw):
    """max(1e-10, 10 nf): nf is the FP64 noise floor of the trajectory, the
    oracle's distance to itself with every sum taken in the opposite order.
    Ill-conditioned block Grams (kappa ~ 1e9) amplify rounding past 1e-10 for
    any two valid FP64 implementations; well-conditioned cases keep 1e-10."""
    alt = oracle_solve(A, b, kind, s, reverse_sums=True, **kw)
    nf = relerr(alt.x, ref.x)
    rho_nf = abs(alt.rho_final - ref.rho_final)
    return max(1e-10, 10.0 * nf), nf, max(1e-9 * abs(ref.rho_final), 1e-12, 10.0 * rho_nf)


# ---------------------------------------------------------------------------
# memo-miss path: Gram + Cholesky
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,m,n,s,lam", [
    ("general", 300, 150, 20, 1e-3),
    ("general", 700, 300, 37, 1e-2),     # ragged tiles
    ("general", 1200, 400, 256, 1e-1),   # LDS-panel factor and inverse (129..256 rows)
    ("general", 1500, 400, 384, 1e-1),   # factor in global memory (257..512 rows)
    ("psd", 1100, 1100, 512, 1e-8),      # the largest block size the library takes
    ("general", 400, 3000, 100, 1e-2),   # wide: Gram split over 47 column chunks, ragged tile
    ("psd", 500, 500, 128, 1e-8),
    ("psd", 300, 300, 1, 1e-8),
])
def test_block_factor_matches_oracle(env, kind, m, n, s, lam):
    kpp, torch, dev, ctx = env
    sysm = synth.tiny_system("psd", n, n, seed=3, cond=20.0) if kind == "psd" else \
        synth.tiny_system("general", m, n, seed=3, cond=20.0)
    A, b = sysm.A, sysm.b
    N = n if kind == "psd" else m
    g = osch.SplitMix64(99)
    blocks = [osch.random_subset(g, N, s) for _ in range(5)]
    blocks.append(osch.random_subset(g, N, max(1, s - 3)))  # a short block
    rows = []
    for blk in blocks:
        rows += blk.tolist() + [0] * (s - len(blk))
    lens = [len(blk) for blk in blocks]
    Ad = torch.from_numpy(A).to(dev)
    bd = torch.from_numpy(b).to(dev)
    ck = kpp.KPP_CD_PSD if kind == "psd" else kpp.KPP_KACZMARZ
    h = kpp.kpp_system_create(ctx, ck, A.shape[0], n, Ad.data_ptr(), n, bd.data_ptr())
    L = torch.full((len(blocks), s, s), float("nan"), dtype=torch.float64, device=dev)
    try:
        kpp.kpp_block_factor(h, s, lam, rows, lens, L.data_ptr())
    finally:
        kpp.kpp_system_destroy(h)
    Lh = L.cpu().numpy()
    for q, blk in enumerate(blocks):
        ref = okpp.cholesky_lower(okpp.regularized_gram(A, blk, lam, kind))
        sb = len(blk)
        got = Lh[q].T[:sb, :sb]  # column-major slot -> row-major view
        assert relerr(got, ref) < 1e-12
        full = Lh[q].T
        assert np.all(full[np.triu_indices(s, 1)] == 0.0)
        assert np.all(full[sb:, :] == 0.0) and np.all(full[:, sb:] == 0.0)


def test_block_factor_reports_breakdown(env):
    """A block whose regularized Gram has a negative pivot has no Cholesky factor."""
    kpp, torch, dev, ctx = env
    A = np.diag([1.0, 2.0, -3.0, 4.0, 5.0, 6.0])
    b = np.ones(6)
    Ad = torch.from_numpy(A).to(dev)
    bd = torch.from_numpy(b).to(dev)
    h = kpp.kpp_system_create(ctx, kpp.KPP_CD_PSD, 6, 6, Ad.data_ptr(), 6, bd.data_ptr())
    L = torch.zeros((2, 4, 4), dtype=torch.float64, device=dev)
    try:
        kpp.kpp_block_factor(h, 4, 0.0, [0, 1, 3, 4, 0, 1, 2, 3], [4, 4], L.data_ptr())
        assert False, "expected KPP_ERR_NOT_SPD"
    except kpp.KppError as e:
        assert e.status == kpp.KPP_ERR_NOT_SPD
    finally:
        kpp.kpp_system_destroy(h)


def test_residual_norm(env):
    kpp, torch, dev, ctx = env
    rng = np.random.default_rng(4)
    A = rng.standard_normal((333, 77))
    b = rng.standard_normal(333)
    x = rng.standard_normal(77)
    Ad, bd, xd = (torch.from_numpy(v).to(dev) for v in (A, b, x))
    h = kpp.kpp_system_create(ctx, 0, 333, 77, Ad.data_ptr(), 77, bd.data_ptr())
    try:
        got = kpp.kpp_residual_norm(h, xd.data_ptr())
    finally:
        kpp.kpp_system_destroy(h)
    assert got == pytest.approx(np.linalg.norm(A @ x - b), rel=1e-13)


# ---------------------------------------------------------------------------
# iterate parity at fixed step counts
# ---------------------------------------------------------------------------

ITER_CASES = [
    # name, kind, builder, s, lam, mode, T, extra
    ("c1", "general", lambda: synth.config("c1"), 20, 1e-3, "online", 600, {}),
    ("c2_small", "psd", lambda: synth.config("c2_small"), 128, 1e-8, "online", 320, {}),
    ("c2_small_partition", "psd", lambda: synth.config("c2_small"), 128, 1e-8, "fixed", 160, {}),
    ("c3_small", "general", lambda: synth.config("c3_small"), 256, 1e-8, "fixed", 200, {}),
    ("c4_small", "general", lambda: synth.config("c4_small"), 64, 1e-4, "online", 200, {}),
    # Kaczmarz++ blocks of 128+ rows on 4+ workgroups split y across the team
    ("c4_small_s128", "general", lambda: synth.config("c4_small"), 128, 1e-4, "online", 120, {}),
    ("tiny_over_s1", "general", lambda: synth.tiny_system("general", 50, 9, seed=5), 1, 1e-6, "online", 300, {}),
    ("tiny_psd_sN", "psd", lambda: synth.tiny_system("psd", 24, 24, seed=6), 24, 1e-6, "online", 40, {}),
    ("tiny_under_off", "general", lambda: synth.tiny_system("general", 30, 90, seed=8), 7, 1e-5, "off", 150, {}),
    ("tiny_fixed_subsets", "general", lambda: synth.tiny_system("general", 80, 30, seed=9), 9, 1e-5, "fixed", 200,
     dict(num_blocks=11, partition=False)),
    ("tiny_noaccel", "psd", lambda: synth.tiny_system("psd", 60, 60, seed=10, cond=100.0), 8, 1e-8, "online", 300,
     dict(accel=False)),
    ("tiny_eta_rho_fixed", "general", lambda: synth.tiny_system("general", 90, 40, seed=11), 10, 1e-6, "online", 300,
     dict(eta=0.1, adaptive=False)),
]


@pytest.mark.parametrize("engine", [1, 2], ids=["launch", "fused"])
@pytest.mark.parametrize("case", ITER_CASES, ids=[c[0] for c in ITER_CASES])
def test_iterates_match_oracle(env, case, engine):
    name, kind, build, s, lam, mode, T, extra = case
    sysm = build()
    A, b = sysm.A, sysm.b
    print(f"[parity] {name} engine={engine} shape={A.shape} s={s} T={T}", flush=True)
    for Tk in (T // 2, T):
        x, st, res = gpu_solve(env, A, b, kind, s, lam=lam, T=Tk, mode=mode, seed=31, engine=engine, **extra)
        assert res.engine_used == engine
        ref = oracle_solve(A, b, kind, s, lam=lam, T=Tk, mode=mode, seed=31, **extra)
        bound, nf, rho_bound = parity_bound(A, b, kind, s, ref, lam=lam, T=Tk, mode=mode, seed=31, **extra)
        err = relerr(x, ref.x)
        print(f"[parity] {name} T={Tk}: |x_gpu - x_orc|/|x_orc| = {err:.3e}, noise floor {nf:.3e}", flush=True)
        assert err <= bound, f"{name} after {Tk} steps: relative difference {err:.3e} (noise floor {nf:.3e})"
        assert res.iters == Tk
        assert res.memo_misses == ref.factorizations
        assert abs(res.rho_final - ref.rho_final) <= rho_bound


@pytest.mark.parametrize("name,kind,m,n,s,lam,mode,T", [
    # 257..512 rows: global-memory factor kernels, the projection's rows over
    # 16-row workgroups; a 7-block partition whose last block has 200 rows
    ("general_s300", "general", 2000, 500, 300, 1e-6, "fixed", 60),
    ("psd_s384_online", "psd", 900, 900, 384, 1e-8, "online", 40),
])
def test_large_blocks_match_oracle(env, name, kind, m, n, s, lam, mode, T):
    """Blocks above 256 rows run on the launch-per-phase engine only."""
    sysm = synth.tiny_system(kind, m, n, seed=s, cond=30.0)
    A, b = sysm.A, sysm.b
    print(f"[parity] {name} shape={A.shape} s={s} T={T}", flush=True)
    x, st, res = gpu_solve(env, A, b, kind, s, lam=lam, T=T, mode=mode, seed=19, engine=1)
    assert res.engine_used == 1 and res.iters == T
    ref = oracle_solve(A, b, kind, s, lam=lam, T=T, mode=mode, seed=19)
    bound, nf, rho_bound = parity_bound(A, b, kind, s, ref, lam=lam, T=T, mode=mode, seed=19)
    err = relerr(x, ref.x)
    print(f"[parity] {name}: {err:.3e} (noise floor {nf:.3e})", flush=True)
    assert err <= bound
    assert res.memo_misses == ref.factorizations
    assert abs(res.rho_final - ref.rho_final) <= rho_bound
    with pytest.raises(Exception):   # the fused engine takes at most 256 rows
        gpu_solve(env, A, b, kind, s, lam=lam, T=T, mode=mode, seed=19, engine=2)


@pytest.mark.parametrize("kind,m,n", [("general", 1100, 300), ("psd", 700, 700)])
@pytest.mark.parametrize("s", [129, 176, 255])
def test_panel_factor_block_sizes_match_oracle(env, kind, m, n, s):
    """Blocks of 129..256 rows (the LDS-panel Cholesky and the matrix-core
    inverse), at sizes that are not multiples of the 32-row panels or the
    16-row tiles, with a ragged last block of the partition, on the fused
    engine."""
    sysm = synth.tiny_system(kind, m, n, seed=s + 7, cond=30.0)
    A, b = sysm.A, sysm.b
    lam, T = 1e-6, 60
    print(f"[parity] panel factor kind={kind} shape={A.shape} s={s} T={T}", flush=True)
    x, st, res = gpu_solve(env, A, b, kind, s, lam=lam, T=T, mode="fixed", seed=23)
    assert res.iters == T
    ref = oracle_solve(A, b, kind, s, lam=lam, T=T, mode="fixed", seed=23)
    bound, nf, rho_bound = parity_bound(A, b, kind, s, ref, lam=lam, T=T, mode="fixed", seed=23)
    err = relerr(x, ref.x)
    print(f"[parity] panel factor s={s}: {err:.3e} (noise floor {nf:.3e})", flush=True)
    assert err <= bound
    assert res.memo_misses == ref.factorizations
    assert abs(res.rho_final - ref.rho_final) <= rho_bound


def test_converges_like_oracle_c1(env):
    sysm = synth.config("c1")
    A, b = sysm.A, sysm.b
    x, st, res = gpu_solve(env, A, b, "general", 20, lam=1e-3, T=20000, tol=1e-10, seed=101)
    ref = oracle_solve(A, b, "general", 20, lam=1e-3, T=20000, tol=1e-10, seed=101)
    assert st == 0 and res.converged == 1 and ref.converged
    assert res.true_rel_res <= 1e-10
    assert np.linalg.norm(A @ x - b) <= 1.01e-10 * np.linalg.norm(b)
    assert relerr(x, sysm.xstar) < 1e-8
    assert abs(res.iters - ref.iters) <= 2 * 50 * 2  # same or a neighbouring checkpoint


@pytest.mark.parametrize("engine", [1, 2])
def test_bitwise_repeatable(env, engine):
    sysm = synth.config("c2_small")
    x1, _, _ = gpu_solve(env, sysm.A, sysm.b, "psd", 128, lam=1e-8, T=200, seed=3, engine=engine)
    x2, _, _ = gpu_solve(env, sysm.A, sysm.b, "psd", 128, lam=1e-8, T=200, seed=3, engine=engine)
    assert np.array_equal(x1, x2)


@pytest.mark.parametrize("groups", [1, 3, 8, 64])
def test_fused_team_sizes_agree_with_oracle(env, groups):
    """The fused engine's result does not depend on how many workgroups share
    a step beyond rounding (columns per workgroup change the summation order)."""
    sysm = synth.tiny_system("general", 400, 700, seed=12, cond=30.0)
    A, b = sysm.A, sysm.b
    x, st, res = gpu_solve(env, A, b, "general", 32, lam=1e-6, T=150, seed=5, engine=2, team_groups=groups)
    ref = oracle_solve(A, b, "general", 32, lam=1e-6, T=150, seed=5)
    assert relerr(x, ref.x) <= 1e-10


@pytest.mark.parametrize("n", [150, 250, 700, 4000])
def test_split_y_team_sizes_agree_with_oracle(env, n):
    """Kaczmarz++ with 130-row blocks (one column per lane, so ceil(n/64)
    workgroups: 3, 4, 11, 63): y is formed whole in every workgroup (3) or by
    the workgroup owning each row and all-gathered (4+).  The partition of 1000
    rows ends in a ragged 90-row block, and ceil(s/G) rows per workgroup do not
    divide the block."""
    sysm = synth.tiny_system("general", 1000, n, seed=15, cond=30.0)
    A, b = sysm.A, sysm.b
    x, st, res = gpu_solve(env, A, b, "general", 130, lam=1e-6, T=120, mode="fixed", seed=5, engine=2)
    ref = oracle_solve(A, b, "general", 130, lam=1e-6, T=120, mode="fixed", seed=5)
    assert res.iters == 120
    assert relerr(x, ref.x) <= 1e-10


@pytest.mark.parametrize("engine", [1, 2], ids=["launch", "fused"])
def test_explicit_schedule_matches_oracle(env, engine):
    """A caller-given schedule (overlapping blocks, one of them ragged, steps
    drawn by numpy) gives the oracle's iterates on the same schedule; a step
    budget past the schedule's end stops at its end."""
    kpp, torch, dev, ctx = env
    sysm = synth.tiny_system("general", 300, 120, seed=21, cond=20.0)
    A, b = sysm.A, sysm.b
    m, n = A.shape
    s, T = 16, 150
    rng = np.random.default_rng(4)
    blocks = [np.sort(rng.choice(m, size=s, replace=False)) for _ in range(6)]
    blocks.append(np.sort(rng.choice(m, size=10, replace=False)))
    steps = rng.integers(0, len(blocks), size=T)
    table = [list(map(int, blk)) + [-1] * (s - len(blk)) for blk in blocks]
    p = kpp.kpp_params_default(kpp.KPP_KACZMARZ)
    p.block_size = s
    p.lambda_ = 1e-4
    p.tol = 0.0
    p.max_iters = T + 40
    p.engine = engine
    keep = kpp.kpp_set_schedule(p, steps.tolist(), table)
    Ad = torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    bd = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    xd = torch.zeros(n, dtype=torch.float64, device=dev)
    h = kpp.kpp_system_create(ctx, kpp.KPP_KACZMARZ, m, n, Ad.data_ptr(), n, bd.data_ptr())
    try:
        st, res = kpp.kpp_solve(h, p, xd.data_ptr())
    finally:
        kpp.kpp_system_destroy(h)
    del keep
    x = xd.cpu().numpy()
    first = np.zeros(T, dtype=bool)
    seen = set()
    for t, blk_id in enumerate(steps.tolist()):
        first[t] = blk_id not in seen
        seen.add(blk_id)
    schd = osch.Schedule(blocks=[blk.astype(np.int64) for blk in blocks], step_block=steps.astype(np.int64),
                         new_block=first)
    ref = okpp.solve(A, b, "general", okpp.Params(s=s, lam=1e-4, tol=0.0, max_iters=T), schd)
    assert st == kpp.KPP_NOT_CONVERGED and res.iters == T
    assert res.memo_misses == len(set(steps.tolist())) == ref.factorizations
    assert relerr(x, ref.x) <= 1e-10


def _resume_params(kpp, kind, s, lam, steps, resume):
    p = kpp.kpp_params_default(kind)
    p.block_size = s
    p.lambda_ = lam
    p.tol = 0.0
    p.seed = 77
    p.max_iters = steps
    p.memo = MODES["online"]
    p.num_blocks = 0
    p.fixed_partition = 1
    p.accel = 1
    p.adaptive_rho = 1
    p.resume = 1 if resume else 0
    return p


@pytest.mark.parametrize("via", ["export_import", "same_system"])
def test_resumed_cdpp_solve_equals_uninterrupted(env, via):
    """A CD++ solve cut after 170 steps (mid-window) and continued for 230 --
    on the same system, or on a fresh one through kpp_state_export/import --
    gives the iterate of one 400-step solve bit for bit."""
    kpp, torch, dev, ctx = env
    sysm = synth.config("c2_small")
    A = torch.from_numpy(np.ascontiguousarray(sysm.A)).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(sysm.b)).to(dev)
    n = A.shape[0]
    ck = kpp.KPP_CD_PSD

    def new_system():
        return kpp.kpp_system_create(ctx, ck, n, n, A.data_ptr(), n, b.data_ptr())

    h = new_system()
    x_full = torch.zeros(n, dtype=torch.float64, device=dev)
    st, full = kpp.kpp_solve(h, _resume_params(kpp, ck, 128, 1e-8, 400, False), x_full.data_ptr())
    kpp.kpp_system_destroy(h)
    h = new_system()
    h2 = None
    try:
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        kpp.kpp_solve(h, _resume_params(kpp, ck, 128, 1e-8, 170, False), x.data_ptr())
        target = h
        if via == "export_import":
            state = kpp.kpp_state_export(h)
            h2 = new_system()
            kpp.kpp_state_import(h2, state)
            target = h2
        st, part = kpp.kpp_solve(target, _resume_params(kpp, ck, 128, 1e-8, 230, True), x.data_ptr())
        assert part.iters == 230 and full.iters == 400
        assert torch.equal(x, x_full), float(torch.max(torch.abs(x - x_full)))
        assert part.rho_final == full.rho_final
        with pytest.raises(kpp.KppError):   # the saved state is of a solve with blocks of 128
            kpp.kpp_solve(target, _resume_params(kpp, ck, 64, 1e-8, 10, True), x.data_ptr())
    finally:
        kpp.kpp_system_destroy(h)
        if h2 is not None:
            kpp.kpp_system_destroy(h2)


def test_resumed_kaczmarz_solve_matches_oracle(env):
    """Kaczmarz++ (1000 x 200, blocks of 20): 250 steps, export, import into a
    fresh system, 350 more; the oracle runs 600 steps in one go (the resumed
    run forms its Grams again in other batches: equal up to rounding)."""
    kpp, torch, dev, ctx = env
    sysm = synth.config("c1")
    m, n = sysm.A.shape
    A = torch.from_numpy(np.ascontiguousarray(sysm.A)).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(sysm.b)).to(dev)
    ck = kpp.KPP_KACZMARZ
    h = kpp.kpp_system_create(ctx, ck, m, n, A.data_ptr(), n, b.data_ptr())
    h2 = kpp.kpp_system_create(ctx, ck, m, n, A.data_ptr(), n, b.data_ptr())
    try:
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        kpp.kpp_solve(h, _resume_params(kpp, ck, 20, 1e-3, 250, False), x.data_ptr())
        kpp.kpp_state_import(h2, kpp.kpp_state_export(h))
        st, res = kpp.kpp_solve(h2, _resume_params(kpp, ck, 20, 1e-3, 350, True), x.data_ptr())
    finally:
        kpp.kpp_system_destroy(h)
        kpp.kpp_system_destroy(h2)
    kw = dict(lam=1e-3, T=600, seed=77)
    ref = oracle_solve(sysm.A, sysm.b, "general", 20, **kw)
    bound, nf, _ = parity_bound(sysm.A, sysm.b, "general", 20, ref, **kw)
    assert res.iters == 350
    assert relerr(x.cpu().numpy(), ref.x) <= bound, (relerr(x.cpu().numpy(), ref.x), nf)


# ---------------------------------------------------------------------------
# edge cases and error paths
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("engine", [1, 2])
def test_zero_steps_and_zero_rhs(env, engine):
    sysm = synth.tiny_system("general", 40, 10, seed=1)
    x0 = np.arange(10, dtype=np.float64)
    x, st, res = gpu_solve(env, sysm.A, sysm.b, "general", 4, lam=1e-6, T=0, x0=x0, engine=engine)
    assert st == 1 and res.iters == 0 and np.array_equal(x, x0)
    x, st, res = gpu_solve(env, sysm.A, np.zeros(40), "general", 4, lam=1e-6, T=100, tol=1e-10, engine=engine)
    assert st == 0 and res.converged == 1 and np.all(x == 0.0)


@pytest.mark.parametrize("engine", [1, 2])
def test_one_by_one_system(env, engine):
    """n = s = 1, lambda = 0: without momentum one step lands on x = b/a exactly
    and the first checkpoint stops; with momentum (eta = 1/2) it matches the oracle."""
    A = np.array([[4.0]])
    b = np.array([2.0])
    x, st, res = gpu_solve(env, A, b, "psd", 1, lam=0.0, T=10, tol=1e-12, accel=False, engine=engine)
    assert st == 0 and x[0] == 0.5 and res.iters == 2
    x, st, res = gpu_solve(env, A, b, "psd", 1, lam=0.0, T=10, engine=engine)
    ref = oracle_solve(A, b, "psd", 1, lam=0.0, T=10)
    assert abs(x[0] - ref.x[0]) <= 1e-15 * abs(ref.x[0])


def test_errors(env):
    kpp, torch, dev, ctx = env
    sysm = synth.tiny_system("general", 20, 6, seed=2)
    A = sysm.A.copy()
    A[3, 2] = math.nan
    with pytest.raises(kpp.KppError) as e:
        gpu_solve(env, A, sysm.b, "general", 4, lam=1e-6, T=10)
    assert e.value.status == kpp.KPP_ERR_NONFINITE
    Aind = np.diag(np.linspace(1.0, 2.0, 12))
    Aind[7, 7] = -1.0  # indefinite "PSD" input
    with pytest.raises(kpp.KppError) as e:
        gpu_solve(env, Aind, np.ones(12), "psd", 12, lam=0.0, T=10, mode="fixed")
    assert e.value.status == kpp.KPP_ERR_NOT_SPD
    with pytest.raises(kpp.KppError) as e:
        gpu_solve(env, sysm.A, sysm.b, "general", 21, lam=1e-6, T=10)
    assert e.value.status == kpp.KPP_ERR_INVALID_ARG
    with pytest.raises(kpp.KppError) as e:
        gpu_solve(env, np.ones((5, 6)), np.ones(5), "psd", 2, lam=1e-6, T=10)
    assert e.value.status == kpp.KPP_ERR_SHAPE


# ---------------------------------------------------------------------------
# mixed precision: FP32 inner block iteration, FP64 refinement
# ---------------------------------------------------------------------------

MIXED_CASES = [
    # name, kind, builder, s, lam, mode, team_groups (0: default team)
    ("c1", "general", lambda: synth.config("c1"), 20, 1e-3, "online", 0),
    ("c2_small", "psd", lambda: synth.config("c2_small"), 128, 1e-8, "online", 0),
    # 4 workgroups: 4 columns per lane, FP32 tile of 128 entries per lane
    ("c2_small_cpl4", "psd", lambda: synth.config("c2_small"), 128, 1e-8, "online", 4),
    ("c3_small", "general", lambda: synth.config("c3_small"), 256, 1e-8, "fixed", 0),
    # s = 256 in a team of 11 workgroups (one column per lane)
    ("c3_small_team11", "general", lambda: synth.config("c3_small"), 256, 1e-8, "fixed", 6),
    ("c4_small", "general", lambda: synth.config("c4_small"), 64, 1e-4, "online", 0),
]


@pytest.mark.parametrize("case", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_precision_reaches_fp64_accuracy(env, case):
    """Iterative refinement recovers a true FP64 relative residual of 1e-10;
    the error against the FP64 oracle's converged solution is stated."""
    kpp, torch, dev, ctx = env
    name, kind, build, s, lam, mode, team_groups = case
    sysm = build()
    A, b = sysm.A, sysm.b
    m, n = A.shape
    ck = kpp.KPP_CD_PSD if kind == "psd" else kpp.KPP_KACZMARZ
    p = kpp.kpp_params_default(ck)
    p.block_size = s
    p.lambda_ = lam
    p.tol = 1e-10
    p.max_iters = 200_000
    p.seed = 77
    p.memo = MODES[mode]
    p.precision = kpp.KPP_MIXED_FP32
    p.team_groups = team_groups
    Ad = torch.from_numpy(A).to(dev)
    bd = torch.from_numpy(b).to(dev)
    xd = torch.zeros(n, dtype=torch.float64, device=dev)
    h = kpp.kpp_system_create(ctx, ck, m, n, Ad.data_ptr(), n, bd.data_ptr())
    try:
        st, res = kpp.kpp_solve(h, p, xd.data_ptr())
    finally:
        kpp.kpp_system_destroy(h)
    x = xd.cpu().numpy()
    true_rel = np.linalg.norm(A @ x - b) / np.linalg.norm(b)
    ref = oracle_solve(A, b, kind, s, lam=lam, T=200_000, tol=1e-10, mode=mode, seed=77)
    err_orc = relerr(x, ref.x)
    err_star = relerr(x, sysm.xstar)
    print(f"[mixed] {name}: status {st}, {res.refinements} refinements, {res.iters} inner steps "
          f"(FP64 oracle {ref.iters}), true rel. residual {true_rel:.2e}, "
          f"|x - x_fp64_oracle|/|x| = {err_orc:.2e}, |x - x*|/|x*| = {err_star:.2e}", flush=True)
    assert st == kpp.KPP_OK and res.converged == 1
    assert true_rel <= 1e-10 * 1.0001
    assert res.true_rel_res == pytest.approx(true_rel, rel=1e-6, abs=1e-14)
    assert res.refinements >= 1
    # both solutions satisfy ||A x - b|| <= 1e-10 ||b||, so within the row space
    # of A they differ by at most about kappa(A) * 1e-10 relative.  A wide system
    # also has a null space; its corrections are formed as A^T z with the FP64 A
    # (z the dual of the inner iterate), so x stays in the row space and the
    # minimum-norm solution is reached, not just some solution.
    kappa = synth_kappa(sysm)
    if m < n:
        Q, _ = np.linalg.qr(A.T)
        xr = Q @ (Q.T @ x)
        drift = np.linalg.norm(x - xr) / np.linalg.norm(x)
        print(f"[mixed] {name}: null-space component |x - P_row x|/|x| = {drift:.2e}", flush=True)
        assert drift <= 1e-10
    assert err_orc <= 2.0 * kappa * 1e-10 + 1e-12


def synth_kappa(sysm):
    sp = np.abs(np.asarray(sysm.spectrum))
    return float(sp.max() / sp.min())


def test_mixed_inner_round_ends_at_precision_floor(env):
    """An inner tolerance below what FP32 products can reach (1e-7 relative on
    a kappa = 1e5 system) does not trap the inner solve: a round ends once its
    residual estimate stalls and refinement still reaches 1e-10."""
    kpp, torch, dev, ctx = env
    sysm = synth.config("c2_small")
    A, b = sysm.A, sysm.b
    n = A.shape[0]
    p = kpp.kpp_params_default(kpp.KPP_CD_PSD)
    p.block_size = 128
    p.lambda_ = 1e-8
    p.tol = 1e-10
    p.max_iters = 200_000
    p.seed = 77
    p.precision = kpp.KPP_MIXED_FP32
    p.inner_tol = 1e-7
    Ad = torch.from_numpy(A).to(dev)
    bd = torch.from_numpy(b).to(dev)
    xd = torch.zeros(n, dtype=torch.float64, device=dev)
    h = kpp.kpp_system_create(ctx, kpp.KPP_CD_PSD, n, n, Ad.data_ptr(), n, bd.data_ptr())
    try:
        st, res = kpp.kpp_solve(h, p, xd.data_ptr())
    finally:
        kpp.kpp_system_destroy(h)
    print(f"[mixed floor] status {st}, {res.refinements} rounds, {res.iters} steps, true {res.true_rel_res:.2e}",
          flush=True)
    assert st == kpp.KPP_OK and res.true_rel_res <= 1e-10
    assert res.iters < 50_000


@pytest.mark.parametrize("name,kind,s,lam", [("c2_small", "psd", 128, 1e-8), ("c4_small", "general", 64, 1e-4)])
def test_untimed_launches_change_nothing(env, name, kind, s, lam):
    """Solves to a tolerance with the next window's launch enqueued before the
    current one ends, with and without per-launch HIP events: the same iterate
    bit for bit, the same steps and launches; without events no kernel time."""
    kpp, torch, dev, ctx = env
    sysm = synth.config(name)
    m, n = sysm.A.shape
    ck = kpp.KPP_CD_PSD if kind == "psd" else kpp.KPP_KACZMARZ
    Ad = torch.from_numpy(np.ascontiguousarray(sysm.A)).to(dev)
    bd = torch.from_numpy(np.ascontiguousarray(sysm.b)).to(dev)
    h = kpp.kpp_system_create(ctx, ck, m, n, Ad.data_ptr(), n, bd.data_ptr())
    try:
        out = []
        for untimed in (0, 1, 0):
            p = kpp.kpp_params_default(ck)
            p.block_size = s
            p.lambda_ = lam
            p.tol = 1e-10
            p.max_iters = 50000
            p.seed = 5
            p.engine = 2
            p.no_launch_timing = untimed
            xd = torch.zeros(n, dtype=torch.float64, device=dev)
            st, res = kpp.kpp_solve(h, p, xd.data_ptr())
            torch.cuda.synchronize()
            out.append((st, res, xd.cpu().numpy()))
        for st, res, _ in out:
            assert st == 0 and res.converged == 1 and res.engine_used == 2
        (_, r0, x0), (_, r1, x1), (_, r2, x2) = out
        assert np.array_equal(x0, x1) and np.array_equal(x0, x2)
        assert r0.iters == r1.iters == r2.iters and r0.kernel_launches == r1.kernel_launches
        assert r1.kernel_seconds == 0.0 and r0.kernel_seconds > 0.0 and r2.kernel_seconds > 0.0
    finally:
        kpp.kpp_system_destroy(h)
