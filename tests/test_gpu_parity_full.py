"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark runs: the fused step kernel with its real team geometry against the
CPU oracle on the same seeded input and the same seeded block schedule.

  * n = 4096 SPD, CD++, blocks of 128, online memo: k_fused<CD++, 2 columns
    per lane, FP64> with 32 workgroups and 16-byte tile loads;
  * 2048 x 32768, Kaczmarz++, blocks of 128, online memo: 256 workgroups
    (the largest team), y split across the team;
  * 65536 x 2048, Kaczmarz++, blocks of 256, fixed partition into 256 blocks:
    32 workgroups of one column per lane, 1024 steps (two checkpoint windows).

The systems are generated on the device (seeded torch generators) and copied
to the host for the oracle.  Bar: max(1e-10, 10 nf) relative, nf the oracle's
distance to itself with every sum taken in the opposite order (block Grams of
the tall workload have kappa ~ 1e9, which amplifies rounding past 1e-10 for
any two valid FP64 implementations); rho within its own noise floor; the
memo-miss count equal to the oracle's factorization count.
"""
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


_CACHE = {}


def full_system(name):
    """The named workload on the device plus a host copy (one kept at a time)."""
    if name not in _CACHE:
        _CACHE.clear()
        sysm = synth.config(name, device="cuda")
        _CACHE[name] = (sysm, sysm.A.cpu().numpy(), sysm.b.cpu().numpy())
    return _CACHE[name]


def relerr(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / (nb if nb > 0 else 1.0)


# name, kind, s, lambda, memo mode, step counts, fused geometry (groups, columns per lane)
FULL = [
    ("c2", "psd", 128, 1e-8, "online", (128, 256), (32, 2)),
    ("c4", "general", 128, 1e-4, "online", (96,), (256, 2)),
    ("c3", "general", 256, 1e-8, "fixed", (1024,), (32, 1)),
]


@pytest.mark.parametrize("engine", [2, 1], ids=["fused", "launch"])
@pytest.mark.parametrize("case", FULL, ids=[c[0] for c in FULL])
def test_full_size_iterates_match_oracle(env, case, engine):
    kpp, torch, dev, ctx = env
    name, kind, s, lam, mode, steps, geometry = case
    sysm, A, b = full_system(name)
    m, n = A.shape
    ck = kpp.KPP_CD_PSD if kind == "psd" else kpp.KPP_KACZMARZ
    N = n if kind == "psd" else m
    for T in steps:
        print(f"[full parity] {name} {m}x{n} s={s} engine={engine} T={T}", flush=True)
        p = kpp.kpp_params_default(ck)
        p.block_size = s
        p.lambda_ = lam
        p.tol = 0.0
        p.max_iters = T
        p.seed = 41
        p.memo = {"online": 1, "fixed": 2}[mode]
        p.fixed_partition = 1
        p.engine = engine
        xd = torch.zeros(n, dtype=torch.float64, device=dev)
        h = kpp.kpp_system_create(ctx, ck, m, n, sysm.A.data_ptr(), n, sysm.b.data_ptr())
        try:
            st, res = kpp.kpp_solve(h, p, xd.data_ptr())
        finally:
            kpp.kpp_system_destroy(h)
        x = xd.cpu().numpy()
        assert res.iters == T and res.engine_used == engine
        if engine == 2:
            assert (res.team_groups, res.cols_per_lane) == geometry
        schd = osch.make_schedule(mode, N, s, T, 41, B0=osch.online_rate(kind, m, n, s), partition=True)
        prm = dict(s=s, lam=lam, tol=0.0, max_iters=T)
        ref = okpp.solve(A, b, kind, okpp.Params(**prm), schd)
        alt = okpp.solve(A, b, kind, okpp.Params(reverse_sums=True, **prm), schd)
        nf = relerr(alt.x, ref.x)
        err = relerr(x, ref.x)
        print(f"[full parity] {name} engine={engine} T={T}: |x_gpu - x_orc|/|x_orc| = {err:.3e}, "
              f"noise floor {nf:.3e}, rho gpu {res.rho_final:.6g} oracle {ref.rho_final:.6g}", flush=True)
        assert err <= max(1e-10, 10.0 * nf), (name, T, err, nf)
        assert res.memo_misses == ref.factorizations
        rho_nf = abs(alt.rho_final - ref.rho_final)
        assert abs(res.rho_final - ref.rho_final) <= max(1e-9 * abs(ref.rho_final), 1e-12, 10.0 * rho_nf)
