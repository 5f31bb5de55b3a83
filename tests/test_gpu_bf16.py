"""Mixed precision with bfloat16 storage of A (GPU, through the C ABI).

The inner solves of the iterative refinement read A in bfloat16 (8-bit
significand, widened to FP32 in the step kernel's tile, FP32 products); the
Grams, factors, residuals and x stay FP64.  Each refinement round can gain
at most about -log10(kappa(A) 2^-8) digits, so the method converges when
kappa(A) is well below 2^8 and cannot converge above it.  Bar: on
well-conditioned systems (kappa <= 10) the refined solve reaches the FP64
tolerance 1e-10 and the planted solution to 1e-8; on a kappa ~ 1e4 system
(the outlier spectrum of the 2048 x 32768 workload, reduced) it reports
KPP_NOT_CONVERGED with a finite true residual above the tolerance (a
diverging refinement ends early and the iterate with the lowest true
residual is returned).
"""
import numpy as np
import pytest

import synth

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


def solve(env, sysm, kind, s, lam, precision, rounds=30):
    kpp, torch, dev, ctx = env
    A, b = np.ascontiguousarray(sysm.A), np.ascontiguousarray(sysm.b)
    m, n = A.shape
    ck = kpp.KPP_CD_PSD if kind == "psd" else kpp.KPP_KACZMARZ
    Ad, bd = torch.from_numpy(A).to(dev), torch.from_numpy(b).to(dev)
    h = kpp.kpp_system_create(ctx, ck, m, n, Ad.data_ptr(), n, bd.data_ptr())
    p = kpp.kpp_params_default(ck)
    p.block_size = s
    p.lambda_ = lam
    p.tol = 1e-10
    p.max_iters = 400_000
    p.seed = 13
    p.precision = precision
    p.refine_max_rounds = rounds
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    try:
        st, r = kpp.kpp_solve(h, p, x.data_ptr())
    finally:
        kpp.kpp_system_destroy(h)
    return x.cpu().numpy(), st, r


@pytest.mark.parametrize("kind,m,n,s", [("general", 1200, 300, 32), ("general", 200, 1500, 32), ("psd", 600, 600, 48)])
def test_bf16_converges_on_well_conditioned_systems(env, kind, m, n, s):
    kpp = env[0]
    sysm = synth.tiny_system(kind, m, n, seed=41, cond=10.0)
    x, st, r = solve(env, sysm, kind, s, 1e-8, kpp.KPP_MIXED_BF16)
    err = float(np.linalg.norm(x - sysm.xstar) / np.linalg.norm(sysm.xstar))
    print(f"[bf16] {kind} {m}x{n}: st={st} rounds={r.refinements} iters={r.iters} "
          f"true_rel={r.true_rel_res:.2e} err={err:.2e}", flush=True)
    assert st == kpp.KPP_OK and r.converged and r.true_rel_res <= 1e-10
    assert err < 1e-8
    assert r.refinements >= 2   # bfloat16 alone cannot reach 1e-10: the FP64 outer loop does


def test_bf16_reports_non_convergence_on_ill_conditioned_system(env):
    kpp = env[0]
    sysm = synth.config("c4_small")
    x, st, r = solve(env, sysm, "general", 64, 1e-4, kpp.KPP_MIXED_BF16, rounds=12)
    print(f"[bf16] c4_small: st={st} rounds={r.refinements} iters={r.iters} true_rel={r.true_rel_res:.2e}",
          flush=True)
    assert st == kpp.KPP_NOT_CONVERGED and not r.converged
    assert np.isfinite(r.true_rel_res) and r.true_rel_res > 1e-10
    assert np.all(np.isfinite(x))   # the best iterate, not the diverged one
    # the same system converges in FP32 mixed precision and in FP64
    for prec in (kpp.KPP_MIXED_FP32, kpp.KPP_FP64):
        _, st2, r2 = solve(env, sysm, "general", 64, 1e-4, prec)
        assert st2 == kpp.KPP_OK and r2.true_rel_res <= 1e-10


def test_bf16_refused_by_the_server(env):
    kpp, torch, dev, ctx = env
    sysm = synth.tiny_system("psd", 64, 64, seed=3)
    Ad, bd = torch.from_numpy(sysm.A).to(dev), torch.from_numpy(sysm.b).to(dev)
    h = kpp.kpp_system_create(ctx, kpp.KPP_CD_PSD, 64, 64, Ad.data_ptr(), 64, bd.data_ptr())
    try:
        p = kpp.kpp_params_default(kpp.KPP_CD_PSD)
        p.block_size = 8
        p.precision = kpp.KPP_MIXED_BF16
        with pytest.raises(kpp.KppError) as e:
            kpp.kpp_request_footprint(h, p)
        assert e.value.status == kpp.KPP_ERR_INVALID_ARG
    finally:
        kpp.kpp_system_destroy(h)
