"""Serving (continuous batching) through the C ABI: every request's result is
the one it gets alone, requests of different sizes share the device, and
admission follows the memory budget.

The same request served alone and in a mix runs the same steps in the same
arithmetic (per-request team geometry, fixed-order reductions, the same block
schedule and stop decisions), so iterates are compared bit for bit.  Served
results are also checked against kpp_solve (a different team geometry: 1e-10
relative, the FP64 parity bar) and against the planted solution.
"""
import time

import numpy as np
import pytest

import synth
from oracle import kpp as okpp
from oracle import schedule as osch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def senv():
    import torch

    import paper_2501_11673_amd as kpp

    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)   # the server's worker runs on this stream
    ctx = kpp.kpp_context_create(0, stream.cuda_stream)
    yield kpp, torch, dev, ctx
    kpp.kpp_context_destroy(ctx)


# (kind, m, n, s, lam, tol, precision, seed): a mix of sizes, kinds and precisions
MIX = [
    ("psd", 500, 500, 64, 1e-8, 1e-10, "fp64", 31),
    ("psd", 1100, 1100, 128, 1e-8, 1e-6, "mixed", 32),
    ("psd", 300, 300, 32, 1e-8, 1e-10, "mixed", 33),
    ("general", 900, 350, 50, 1e-6, 1e-10, "fp64", 34),
    ("psd", 1500, 1500, 128, 1e-8, 1e-10, "fp64", 35),
    ("general", 400, 1200, 64, 1e-4, 1e-8, "mixed", 36),
]


def make_case(env, case):
    kpp, torch, dev, ctx = env
    kind, m, n, s, lam, tol, prec, seed = case
    if kind == "psd":
        sysm = synth.psd_system(n, lambda rng, k: synth.spectrum_c2(rng, k, 8), seed, device="cuda")
    else:
        sysm = synth.svd_system(m, n, synth.spectrum_c1, seed, x_in_rowspace=m < n, device="cuda")
    ck = kpp.KPP_CD_PSD if kind == "psd" else kpp.KPP_KACZMARZ
    p = kpp.kpp_params_default(ck)
    p.block_size = s
    p.lambda_ = lam
    p.tol = tol
    p.seed = 1000 + seed
    p.max_iters = 200_000
    p.precision = kpp.KPP_MIXED_FP32 if prec == "mixed" else kpp.KPP_FP64
    p.memo = kpp.KPP_MEMO_ONLINE   # a fixed partition stalls on these outlier spectra
    h = kpp.kpp_system_create(ctx, ck, sysm.A.shape[0], n, sysm.A.data_ptr(), n, sysm.b.data_ptr())
    return sysm, h, p


def serve(env, jobs, *, budget=64 << 30, max_active=16, wait=60.0):
    """jobs: [(system handle, params, x tensor)]; returns ({id: (status, result)}, stats)."""
    kpp, torch, dev, ctx = env
    torch.cuda.synchronize()
    srv = kpp.kpp_server_create(ctx, budget, max_active)
    try:
        ids = [kpp.kpp_server_submit(srv, h, p, x.data_ptr()) for h, p, x in jobs]
        out = {}
        t_end = time.time() + wait
        while len(out) < len(ids) and time.time() < t_end:
            for rid, st, res in kpp.kpp_server_poll(srv, 64, 0.5):
                out[rid] = (st, res)
        stats = kpp.kpp_server_stats(srv).as_dict()
    finally:
        kpp.kpp_server_destroy(srv)
    assert len(out) == len(ids), f"only {len(out)} of {len(ids)} requests finished"
    return [out[i] for i in ids], stats


def oracle_of(case, sysm, p, tol, T):
    """The FP64 oracle on the request's system, parameters and block schedule;
    also the run with every sum reversed (the FP64 noise floor)."""
    kind, m, n, s, lam = case[:5]
    A = sysm.A.cpu().numpy()
    b = sysm.b.cpu().numpy()
    N = n if kind == "psd" else m
    schd = osch.make_schedule("online", N, s, T, int(p.seed), B0=osch.online_rate(kind, m, n, s))
    prm = dict(s=s, lam=lam, tol=tol, max_iters=T)
    ref = okpp.solve(A, b, kind, okpp.Params(**prm), schd)
    alt = okpp.solve(A, b, kind, okpp.Params(reverse_sums=True, **prm), schd)
    return ref, alt, A, b


def relerr(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / (nb if nb > 0 else 1.0)


def test_served_request_matches_kpp_solve(senv):
    kpp, torch, dev, ctx = senv
    sysm, h, p = make_case(senv, MIX[0])
    try:
        x_srv = torch.zeros(sysm.A.shape[1], dtype=torch.float64, device=dev)
        [(st, res)], stats = serve(senv, [(h, p, x_srv)])
        assert st == kpp.KPP_OK and res.converged
        assert res.true_rel_res <= p.tol
        x_ref = torch.zeros_like(x_srv)
        st2, res2 = kpp.kpp_solve(h, p, x_ref.data_ptr())
        torch.cuda.synchronize()
        assert st2 == kpp.KPP_OK
        assert res.iters == res2.iters
        rel = float(torch.linalg.norm(x_srv - x_ref) / torch.linalg.norm(x_ref))
        assert rel <= 1e-10, rel
        assert stats["completed"] == 1 and stats["peak_active"] == 1
    finally:
        kpp.kpp_system_destroy(h)


def test_mix_equals_alone(senv):
    """Each result of a mixed batch is bit-identical to the same request served
    alone, the requests were on the device together, and every one reached its
    tolerance (the mixed-precision ones through FP64 refinement)."""
    kpp, torch, dev, ctx = senv
    built = [make_case(senv, c) for c in MIX]
    try:
        xs_mix = [torch.zeros(s.A.shape[1], dtype=torch.float64, device=dev) for s, _, _ in built]
        mix, stats = serve(senv, [(h, p, x) for (s, h, p), x in zip(built, xs_mix)])
        assert stats["peak_active"] >= 3, stats
        for (case, (sysm, h, p), x, (st, res)) in zip(MIX, built, xs_mix, mix):
            print(case, st, res.iters, res.refinements, res.true_rel_res, res.seconds_queued, flush=True)
            assert st == kpp.KPP_OK, (case, st)
            assert res.true_rel_res <= p.tol, (case, res.true_rel_res)
            err = float(torch.linalg.norm(x - sysm.xstar) / torch.linalg.norm(sysm.xstar))
            bound = 1e-2 if p.tol > 1e-8 else 1e-5
            assert err < bound, (case, err)
        # against the FP64 oracle on the same schedule: an FP64 request stops at
        # the oracle's step with the oracle's iterate (FP64 parity bar); a
        # mixed-precision request is within kappa * tol of it (both solve the
        # system to tol), the distance printed
        for (case, (sysm, h, p), x_m, (st_m, res_m)) in zip(MIX, built, xs_mix, mix):
            ref, alt, A, b = oracle_of(case, sysm, p, p.tol, 200_000)
            assert ref.converged
            err = relerr(x_m.cpu().numpy(), ref.x)
            print(f"[serve vs oracle] {case}: served {res_m.iters} steps, oracle {ref.iters}, "
                  f"|x - x_oracle|/|x_oracle| = {err:.2e}", flush=True)
            if case[6] == "fp64":
                assert res_m.iters == ref.iters, case
                assert err <= max(1e-10, 10.0 * relerr(alt.x, ref.x)), (case, err)
            else:
                sp = np.abs(np.asarray(sysm.spectrum))
                assert err <= 2.0 * float(sp.max() / sp.min()) * p.tol + 1e-12, (case, err)
        for (case, (sysm, h, p), x_m, (st_m, res_m)) in zip(MIX, built, xs_mix, mix):
            x_a = torch.zeros_like(x_m)
            [(st_a, res_a)], stats_a = serve(senv, [(h, p, x_a)])
            assert stats_a["peak_active"] == 1
            assert st_a == st_m and res_a.iters == res_m.iters and res_a.refinements == res_m.refinements, case
            assert torch.equal(x_a, x_m), (case, float(torch.max(torch.abs(x_a - x_m))))
    finally:
        for _, h, _ in built:
            kpp.kpp_system_destroy(h)


# FP64 requests of different kinds and sizes run for a fixed number of steps
# (tol = 0): (kind, m, n, s, lam, steps, seed)
FIXED_MIX = [
    ("psd", 700, 700, 64, 1e-8, 300, 41),
    ("general", 900, 350, 50, 1e-6, 250, 42),
    ("psd", 1500, 1500, 128, 1e-8, 200, 43),
    ("general", 400, 1200, 64, 1e-4, 150, 44),
    ("psd", 4096, 4096, 128, 1e-8, 128, 45),
]


def test_served_fixed_steps_match_oracle(senv):
    """Requests served together (shared persistent launches, one team each)
    give the oracle's iterates after their step budget, within the FP64
    parity bar max(1e-10, 10 nf)."""
    kpp, torch, dev, ctx = senv
    built = []
    try:
        for case in FIXED_MIX:
            kind, m, n, s, lam, T, seed = case
            sysm, h, p = make_case(senv, (kind, m, n, s, lam, 0.0, "fp64", seed))
            p.max_iters = T
            built.append((case, sysm, h, p))
        xs = [torch.zeros(c[2], dtype=torch.float64, device=dev) for c, _, _, _ in built]
        out, stats = serve(senv, [(h, p, x) for (_, _, h, p), x in zip(built, xs)])
        assert stats["peak_active"] >= 2, stats
        for (case, sysm, h, p), x, (st, res) in zip(built, xs, out):
            kind, m, n, s, lam, T, seed = case
            assert st == kpp.KPP_NOT_CONVERGED and res.iters == T, (case, st, res.iters)
            ref, alt, A, b = oracle_of(case, sysm, p, 0.0, T)
            err = relerr(x.cpu().numpy(), ref.x)
            nf = relerr(alt.x, ref.x)
            print(f"[serve fixed] {case}: |x - x_oracle|/|x_oracle| = {err:.2e} (noise floor {nf:.2e})", flush=True)
            assert err <= max(1e-10, 10.0 * nf), (case, err, nf)
            assert res.memo_misses == ref.factorizations
    finally:
        for _, _, h, _ in built:
            kpp.kpp_system_destroy(h)


def test_admission_by_memory_budget(senv):
    """A budget that fits one request at a time still serves them all (one by
    one); a request larger than the budget is refused at submission."""
    kpp, torch, dev, ctx = senv
    built = [make_case(senv, c) for c in MIX[:3]]
    try:
        xs = [torch.zeros(s.A.shape[1], dtype=torch.float64, device=dev) for s, _, _ in built]
        # the largest footprint: the middle request (n = 1100, mixed) fits with
        # neither neighbour, and admission in arrival order keeps the third
        # one waiting behind it
        feet = [kpp.kpp_request_footprint(h, p) for _, h, p in built]
        budget = max(feet)
        assert feet[1] == budget and feet[0] + feet[1] > budget and feet[1] + feet[2] > budget
        res, stats = serve(senv, [(h, p, x) for (s, h, p), x in zip(built, xs)], budget=budget)
        assert all(st == kpp.KPP_OK for st, _ in res)
        assert stats["peak_active"] == 1 and stats["peak_bytes"] <= budget, stats
        assert max(r.seconds_queued for _, r in res) > 0.0
        srv = kpp.kpp_server_create(ctx, 1 << 20, 4)
        try:
            with pytest.raises(kpp.KppError) as ei:
                kpp.kpp_server_submit(srv, built[1][1], built[1][2], xs[1].data_ptr())
            assert ei.value.status == kpp.KPP_ERR_REJECTED
            assert kpp.kpp_server_stats(srv).rejected == 1
        finally:
            kpp.kpp_server_destroy(srv)
    finally:
        for _, h, _ in built:
            kpp.kpp_system_destroy(h)


def test_requests_on_one_system_are_serialized(senv):
    """Two requests on the same system (different starting points) are not
    active together and each matches its own solve alone."""
    kpp, torch, dev, ctx = senv
    sysm, h, p = make_case(senv, MIX[3])
    try:
        n = sysm.A.shape[1]
        g = torch.Generator(device=dev)
        g.manual_seed(5)
        x0 = torch.randn(n, dtype=torch.float64, device=dev, generator=g)
        xa = torch.zeros(n, dtype=torch.float64, device=dev)
        xb = x0.clone()
        res, stats = serve(senv, [(h, p, xa), (h, p, xb)])
        assert stats["peak_active"] == 1
        assert all(st == kpp.KPP_OK for st, _ in res)
        xb_alone = x0.clone()
        [(st, r)], _ = serve(senv, [(h, p, xb_alone)])
        assert torch.equal(xb_alone, xb)
        assert r.iters == res[1][1].iters
    finally:
        kpp.kpp_system_destroy(h)


def test_invalid_request_is_refused(senv):
    kpp, torch, dev, ctx = senv
    sysm, h, p = make_case(senv, MIX[0])
    try:
        srv = kpp.kpp_server_create(ctx, 1 << 30, 4)
        try:
            x = torch.zeros(sysm.A.shape[1], dtype=torch.float64, device=dev)
            bad = kpp.kpp_params_default(kpp.KPP_CD_PSD)
            bad.block_size = 0
            with pytest.raises(kpp.KppError) as ei:
                kpp.kpp_server_submit(srv, h, bad, x.data_ptr())
            assert ei.value.status == kpp.KPP_ERR_INVALID_ARG
            eng = kpp.kpp_params_default(kpp.KPP_CD_PSD)
            eng.engine = 1
            with pytest.raises(kpp.KppError):
                kpp.kpp_server_submit(srv, h, eng, x.data_ptr())
        finally:
            kpp.kpp_server_destroy(srv)
    finally:
        kpp.kpp_system_destroy(h)
