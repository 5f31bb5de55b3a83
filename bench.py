"""Benchmark: time to a true 1e-10 relative residual and block-iterations/s.

Workload: CD++ (Algorithm 2, no randomized Hadamard preprocessing) on a dense
SPD system A = Q diag(lambda) Q^T, n = 4096, Q Haar, 32 eigenvalues log-spaced
in [1e3, 1e5] and 4064 uniform in [1, 10]; b = A x*, x* ~ N(0, I); block size
128, lambda = 1e-8, online block memoization (Section 5.2), tolerance 1e-10 on
||A x - b|| / ||b|| confirmed in FP64.  Inputs are synthetic and seeded and are
resident in HBM before the timed region.

One "step" is one full solve from x0 = 0 with an empty memo cache (every
factorization is paid inside the timed region).  value = block steps per
second over the timed solves; ms_per_step = time to tolerance per solve.
The same solves are then timed with mixed precision (FP32 block products,
FP64 factors and iterative refinement) and reported under "mixed", and the
serving workload (continuous batching of 512 solves arriving at 200/s) is
replayed in real time and reported under "serving" (p50/p99 latency).  Under
"rht": the randomized Hadamard preprocessing (Definition d:rht) timed at the
workloads' shapes, and the same CD++ solve with it.  Under "flops_to_tol": the
paper's FLOP comparison (Section 6.3) re-run on synthetic kernel matrices.
Under "lsqr": Kaczmarz++ with the exact and with the LSQR projection.  Under
"ablation": the four Kaczmarz++ variants of the paper's ablation table.  Under
"multi_rhs": 16 right-hand sides on the n = 4096 system solved together.

Also printed: the roofline of the dominant kernel (the step kernel, timed with
HIP events inside the library on the stream it runs on) and the CPU oracle
timed on the host on one full solve of the same system.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--engine", type=int, default=0, help="0 auto, 1 one launch per phase, 2 fused")
    ap.add_argument("--team-groups", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=202)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB three times (HBM counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--no-rht", action="store_true")
    ap.add_argument("--no-flops", action="store_true")
    ap.add_argument("--no-lsqr", action="store_true")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--rht-only", action="store_true",
                    help="only the randomized Hadamard transforms (for profiling them)")
    return ap.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_fused_cdpp_n4096_s128_fp64.md")


def measured_traffic(kernel_name):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes, each scaled by what the counter read for a
    device copy of known size.  None when the kernel's sources have changed
    since the counters were taken, or for another kernel."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"```json kpp-traffic\n(.*?)```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec["kernel"] != kernel_name:
        return None
    for rel, digest in rec["sources"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    fetch = rec["fetch_kib_per_dispatch"] * rec["copy_bytes"] / rec["copy_fetch_kib"]
    write = rec["write_kib_per_dispatch"] * rec["copy_bytes"] / rec["copy_write_kib"]
    return round(fetch + write, 1)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        n = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:  # pragma: no cover
        return 1


def cpu_baseline(A, b, s, lam, tol, seed):
    """The oracle as it stands, one full solve of the same system on the host."""
    from oracle import kpp as okpp
    from oracle import schedule as osch

    n = A.shape[0]
    T = 100_000
    schd = osch.make_schedule("online", n, s, T, seed, B0=osch.online_rate("psd", n, n, s))
    t0 = time.perf_counter()
    res = okpp.solve(A, b, "psd", okpp.Params(s=s, lam=lam, tol=tol, max_iters=T), schd)
    dt = time.perf_counter() - t0
    return {"value": res.iters / dt, "unit": "block-iters/s", "cores": blas_threads(),
            "kind": "oracle",
            "sample": f"one full CD++ solve of the n=4096 system to {tol:g} "
                      f"({res.iters} block steps, {dt:.2f} s, converged={res.converged})",
            "time_to_tol_s": dt}


def serving(kpp, torch, dev, num_requests, seed=5):
    """Serving workload: Poisson arrivals (200/s) of CD++ solves, n uniform over
    {512, ..., 8192} (each a seeded matrix from a pool of 8 per size, outlier
    spectrum as the n = 4096 workload), own right-hand side b = A x*, tolerance
    1e-6 or 1e-10, mixed precision.  Arrivals are replayed in real time against
    the server; latency = completion - scheduled arrival."""
    import numpy as np

    import synth

    reqs = synth.serving_workload(num_requests=num_requests, rate_per_s=200.0, seed=seed)
    pool = {}
    for r in reqs:
        key = (r["n"], r["pool_index"])
        if key not in pool:
            pool[key] = synth.serving_matrix(r["n"], r["pool_index"], device="cuda").A
    stream = torch.cuda.Stream(device=dev)
    ctx = kpp.kpp_context_create(0, stream.cuda_stream)
    systems, xs, bs, params = [], [], [], []
    for r in reqs:
        A = pool[(r["n"], r["pool_index"])]
        g = torch.Generator(device=dev)
        g.manual_seed(r["x_seed"])
        xstar = torch.randn(r["n"], dtype=torch.float64, device=dev, generator=g)
        b = A @ xstar
        bs.append(b)
        xs.append(torch.zeros(r["n"], dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        systems.append(kpp.kpp_system_create(ctx, kpp.KPP_CD_PSD, r["n"], r["n"], A.data_ptr(), r["n"], b.data_ptr()))
        p = kpp.kpp_params_default(kpp.KPP_CD_PSD)
        p.block_size = 128
        p.lambda_ = 1e-8
        p.tol = r["tol"]
        p.memo = kpp.KPP_MEMO_ONLINE
        p.precision = kpp.KPP_MIXED_FP32
        p.seed = r["x_seed"]
        p.max_iters = 400_000
        params.append(p)
    torch.cuda.synchronize()
    srv = kpp.kpp_server_create(ctx, 96 << 30, 64)
    arrivals = [r["arrival_s"] for r in reqs]
    done = {}
    rid_of = {}
    i = 0
    t0 = time.perf_counter()
    while len(done) < len(reqs):
        now = time.perf_counter() - t0
        while i < len(reqs) and arrivals[i] <= now:
            rid_of[kpp.kpp_server_submit(srv, systems[i], params[i], xs[i].data_ptr())] = i
            i += 1
        wait = min(0.002, max(0.0, arrivals[i] - now)) if i < len(reqs) else 0.02
        for rid, st, res in kpp.kpp_server_poll(srv, 64, wait):
            done[rid_of[rid]] = (st, res, time.perf_counter() - t0)
        if now > 600:
            break
    wall = time.perf_counter() - t0
    info = kpp.kpp_server_stats(srv).as_dict()
    kpp.kpp_server_destroy(srv)
    for h in systems:
        kpp.kpp_system_destroy(h)
    kpp.kpp_context_destroy(ctx)
    lat = np.array([done[k][2] - arrivals[k] for k in sorted(done)])
    ok = [done[k][0] == kpp.KPP_OK and done[k][1].true_rel_res <= reqs[k]["tol"] for k in sorted(done)]
    iters = sum(done[k][1].iters for k in done)
    by_n = {}
    for k in sorted(done):
        by_n.setdefault(reqs[k]["n"], []).append(done[k][2] - arrivals[k])
    last = max(v[2] for v in done.values()) if done else wall
    return {
        "workload": f"{len(reqs)} CD++ solves, Poisson 200/s, n in {{512..8192}}, tol 1e-6/1e-10, mixed precision",
        "completed": len(done), "all_reached_tol": bool(all(ok)) and len(done) == len(reqs),
        "p50_latency_ms": float(1e3 * np.percentile(lat, 50)), "p99_latency_ms": float(1e3 * np.percentile(lat, 99)),
        "mean_latency_ms": float(1e3 * lat.mean()),
        "latency_ms_by_n": {str(n): {"p50": float(1e3 * np.percentile(v, 50)), "p99": float(1e3 * np.percentile(v, 99)),
                                     "count": len(v)} for n, v in sorted(by_n.items())},
        "requests_per_s": len(done) / last, "block_iters_per_s": iters / last,
        "makespan_s": last, "arrival_span_s": arrivals[-1],
        "peak_active": info["peak_active"], "rounds": info["rounds"],
        "device_busy_fraction": info["busy_seconds"] / last,
        "max_true_rel_res_over_tol": float(max(done[k][1].true_rel_res / reqs[k]["tol"] for k in done)),
    }


def rht_transforms(kpp, torch, dev, ctx, A, b, reps=5):
    """Randomized Hadamard preprocessing at the workloads' shapes, timed with
    events on the library's stream: the two-sided CD++ transform of the n = 4096
    system (two passes), and the Kaczmarz++ row transform of a 2048 x 32768
    (one pass) and a 65536 x 2048 (two passes) seeded normal matrix.
    Algorithmic bytes: read the input once, write the output once."""
    out = {}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / reps

    n = A.shape[0]
    R = n
    sg = torch.tensor(kpp.kpp_rht_signs(11, R), dtype=torch.int8, device=dev)
    At = torch.empty((R, R), dtype=torch.float64, device=dev)
    bt = torch.empty((R,), dtype=torch.float64, device=dev)
    t = timed(lambda: kpp.kpp_rht_psd(ctx, n, A.data_ptr(), n, b.data_ptr(), sg.data_ptr(), R, At.data_ptr(), R,
                                      bt.data_ptr()))
    alg = 8.0 * (n * n + R * R + n + R)
    out["psd_n4096"] = {"us": round(t * 1e6, 2), "passes_over_A": 2, "bytes_algorithmic": alg,
                        "achieved_GBs": round(alg / t / 1e9, 1), "frac": round(alg / t / 1e9 / HBM_PEAK_GBS, 4)}
    del At, bt
    g = torch.Generator(device=dev)
    g.manual_seed(404)
    for name, m, nn in (("general_2048x32768", 2048, 32768), ("general_65536x2048", 65536, 2048)):
        M = 1
        while M < m:
            M *= 2
        X = torch.randn((m, nn), generator=g, dtype=torch.float64, device=dev)
        y = torch.randn((m,), generator=g, dtype=torch.float64, device=dev)
        sg = torch.tensor(kpp.kpp_rht_signs(12, M), dtype=torch.int8, device=dev)
        Xt = torch.empty((M, nn), dtype=torch.float64, device=dev)
        yt = torch.empty((M,), dtype=torch.float64, device=dev)
        t = timed(lambda: kpp.kpp_rht_general(ctx, m, nn, X.data_ptr(), nn, y.data_ptr(), sg.data_ptr(), M,
                                              Xt.data_ptr(), nn, yt.data_ptr()))
        alg = 8.0 * (m * nn + M * nn + m + M)
        out[name] = {"us": round(t * 1e6, 2), "passes_over_A": 1 if M <= 4096 else 2, "bytes_algorithmic": alg,
                     "achieved_GBs": round(alg / t / 1e9, 1), "frac": round(alg / t / 1e9 / HBM_PEAK_GBS, 4)}
        del X, Xt
    return out


def rht_solves(kpp, torch, dev, h, p, x, reps):
    """CD++ on the same system with params.rht = 1: the first solve forms the
    transformed system, later ones reuse it."""
    q = kpp.kpp_params_default(kpp.KPP_CD_PSD)
    for f, _ in kpp.kpp_params._fields_:
        setattr(q, f, getattr(p, f))
    q.rht = 1
    q.rht_seed = 2
    times, res = [], []
    for _ in range(1 + reps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, r = kpp.kpp_solve(h, q, x.data_ptr())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        res.append((st, r))
    cached = times[1:]
    return {"first_solve_ms": round(1e3 * times[0], 3),
            "time_to_tol_ms": round(1e3 * sum(cached) / max(len(cached), 1), 3),
            "iters_per_solve": sum(r.iters for _, r in res[1:]) / max(len(cached), 1),
            "converged": all(st == kpp.KPP_OK and r.converged for st, r in res),
            "true_rel_res": res[-1][1].true_rel_res}


PAPER_TAB_FLOPS = {
    # Table tab:flops (Section 6.3 and its appendix), over its 20 matrices: min and max
    "full_cdpp": {"1e-04": [2.23e8, 5.71e9], "1e-08": [1.80e9, 3.64e10]},
    "cdpp_wo_rht": {"1e-04": [4.39e6, 3.63e9], "1e-08": [1.79e9, 3.11e10]},
    "gmres": {"1e-04": [3.37e8, 4.87e9], "1e-08": [1.33e9, 1.70e10]},
    "cg": {"1e-04": [3.70e8, 1.65e10], "1e-08": [3.26e9, 5.55e10]},
}


def flops_to_tol(kpp, torch, dev, ctx, seed):
    """The paper's FLOP comparison (Section 6.3, Table tab:flops) on synthetic
    data: CD++ with and without RHT on Gaussian and Laplacian kernel matrices
    (gamma 0.1 and 0.01) of n = 4096 seeded points plus 1e-3 I, b ~ N(0, I),
    s = 200, lambda = 1e-8, online memo; FLOPs counted as the paper counts them
    (kpp_result.flops, RHT included), next to the range of the paper's own
    numbers over its 20 matrices (other data, no hardware stated)."""
    import synth

    rows = []
    n, s = 4096, 200
    for kern in ("gaussian", "laplacian"):
        for gamma in (0.1, 0.01):
            sysm = synth.kernel_system(kern, n, gamma, seed=seed, device="cuda")
            for rht in (1, 0):
                for tol in (1e-4, 1e-8):
                    h = kpp.kpp_system_create(ctx, kpp.KPP_CD_PSD, n, n, sysm.A.data_ptr(), n, sysm.b.data_ptr())
                    p = kpp.kpp_params_default(kpp.KPP_CD_PSD)
                    p.block_size = s
                    p.lambda_ = 1e-8
                    p.tol = tol
                    p.max_iters = 400_000
                    p.seed = seed
                    p.rht = rht
                    p.rht_seed = seed + 1
                    x = torch.zeros(n, dtype=torch.float64, device=dev)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st, r = kpp.kpp_solve(h, p, x.data_ptr())
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    kpp.kpp_system_destroy(h)
                    rows.append({"matrix": f"{kern} gamma={gamma:g}", "method": "full_cdpp" if rht else "cdpp_wo_rht",
                                 "tol": tol, "flops": r.flops, "iters": r.iters, "ms": round(1e3 * dt, 3),
                                 "converged": bool(st == kpp.KPP_OK and r.converged),
                                 "true_rel_res": r.true_rel_res})
            del sysm
    return {"workload": "CD++ on n=4096 kernel matrices + 1e-3 I (seeded Gaussian points, d=8), s=200, "
                        "lambda=1e-8, online memo; b ~ N(0, I)",
            "runs": rows, "paper_tab_flops_range": PAPER_TAB_FLOPS}


def ablation(kpp, torch, dev, ctx):
    """The four Kaczmarz++ variants of Table tab:kacz-variants (Appendix F.1)
    on the 1000 x 200 workload to 1e-10, with its block size 20 and with 5
    (fewer rows than the 10 outlying singular values): Full K++ (acceleration
    and online memo), w/o Accel (eta = 0), w/o Memo (a new block, and its
    factor, every step) and plain randomized block Kaczmarz (neither)."""
    import synth

    sysm = synth.config("c1", device="cuda")
    A, b = sysm.A, sysm.b
    m, n = A.shape
    h = kpp.kpp_system_create(ctx, kpp.KPP_KACZMARZ, m, n, A.data_ptr(), n, b.data_ptr())
    out = {}
    for s, name, accel, memo in [(s, nm, a, mm) for s in (20, 5)
                                 for nm, a, mm in (("full_kpp", 1, 1), ("wo_accel", 0, 1), ("wo_memo", 1, 0),
                                                   ("kaczmarz", 0, 0))]:
        p = kpp.kpp_params_default(kpp.KPP_KACZMARZ)
        p.block_size = s
        p.lambda_ = 1e-3
        p.tol = 1e-10
        p.memo = memo
        p.accel = accel
        p.max_iters = 200_000
        p.seed = sysm.params["schedule_seed"]
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, r = kpp.kpp_solve(h, p, x.data_ptr())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.setdefault(f"s{s}", {})[name] = {"iters": r.iters, "time_to_tol_ms": round(1e3 * dt, 3), "flops": r.flops,
                     "factorizations": r.memo_misses, "converged": bool(st == kpp.KPP_OK and r.converged),
                     "true_rel_res": r.true_rel_res}
    kpp.kpp_system_destroy(h)
    return out


def multi_rhs(kpp, torch, dev, ctx, h, A, n, p, k=16):
    """k right-hand sides b_c = A x*_c (seeded x*_c ~ N(0, I)) on the n = 4096
    system, solved together to 1e-10 (kpp_solve_multi: one pass over A_S per
    step for all k): aggregate block steps per second."""
    g = torch.Generator(device=dev)
    g.manual_seed(77)
    Xs = torch.randn((n, k), generator=g, dtype=torch.float64, device=dev)
    B = (A @ Xs).contiguous()
    X = torch.zeros((n, k), dtype=torch.float64, device=dev)
    q = kpp.kpp_params_default(kpp.KPP_CD_PSD)
    for f, _ in kpp.kpp_params._fields_:
        setattr(q, f, getattr(p, f))
    q.engine = 0
    kpp.kpp_solve_multi(h, q, k, B.data_ptr(), k, X.data_ptr(), k)   # warm-up
    X.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, res = kpp.kpp_solve_multi(h, q, k, B.data_ptr(), k, X.data_ptr(), k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = [r.iters for r in res]
    err = float(torch.max(torch.linalg.norm(X - Xs, dim=0) / torch.linalg.norm(Xs, dim=0)))
    return {"k": k, "time_ms": round(1e3 * dt, 3), "iters_min": min(iters), "iters_max": max(iters),
            "block_iters_per_s_aggregate": sum(iters) / dt, "steps_per_s": max(iters) / dt,
            "all_converged": bool(st == kpp.KPP_OK and all(r.converged for r in res)),
            "max_true_rel_res": max(r.true_rel_res for r in res), "max_rel_err_vs_planted": err}


def lsqr_solves(kpp, torch, dev, ctx):
    """Kaczmarz++ to 1e-10 with the exact projection (the memoized Cholesky
    factor) and with the sketch-preconditioned LSQR projection (t_max = 8,
    tau = 2s; Section 4.1) on the 1000 x 200 and 65536 x 2048 workloads."""
    import synth

    out = {}
    for name, cfg, s, lam, memo in (("k_1000x200_s20", "c1", 20, 1e-3, 1), ("k_65536x2048_s256", "c3", 256, 1e-8, 2)):
        sysm = synth.config(cfg, device="cuda")
        A, b = sysm.A, sysm.b
        m, n = A.shape
        h = kpp.kpp_system_create(ctx, kpp.KPP_KACZMARZ, m, n, A.data_ptr(), n, b.data_ptr())
        rec = {}
        for proj in (kpp.KPP_PROJ_EXACT, kpp.KPP_PROJ_LSQR):
            p = kpp.kpp_params_default(kpp.KPP_KACZMARZ)
            p.block_size = s
            p.lambda_ = lam
            p.tol = 1e-10
            p.memo = memo
            p.fixed_partition = 1
            p.max_iters = 200_000
            p.seed = sysm.params["schedule_seed"]
            p.projection = proj
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, r = kpp.kpp_solve(h, p, x.data_ptr())
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec["exact" if proj == 0 else "lsqr_t8"] = {
                "time_to_tol_ms": round(1e3 * dt, 3), "iters": r.iters, "us_per_step": round(1e6 * dt / max(r.iters, 1), 2),
                "flops": r.flops, "converged": bool(st == kpp.KPP_OK and r.converged), "true_rel_res": r.true_rel_res,
                "engine": r.engine_used,
                "rel_err_vs_planted": float(torch.linalg.norm(x - sysm.xstar) / torch.linalg.norm(sysm.xstar))}
        kpp.kpp_system_destroy(h)
        out[name] = rec
        del sysm, A, b
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 "
              "(the multi-GPU design is described in DESIGN.md, not run)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2501_11673_amd as kpp
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    s, lam, tol = 128, 1e-8, 1e-10
    sysm = synth.config("c2", device="cuda")
    A, b = sysm.A, sysm.b
    n = A.shape[0]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ctx = kpp.kpp_context_create(0, stream.cuda_stream)
    h = kpp.kpp_system_create(ctx, kpp.KPP_CD_PSD, n, n, A.data_ptr(), n, b.data_ptr())
    p = kpp.kpp_params_default(kpp.KPP_CD_PSD)
    p.block_size = s
    p.lambda_ = lam
    p.tol = tol
    p.memo = kpp.KPP_MEMO_ONLINE
    p.max_iters = 200_000
    p.seed = args.seed
    p.keep_memo = 0
    p.engine = args.engine
    p.team_groups = args.team_groups
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    if args.rht_only:
        rec = {"rht": rht_transforms(kpp, torch, dev, ctx, A, b, reps=args.steps)}
        if args.calibrate_copy > 0:
            src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device=dev).fill_(1)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            rec["copy_calibration_bytes"] = args.calibrate_copy << 20
        print(json.dumps(rec), flush=True)
        kpp.kpp_system_destroy(h)
        kpp.kpp_context_destroy(ctx)
        return

    def one():
        x.zero_()
        st, res = kpp.kpp_solve(h, p, x.data_ptr())
        return st, res

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(one())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    iters = sum(r.iters for _, r in results)
    conv = all(st == kpp.KPP_OK and r.converged for st, r in results)
    ktime = sum(r.kernel_seconds for _, r in results)
    klaunch = sum(r.kernel_launches for _, r in results)
    bytes_alg = sum(r.bytes_algorithmic for _, r in results)
    xs = x.cpu().numpy()
    err_vs_xstar = float(np.linalg.norm(xs - sysm.xstar.cpu().numpy()) / np.linalg.norm(sysm.xstar.cpu().numpy()))
    last = results[-1][1]
    engine_name = {1: "one launch per phase (block gemv kernel)", 2: "fused persistent step kernel"}[last.engine_used]
    per_launch_bytes = bytes_alg / max(klaunch, 1)
    per_launch_s = ktime / max(klaunch, 1)
    achieved = per_launch_bytes / per_launch_s / 1e9 if per_launch_s > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic("k_fused<1, 2, double>") if last.engine_used == 2 else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": engine_name, "launches": int(klaunch),
                "avg_launch_us": round(per_launch_s * 1e6, 3),
                "bytes_per_launch": round(per_launch_bytes, 1)}

    line = {
        "metric": "block-iters/s (CD++ n=4096 SPD, time to true 1e-10 relative residual)",
        "value": iters / elapsed,
        "unit": "block-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded outlier-spectrum SPD system, generated on device)",
        "config": {"workload": "cdpp_spd_n4096_s128_online_memo_fp64", "n": n, "block": s,
                   "lambda": lam, "tol": tol, "memo": "online", "precision": "fp64",
                   "engine": last.engine_used},
        "time_to_tol_ms": 1e3 * elapsed / args.steps,
        "iters_per_solve": iters / args.steps,
        "converged": conv,
        "true_rel_res": last.true_rel_res,
        "rel_err_vs_planted": err_vs_xstar,
        "factorizations_per_solve": last.memo_misses,
        "factor_ms_per_solve": 1e3 * last.seconds_factor,
        "kernel_ms_per_solve": 1e3 * ktime / args.steps,
        "roofline": roofline,
    }
    if args.calibrate_copy > 0:
        src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = args.calibrate_copy << 20
        del src, dst
    # the same workload with mixed precision (FP32 block products, FP64 refinement)
    x_fp64 = x.clone()
    pm = kpp.kpp_params_default(kpp.KPP_CD_PSD)
    for f, _ in kpp.kpp_params._fields_:
        setattr(pm, f, getattr(p, f))
    pm.precision = kpp.KPP_MIXED_FP32
    pm.engine = 0

    def one_mixed():
        x.zero_()
        return kpp.kpp_solve(h, pm, x.data_ptr())

    for _ in range(args.warmup if not args.no_mixed else 0):
        one_mixed()
    torch.cuda.synchronize()
    mres = []
    t0 = time.perf_counter()
    for _ in range(args.steps if not args.no_mixed else 0):
        mres.append(one_mixed())
    torch.cuda.synchronize()
    melapsed = time.perf_counter() - t0
    miters = sum(r.iters for _, r in mres)
    mlast = mres[-1][1] if mres else None
    line["mixed"] = None if not mres else {
        "time_to_tol_ms": 1e3 * melapsed / args.steps,
        "block_iters_per_s": miters / melapsed,
        "iters_per_solve": miters / args.steps,
        "refinements": mlast.refinements,
        "converged": all(st == kpp.KPP_OK and r.converged for st, r in mres),
        "true_rel_res": mlast.true_rel_res,
        "rel_diff_vs_fp64_solution": float(torch.linalg.norm(x - x_fp64) / torch.linalg.norm(x_fp64)),
        "rel_err_vs_planted": float(torch.linalg.norm(x - sysm.xstar) / torch.linalg.norm(sysm.xstar)),
        "factorizations_per_solve": mlast.memo_misses,
        "factors_redone_fp64": mlast.factors_fp64,
        "kernel_ms_per_solve": 1e3 * sum(r.kernel_seconds for _, r in mres) / args.steps,
        "speedup_vs_fp64": (1e3 * elapsed / args.steps) / (1e3 * melapsed / args.steps),
    }
    if not args.no_multi:
        line["multi_rhs"] = multi_rhs(kpp, torch, dev, ctx, h, A, n, p)
    if not args.no_rht:
        rh = rht_transforms(kpp, torch, dev, ctx, A, b)
        rh["cdpp_n4096_with_rht"] = rht_solves(kpp, torch, dev, h, p, x, args.steps)
        line["rht"] = rh
    if not args.no_flops:
        line["flops_to_tol"] = flops_to_tol(kpp, torch, dev, ctx, args.seed)
    if not args.no_lsqr:
        line["lsqr"] = lsqr_solves(kpp, torch, dev, ctx)
    if not args.no_flops:
        line["ablation"] = ablation(kpp, torch, dev, ctx)
    kpp.kpp_system_destroy(h)
    kpp.kpp_context_destroy(ctx)
    if not args.no_serving:
        line["serving"] = serving(kpp, torch, dev, args.serve_requests)
    if not args.no_cpu_baseline:
        Ah = A.cpu().numpy()
        bh = b.cpu().numpy()
        del A, b
        line["cpu_baseline"] = cpu_baseline(Ah, bh, s, lam, tol, args.seed)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
