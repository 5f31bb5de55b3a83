"""Benchmark: time to a true 1e-10 relative residual and block-iterations/s,
FP64 vs mixed precision, on the Kaczmarz++ and CD++ workloads.

Headline workload: Kaczmarz++ (Algorithm 5 with the exact memoized Cholesky
projection) on the under-determined 2048 x 32768 system A = U diag(sigma) V^T
(U, V Haar; sigma: 20 outliers log-spaced in [1e3, 1e4], 2028 uniform in
[0.5, 1]; x* = V g in the row space, b = A x*); block size 128, lambda 1e-4,
online block memoization (Section 5.2), FP64, tolerance 1e-10 on
||A x - b|| / ||b|| confirmed in FP64.  One "step" is one full solve from
x0 = 0 with an empty memo cache (every Gram and factorization is paid inside
the timed region).  value = block steps per second over the timed solves;
ms_per_step = time to tolerance per solve.  Inputs are synthetic and seeded
and are resident in HBM before the timed region.

Under "mixed": the same solves with mixed precision (FP32 block products,
FP64 factors, FP64 iterative refinement, the library's default inner
tolerance), with the speed-up over FP64 and the error against the FP64
solution, and under "mixed"/"seeds" FP64 and mixed on the same system for two
further schedule seeds (the step count to tolerance of either depends on the
seed) with the means over the three; under "bf16" one solve with bfloat16
storage of A (reported whether or not it converges), and under
"precisions_well_conditioned" FP64, FP32 and bfloat16 on a kappa = 10 system
of the headline's shape.  Under "kpp_65536x2048": the over-determined
65536 x 2048 workload (block 256, fixed partition into 256 blocks), FP64 and
mixed.  Under "cdpp_n4096": CD++ (Algorithm 2) on the n = 4096 SPD workload,
FP64 and mixed.  Also: serving (continuous batching of 512 CD++ solves at
200/s, p50/p99 latency), the randomized Hadamard preprocessing, the paper's
FLOP comparison on synthetic kernel matrices (Full CD++, w/o RHT, w/o Memo),
the regularization sweep, Kaczmarz++ with the LSQR projection (t_max 2, 4, 8),
the ablation table, several right-hand sides, and sparse (CSR) systems
(Kaczmarz++ on a random 262144 x 65536 matrix, CD++ on a random-graph
Laplacian of order 65536: team kernel vs three launches per step, bytes per
step against the SpMV roofline).

Each measured solve carries the roofline of its step kernel (algorithmic bytes
per launch over the launch time from HIP events inside the library, on the
stream the kernel runs on) and the CPU oracle is timed on the host on the
headline workload.
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
    ap.add_argument("--seed", type=int, default=202, help="seed of the kernel-matrix sections")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB three times (HBM counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--no-rht", action="store_true")
    ap.add_argument("--no-flops", action="store_true")
    ap.add_argument("--no-lsqr", action="store_true")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--host-generated", action="store_true",
                    help="draw the headline system with numpy on the host (for counter-profiler runs)")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--only", choices=["c2", "c3", "c4", "sparse_kpp", "sparse_cd"], default=None,
                    help="only one workload, FP64 and mixed: c2 (CD++ n=4096), c3 (65536 x 2048), c4 (2048 x 32768)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline workload, FP64 and mixed (for profiling the step kernel)")
    ap.add_argument("--rht-only", action="store_true",
                    help="only the randomized Hadamard transforms (for profiling them)")
    return ap.parse_args()


# rocprofv3 summaries whose FETCH_SIZE / WRITE_SIZE passes give the step
# kernel's HBM traffic per launch (by workload)
TRAFFIC_PROFILES = {
    "kpp_2048x32768": os.path.join(ROOT, "profiles", "k_fused_kpp_2048x32768_s128_fp64.md"),
    "kpp_65536x2048": os.path.join(ROOT, "profiles", "k_fused_kpp_65536x2048_s256_fp64.md"),
    "cdpp_n4096": os.path.join(ROOT, "profiles", "k_fused_cdpp_n4096_s128_fp64.md"),
    "sparse_kpp": os.path.join(ROOT, "profiles", "k_sparse_team_kpp_262144x65536_d16_s128.md"),
    "sparse_cd": os.path.join(ROOT, "profiles", "k_sparse_team_cdpp_n65536_d6_s128.md"),
}

# Sparse workloads (CSR; the paper's sparse setting): Kaczmarz++ on a random
# 262144 x 65536 matrix with 16 uniform columns per row (N(0, 1) values, 2% of
# the rows scaled by 10), CD++ on a random-graph Laplacian + 0.1 I of order
# 65536 (6 partners per node, 4 hubs of 120 more); block 128, online memo.
SPARSE_WORKLOADS = {
    "sparse_kpp": dict(kind="general", m=262144, n=65536, per_row=16, seed=71, s=128, lam=1e-6, tol=1e-10),
    "sparse_cd": dict(kind="psd", m=65536, n=65536, degree=6, seed=72, s=128, lam=1e-8, tol=1e-8),
}


def measured_traffic(profile, kernel_name):
    """HBM bytes per launch of the step kernel from a committed rocprofv3
    FETCH_SIZE / WRITE_SIZE pass, each scaled by what the counter read for a
    device copy of known size.  None when the kernel's sources have changed
    since the counters were taken, or for another kernel."""
    import hashlib
    import re
    try:
        text = open(profile).read()
    except (OSError, TypeError):
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


def step_kernel_name(kind, cpl, fp32):
    return f"k_fused<{0 if kind == 'general' else 1}, {cpl}, {'float' if fp32 else 'double'}>"


def roofline(results, kind, profile=None):
    """Roofline of the step kernel over a set of solves: algorithmic bytes per
    launch (the library's count) over the average launch time from HIP events
    on the library's stream, against the HBM peak."""
    ktime = sum(r.kernel_seconds for _, r in results)
    klaunch = sum(r.kernel_launches for _, r in results)
    bytes_alg = sum(r.bytes_algorithmic for _, r in results)
    last = results[-1][1]
    per_launch_bytes = bytes_alg / max(klaunch, 1)
    per_launch_s = ktime / max(klaunch, 1)
    achieved = per_launch_bytes / per_launch_s / 1e9 if per_launch_s > 0 else 0.0
    fp32 = last.cols_per_lane > 0 and getattr(last, "refinements", 0) > 0
    name = step_kernel_name(kind, last.cols_per_lane, fp32) if last.engine_used == 2 else "launch-per-phase engine"
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": measured_traffic(profile, name) if (profile and last.engine_used == 2 and not fp32) else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": name, "team_groups": last.team_groups, "cols_per_lane": last.cols_per_lane,
            "launches": int(klaunch), "avg_launch_us": round(per_launch_s * 1e6, 3),
            "bytes_per_launch": round(per_launch_bytes, 1),
            "us_per_step_in_kernel": round(1e6 * ktime / max(sum(r.iters for _, r in results), 1), 3)}


def timed_solves(kpp, torch, h, p, x, warmup, steps):
    """warmup untimed solves, then steps timed ones, each from x0 = 0."""
    for _ in range(warmup):
        x.zero_()
        kpp.kpp_solve(h, p, x.data_ptr())
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        results.append(kpp.kpp_solve(h, p, x.data_ptr()))
    torch.cuda.synchronize()
    return results, time.perf_counter() - t0


def timed_and_launch_timed(kpp, torch, h, p, x, warmup, steps):
    """The time-to-tolerance solves without per-launch HIP events (each event
    pair adds a few microseconds between two launches), then the same solves
    with them, for the step kernel's launch durations (the roofline).  The
    first set's time is the solve time; the iterates are the same."""
    q = copy_params(kpp, None, p)
    q.no_launch_timing = 1
    res, el = timed_solves(kpp, torch, h, q, x, warmup, steps)
    q.no_launch_timing = 0
    tres, _ = timed_solves(kpp, torch, h, q, x, 0, steps)
    return res, el, tres


def solve_record(torch, results, elapsed, steps, x, xstar, kind, profile=None, x_ref=None, timing=None):
    """timing: the same solves run with per-launch HIP events (kernel time and
    roofline); default: results carry them."""
    timing = timing if timing is not None else results
    iters = sum(r.iters for _, r in results)
    last = results[-1][1]
    rec = {"time_to_tol_ms": 1e3 * elapsed / steps, "block_iters_per_s": iters / elapsed,
           "iters_per_solve": iters / steps,
           "converged": all(st == 0 and r.converged for st, r in results),
           "true_rel_res": last.true_rel_res,
           "factorizations_per_solve": last.memo_misses, "factors_fp64": last.factors_fp64,
           "refinements": last.refinements,
           "factor_ms_per_solve": 1e3 * last.seconds_factor,
           "kernel_ms_per_solve": 1e3 * sum(r.kernel_seconds for _, r in timing) / len(timing),
           "engine": last.engine_used,
           "rel_err_vs_planted": float(torch.linalg.norm(x - xstar) / torch.linalg.norm(xstar)),
           "roofline": roofline(timing, kind, profile)}
    if x_ref is not None:
        rec["rel_diff_vs_fp64_solution"] = float(torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref))
    return rec


def copy_params(kpp, kind, p):
    q = kpp.kpp_params_default(kind if kind is not None else kpp.KPP_KACZMARZ)
    for f, _ in kpp.kpp_params._fields_:
        setattr(q, f, getattr(p, f))
    return q


def fp64_and_mixed(kpp, torch, dev, ctx, name, warmup, steps, profile=None, engine=0, host_data=False, bf16=False):
    """One workload (synth config `name`): FP64 solves, then mixed precision.
    host_data: draw the system with numpy on the host and copy it to the device
    (same recipe, another random stream; for runs under a counter profiler)."""
    import synth

    if host_data:
        sysm = synth.config(name)
        sysm.A = torch.from_numpy(sysm.A).to(dev)
        sysm.b = torch.from_numpy(sysm.b).to(dev)
        sysm.xstar = torch.from_numpy(sysm.xstar).to(dev)
    else:
        sysm = synth.config(name, device="cuda")
    cfg = synth.CONFIGS[name]
    A, b = sysm.A, sysm.b
    m, n = A.shape
    kind = kpp.KPP_CD_PSD if cfg["kind"] == "psd" else kpp.KPP_KACZMARZ
    h = kpp.kpp_system_create(ctx, kind, m, n, A.data_ptr(), n, b.data_ptr())
    p = kpp.kpp_params_default(kind)
    p.block_size = cfg["s"]
    p.lambda_ = cfg["lam"]
    p.tol = 1e-10
    p.memo = kpp.KPP_MEMO_FIXED if cfg["memo"] == "fixed" and name != "c2" else kpp.KPP_MEMO_ONLINE
    p.fixed_partition = 1
    p.max_iters = 200_000
    p.seed = cfg["schedule_seed"]
    p.keep_memo = 0
    p.engine = engine
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    res64, el64, t64 = timed_and_launch_timed(kpp, torch, h, p, x, warmup, steps)
    rec = solve_record(torch, res64, el64, steps, x, sysm.xstar, cfg["kind"], profile, timing=t64)
    x64 = x.clone()
    pm = copy_params(kpp, kind, p)
    pm.precision = kpp.KPP_MIXED_FP32
    pm.engine = 0
    resm, elm, tm = timed_and_launch_timed(kpp, torch, h, pm, x, warmup, steps)
    mixed = solve_record(torch, resm, elm, steps, x, sysm.xstar, cfg["kind"], None, x64, timing=tm)
    mixed["speedup_vs_fp64"] = rec["time_to_tol_ms"] / mixed["time_to_tol_ms"]
    rec["mixed"] = mixed
    if bf16:
        # bfloat16 storage of A: one solve, reported whether or not it converges
        pb = copy_params(kpp, kind, pm)
        pb.precision = kpp.KPP_MIXED_BF16
        resb, elb = timed_solves(kpp, torch, h, pb, x, 0, 1)
        rb = resb[-1][1]
        rec["bf16"] = {"converged": bool(resb[-1][0] == kpp.KPP_OK and rb.converged),
                       "true_rel_res": rb.true_rel_res, "refinements": rb.refinements, "iters": rb.iters,
                       "time_ms": 1e3 * elb,
                       "note": "a diverging refinement ends early and returns the iterate with the lowest true "
                               "residual (kappa(A) 2^-8 >= 1 on this system)"}
    rec["workload"] = {"name": name, "m": m, "n": n, "block": cfg["s"], "lambda": cfg["lam"],
                       "memo": "fixed partition" if p.memo == kpp.KPP_MEMO_FIXED else "online", "tol": 1e-10}
    return rec, (sysm, h, p, x64)


def seed_comparison(kpp, torch, h, p, x, head, seeds=(11, 12345), reps=2):
    """FP64 against mixed precision on the headline system for further
    schedule seeds (the step count to 1e-10 of either depends on the seed):
    time to tolerance per seed (mean of `reps` timed solves after one warm-up)
    and the means over these seeds and the headline's."""
    rows = [{"seed": int(p.seed), "fp64_ms": head["time_to_tol_ms"], "mixed_ms": head["mixed"]["time_to_tol_ms"],
             "fp64_iters": head["iters_per_solve"], "mixed_iters": head["mixed"]["iters_per_solve"]}]
    for sd in seeds:
        row = {"seed": sd}
        for tag, prec in (("fp64", kpp.KPP_FP64), ("mixed", kpp.KPP_MIXED_FP32)):
            q = copy_params(kpp, None, p)
            q.seed = sd
            q.precision = prec
            q.engine = 0
            q.no_launch_timing = 1
            results, elapsed = timed_solves(kpp, torch, h, q, x, 1, reps)
            row[f"{tag}_ms"] = 1e3 * elapsed / reps
            row[f"{tag}_iters"] = results[-1][1].iters
            row[f"{tag}_converged"] = all(st == kpp.KPP_OK and r.converged for st, r in results)
        rows.append(row)
    f = sum(r["fp64_ms"] for r in rows) / len(rows)
    mx = sum(r["mixed_ms"] for r in rows) / len(rows)
    return {"per_seed": rows, "fp64_mean_ms": f, "mixed_mean_ms": mx, "speedup_of_means": f / mx,
            "inner_tol": p.inner_tol}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        n = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:  # pragma: no cover
        return 1


def cpu_info():
    """CPU model and core counts of the host the oracle runs on."""
    model, phys = "unknown", set()
    try:
        cur = {}
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if cur.get("physical id") is not None and cur.get("core id") is not None:
                    phys.add((cur["physical id"], cur["core id"]))
                cur = {}
                continue
            k, v = [x.strip() for x in line.split(":", 1)]
            cur[k] = v
            if k == "model name":
                model = v
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "physical_cores": len(phys) or None, "usable_cpus": usable}


def cpu_baseline(A, b, s, lam, tol, seed, single_thread_steps=96):
    """The oracle as it stands on the headline workload: one full Kaczmarz++
    solve to tol with the BLAS threads of the host, and the first
    single_thread_steps block steps of the same solve on one thread."""
    from oracle import kpp as okpp
    from oracle import schedule as osch

    m, n = A.shape
    T = 100_000
    schd = osch.make_schedule("online", m, s, T, seed, B0=osch.online_rate("general", m, n, s))
    t0 = time.perf_counter()
    res = okpp.solve(A, b, "general", okpp.Params(s=s, lam=lam, tol=tol, max_iters=T), schd)
    dt = time.perf_counter() - t0
    one = None
    try:
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            r1 = okpp.solve(A, b, "general", okpp.Params(s=s, lam=lam, tol=0.0, max_iters=single_thread_steps), schd)
            d1 = time.perf_counter() - t1
        one = {"block_iters_per_s": r1.iters / d1, "steps": r1.iters, "seconds": d1,
               "sample": f"the first {r1.iters} block steps of the same solve (every new block's Gram "
                         f"and Cholesky factor included), BLAS on one thread"}
    except Exception as e:  # pragma: no cover
        one = {"error": str(e)}
    rec = {"value": res.iters / dt, "unit": "block-iters/s", "cores": blas_threads(),
           "kind": "oracle",
           "sample": f"one full Kaczmarz++ solve of the 2048 x 32768 system to {tol:g} "
                     f"({res.iters} block steps, {res.factorizations} factorizations, {dt:.2f} s, "
                     f"converged={res.converged}); cores = BLAS threads used",
           "time_to_tol_s": dt, "single_thread": one}
    rec.update(cpu_info())
    return rec


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


def flops_to_tol(kpp, torch, dev, ctx, seed, seeds=3):
    """The paper's FLOP comparison (Section 6.3, Table tab:flops) on synthetic
    data: Full CD++ (with RHT), CD++ w/o RHT and CD++ w/o Memo (with RHT, a new
    block and factor every step) on Gaussian and Laplacian kernel matrices
    (gamma 0.1 and 0.01) of n = 4096 seeded points plus 1e-3 I, b ~ N(0, I),
    s = 200, lambda = 1e-8; FLOPs counted as the paper counts them
    (kpp_result.flops, RHT included), averaged over `seeds` schedule and sign
    seeds, next to the range of the paper's own numbers over its 20 matrices
    (other data, no hardware stated)."""
    import synth

    rows = []
    n, s = 4096, 200
    methods = (("full_cdpp", 1, kpp.KPP_MEMO_ONLINE), ("cdpp_wo_rht", 0, kpp.KPP_MEMO_ONLINE),
               ("cdpp_wo_memo", 1, kpp.KPP_MEMO_OFF))
    for kern in ("gaussian", "laplacian"):
        for gamma in (0.1, 0.01):
            sysm = synth.kernel_system(kern, n, gamma, seed=seed, device="cuda")
            h = kpp.kpp_system_create(ctx, kpp.KPP_CD_PSD, n, n, sysm.A.data_ptr(), n, sysm.b.data_ptr())
            for method, rht, memo in methods:
                for tol in (1e-4, 1e-8):
                    runs = []
                    for k in range(seeds):
                        p = kpp.kpp_params_default(kpp.KPP_CD_PSD)
                        p.block_size = s
                        p.lambda_ = 1e-8
                        p.tol = tol
                        p.max_iters = 400_000
                        p.memo = memo
                        p.seed = seed + 7919 * k
                        p.rht = rht
                        p.rht_seed = seed + 1 + 7919 * k
                        x = torch.zeros(n, dtype=torch.float64, device=dev)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        st, r = kpp.kpp_solve(h, p, x.data_ptr())
                        torch.cuda.synchronize()
                        runs.append((r.flops, r.iters, time.perf_counter() - t0,
                                     bool(st == kpp.KPP_OK and r.converged), r.true_rel_res))
                    rows.append({"matrix": f"{kern} gamma={gamma:g}", "method": method, "tol": tol,
                                 "flops": sum(v[0] for v in runs) / seeds,
                                 "iters": sum(v[1] for v in runs) / seeds,
                                 "ms": round(1e3 * sum(v[2] for v in runs) / seeds, 3),
                                 "runs": seeds, "converged": all(v[3] for v in runs),
                                 "max_true_rel_res": max(v[4] for v in runs)})
            kpp.kpp_system_destroy(h)
            del sysm
    return {"workload": "CD++ on n=4096 kernel matrices + 1e-3 I (seeded Gaussian points, d=8), s=200, "
                        "lambda=1e-8; b ~ N(0, I); averages over %d seeds" % seeds,
            "runs": rows, "paper_tab_flops_range": PAPER_TAB_FLOPS}


def lambda_sweep(kpp, torch, dev, ctx, seed):
    """Regularization in the projection (the appendix's test of lambda on Full
    CD++): lambda in {1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 0} on the Gaussian kernel
    matrix (gamma 0.1) and the n = 4096 outlier SPD workload, s = 200, RHT,
    online memo, tolerance 1e-8: steps, FLOPs and time to tolerance."""
    import synth

    out = {}
    n, s = 4096, 200
    for name in ("gaussian_0.1", "spd_outliers_n4096"):
        if name.startswith("gaussian"):
            sysm = synth.kernel_system("gaussian", n, 0.1, seed=seed, device="cuda")
        else:
            sysm = synth.config("c2", device="cuda")
        h = kpp.kpp_system_create(ctx, kpp.KPP_CD_PSD, n, n, sysm.A.data_ptr(), n, sysm.b.data_ptr())
        rec = []
        for lam in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 0.0):
            p = kpp.kpp_params_default(kpp.KPP_CD_PSD)
            p.block_size = s
            p.lambda_ = lam
            p.tol = 1e-8
            p.max_iters = 400_000
            p.seed = seed
            p.rht = 1
            p.rht_seed = seed + 1
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, r = kpp.kpp_solve(h, p, x.data_ptr())
            torch.cuda.synchronize()
            rec.append({"lambda": lam, "iters": r.iters, "flops": r.flops,
                        "ms": round(1e3 * (time.perf_counter() - t0), 3),
                        "converged": bool(st == kpp.KPP_OK and r.converged), "true_rel_res": r.true_rel_res})
        kpp.kpp_system_destroy(h)
        out[name] = rec
        del sysm
    return out


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
    factor) and with the sketch-preconditioned LSQR projection (tau = 2s;
    Section 4.1): t_max in {2, 4, 8} on the 1000 x 200 workload ("K++(LSQR-t)"
    of the appendix), t_max = 8 on 65536 x 2048."""
    import synth

    out = {}
    for name, cfg, s, lam, memo, tmaxs in (("k_1000x200_s20", "c1", 20, 1e-3, 1, (2, 4, 8)),
                                            ("k_65536x2048_s256", "c3", 256, 1e-8, 2, (8,))):
        sysm = synth.config(cfg, device="cuda")
        A, b = sysm.A, sysm.b
        m, n = A.shape
        h = kpp.kpp_system_create(ctx, kpp.KPP_KACZMARZ, m, n, A.data_ptr(), n, b.data_ptr())
        rec = {}
        for proj, tmax in [(kpp.KPP_PROJ_EXACT, 0)] + [(kpp.KPP_PROJ_LSQR, t) for t in tmaxs]:
            p = kpp.kpp_params_default(kpp.KPP_KACZMARZ)
            p.block_size = s
            p.lambda_ = lam
            p.tol = 1e-10
            p.memo = memo
            p.fixed_partition = 1
            p.max_iters = 50_000 if proj == kpp.KPP_PROJ_LSQR and tmax < 8 else 200_000
            p.seed = sysm.params["schedule_seed"]
            p.projection = proj
            if proj == kpp.KPP_PROJ_LSQR:
                p.lsqr_iters = tmax
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, r = kpp.kpp_solve(h, p, x.data_ptr())
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec["exact" if proj == 0 else f"lsqr_t{tmax}"] = {
                "time_to_tol_ms": round(1e3 * dt, 3), "iters": r.iters, "us_per_step": round(1e6 * dt / max(r.iters, 1), 2),
                "flops": r.flops, "converged": bool(st == kpp.KPP_OK and r.converged), "true_rel_res": r.true_rel_res,
                "engine": r.engine_used,
                "rel_err_vs_planted": float(torch.linalg.norm(x - sysm.xstar) / torch.linalg.norm(sysm.xstar))}
        kpp.kpp_system_destroy(h)
        out[name] = rec
        del sysm, A, b
    return out


def precisions_well_conditioned(kpp, torch, dev, ctx, reps=3):
    """FP64, FP32 and bfloat16 storage of A on a well-conditioned system of
    the headline's shape (2048 x 32768, singular values log-spaced in [1, 10],
    x* in the row space), block 128, lambda 1e-4, online memo, to 1e-10."""
    import numpy as np

    import synth

    sysm = synth.svd_system(2048, 32768, lambda rng, r: np.geomspace(1.0, 10.0, r), 91, x_in_rowspace=True,
                            device="cuda", name="kpp_2048x32768_kappa10")
    A, b = sysm.A, sysm.b
    m, n = A.shape
    h = kpp.kpp_system_create(ctx, kpp.KPP_KACZMARZ, m, n, A.data_ptr(), n, b.data_ptr())
    out = {"workload": {"m": m, "n": n, "kappa": 10.0, "block": 128, "lambda": 1e-4, "tol": 1e-10,
                        "memo": "online"}}
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    for name, prec in (("fp64", kpp.KPP_FP64), ("mixed_fp32", kpp.KPP_MIXED_FP32), ("mixed_bf16", kpp.KPP_MIXED_BF16)):
        p = kpp.kpp_params_default(kpp.KPP_KACZMARZ)
        p.block_size = 128
        p.lambda_ = 1e-4
        p.tol = 1e-10
        p.max_iters = 200_000
        p.seed = 5
        p.precision = prec
        results, elapsed = timed_solves(kpp, torch, h, p, x, 1, reps)
        last = results[-1][1]
        out[name] = {"time_to_tol_ms": 1e3 * elapsed / reps, "iters": last.iters, "refinements": last.refinements,
                     "converged": all(st == kpp.KPP_OK and r.converged for st, r in results),
                     "true_rel_res": last.true_rel_res,
                     "us_per_step_in_kernel": round(1e6 * last.kernel_seconds / max(last.iters, 1), 3),
                     "rel_err_vs_planted": float(torch.linalg.norm(x - sysm.xstar) / torch.linalg.norm(sysm.xstar))}
    kpp.kpp_system_destroy(h)
    del sysm, A, b
    torch.cuda.empty_cache()
    return out


def sparse_solves(kpp, torch, dev, ctx, names, reps=1, engines=(2, 1)):
    """Sparse systems to tolerance: the team kernel (engine 2: one launch per
    window, workgroups owning column slices of x) and three launches per step
    (engine 1).  Bytes per step are the library's count (block rows with
    their nonzeros and gathered iterate entries, G^{-1}, the column-compressed
    copy with every nonzero's column counted as distinct, u and v on the
    updated columns, the folds); the SpMV roofline is that traffic at the HBM
    peak."""
    import synth

    out = {}
    for name in names:
        w = SPARSE_WORKLOADS[name]
        if w["kind"] == "general":
            S = synth.sparse_general(w["m"], w["n"], w["per_row"], seed=w["seed"])
            kind = kpp.KPP_KACZMARZ
        else:
            S = synth.sparse_psd(w["n"], w["degree"], seed=w["seed"])
            kind = kpp.KPP_CD_PSD
        rp, ci, cv, b = S.to(dev)
        xs = torch.from_numpy(S.xstar).to(dev)
        h = kpp.kpp_system_create_csr(ctx, kind, S.m, S.n, S.nnz, rp.data_ptr(), ci.data_ptr(), cv.data_ptr(),
                                      b.data_ptr())
        rec = {"workload": {"m": S.m, "n": S.n, "nnz": S.nnz, "block": w["s"], "lambda": w["lam"], "tol": w["tol"],
                            "memo": "online", "recipe": {k: v for k, v in S.params.items()}}}
        for engine in engines:
            p = kpp.kpp_params_default(kind)
            p.block_size = w["s"]
            p.lambda_ = w["lam"]
            p.tol = w["tol"]
            p.max_iters = 1_000_000
            p.seed = 11
            p.engine = engine
            x = torch.zeros(S.n, dtype=torch.float64, device=dev)
            results, elapsed = timed_solves(kpp, torch, h, p, x, 1 if engine == 2 else 0, reps)
            last = results[-1][1]
            iters = sum(r.iters for _, r in results)
            ksec = sum(r.kernel_seconds for _, r in results)
            bytes_step = sum(r.bytes_algorithmic for _, r in results) / max(iters, 1)
            us_step = 1e6 * ksec / max(iters, 1)
            achieved = bytes_step / (us_step * 1e3) if us_step > 0 else 0.0
            e = {"time_to_tol_ms": 1e3 * elapsed / reps, "block_iters_per_s": iters / elapsed,
                 "iters_per_solve": iters / reps, "us_per_step_in_kernel": round(us_step, 3),
                 "converged": all(st == 0 and r.converged for st, r in results),
                 "true_rel_res": last.true_rel_res,
                 "rel_err_vs_planted": float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs)),
                 "factorizations_per_solve": last.memo_misses, "factor_ms_per_solve": 1e3 * last.seconds_factor,
                 "engine": last.engine_used, "launches_per_solve": last.kernel_launches,
                 "bytes_per_step": round(bytes_step, 1),
                 "spmv_roofline_us_per_step": round(bytes_step / (HBM_PEAK_GBS * 1e3), 4)}
            if engine == 2:
                kname = f"k_sparse_team<{0 if kind == kpp.KPP_KACZMARZ else 1}>"
                per_launch = bytes_step * iters / max(sum(r.kernel_launches for _, r in results), 1)
                e["roofline"] = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(achieved / HBM_PEAK_GBS, 6),
                                 "traffic": measured_traffic(TRAFFIC_PROFILES.get(name), kname),
                                 "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                                 "copy-calibrated)",
                                 "kernel": kname, "bytes_per_launch": round(per_launch, 1)}
                rec["team"] = e
            else:
                rec["launch_per_phase"] = e
        if "team" in rec and "launch_per_phase" in rec:
            rec["team"]["speedup_vs_launch_per_phase"] = (rec["launch_per_phase"]["time_to_tol_ms"] /
                                                          rec["team"]["time_to_tol_ms"])
        kpp.kpp_system_destroy(h)
        out[name] = rec
        del S, rp, ci, cv, b, xs
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 "
              "(the multi-GPU design is described in DESIGN.md, not run)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2501_11673_amd as kpp
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ctx = kpp.kpp_context_create(0, stream.cuda_stream)
    if args.rht_only:
        sysm = synth.config("c2", device="cuda")
        rec = {"rht": rht_transforms(kpp, torch, dev, ctx, sysm.A, sysm.b, reps=args.steps)}
        if args.calibrate_copy > 0:
            src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device=dev).fill_(1)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            rec["copy_calibration_bytes"] = args.calibrate_copy << 20
        print(json.dumps(rec), flush=True)
        kpp.kpp_context_destroy(ctx)
        return

    if args.only in ("sparse_kpp", "sparse_cd"):
        rec = sparse_solves(kpp, torch, dev, ctx, [args.only], reps=max(1, args.steps), engines=(2,))
        kpp.kpp_context_destroy(ctx)
        if args.calibrate_copy > 0:
            src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device=dev).fill_(1)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            rec["copy_calibration_bytes"] = args.calibrate_copy << 20
        print(json.dumps({"only": args.only, **rec}), flush=True)
        return
    if args.only:
        # one workload's FP64 and mixed solves (the command the step kernel's
        # profile summaries are taken with)
        prof = {"c2": "cdpp_n4096", "c3": "kpp_65536x2048", "c4": "kpp_2048x32768"}[args.only]
        rec, (sysm, h, _, _) = fp64_and_mixed(kpp, torch, dev, ctx, args.only, args.warmup, args.steps,
                                              TRAFFIC_PROFILES[prof], host_data=args.host_generated)
        kpp.kpp_system_destroy(h)
        kpp.kpp_context_destroy(ctx)
        if args.calibrate_copy > 0:
            src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device=dev).fill_(1)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            rec["copy_calibration_bytes"] = args.calibrate_copy << 20
        print(json.dumps({"only": args.only, **rec}), flush=True)
        return

    # headline: Kaczmarz++ on 2048 x 32768, FP64, then mixed precision
    head, (c4, h4, p4, x4) = fp64_and_mixed(kpp, torch, dev, ctx, "c4", args.warmup, args.steps,
                                            TRAFFIC_PROFILES["kpp_2048x32768"], engine=args.engine,
                                            host_data=args.host_generated, bf16=not args.headline_only)
    line = {
        "metric": "block-iters/s (Kaczmarz++ 2048x32768, time to true 1e-10 relative residual; FP64 vs mixed)",
        "value": head["block_iters_per_s"],
        "unit": "block-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["time_to_tol_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded outlier-spectrum 2048 x 32768 system, generated on device)",
        "config": {"workload": "kpp_2048x32768_s128_online_fp64", "m": 2048, "n": 32768, "block": 128,
                   "lambda": 1e-4, "tol": 1e-10, "memo": "online", "precision": "fp64", "engine": head["engine"]},
    }
    for k in ("time_to_tol_ms", "iters_per_solve", "converged", "true_rel_res", "rel_err_vs_planted",
              "factorizations_per_solve", "factor_ms_per_solve", "kernel_ms_per_solve"):
        line[k] = head[k]
    line["roofline"] = head["roofline"]
    line["mixed"] = head["mixed"]
    if not args.headline_only:
        line["mixed"]["seeds"] = seed_comparison(kpp, torch, h4, p4, x4, head)
    if "bf16" in head:
        line["bf16"] = head["bf16"]
    if args.calibrate_copy > 0:
        src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = args.calibrate_copy << 20
        del src, dst
    A4h = b4h = None
    if not args.no_cpu_baseline:
        A4h, b4h = c4.A.cpu().numpy(), c4.b.cpu().numpy()
    kpp.kpp_system_destroy(h4)
    del c4, x4
    torch.cuda.empty_cache()
    if args.headline_only:
        line["cpu_baseline"] = None
        print(json.dumps(line), flush=True)
        kpp.kpp_context_destroy(ctx)
        return

    rec3, (c3, h3, _, _) = fp64_and_mixed(kpp, torch, dev, ctx, "c3", args.warmup, args.steps,
                                          TRAFFIC_PROFILES["kpp_65536x2048"])
    kpp.kpp_system_destroy(h3)
    del c3
    torch.cuda.empty_cache()
    line["kpp_65536x2048"] = rec3
    rec2, (c2, h2, p2, x2) = fp64_and_mixed(kpp, torch, dev, ctx, "c2", args.warmup, args.steps,
                                            TRAFFIC_PROFILES["cdpp_n4096"])
    line["cdpp_n4096"] = rec2
    if not args.no_multi:
        line["multi_rhs"] = multi_rhs(kpp, torch, dev, ctx, h2, c2.A, 4096, p2)
    if not args.no_rht:
        rh = rht_transforms(kpp, torch, dev, ctx, c2.A, c2.b)
        rh["cdpp_n4096_with_rht"] = rht_solves(kpp, torch, dev, h2, p2, x2, args.steps)
        line["rht"] = rh
    kpp.kpp_system_destroy(h2)
    del c2
    if not args.no_flops:
        line["flops_to_tol"] = flops_to_tol(kpp, torch, dev, ctx, args.seed)
        line["lambda_sweep"] = lambda_sweep(kpp, torch, dev, ctx, args.seed)
    if not args.no_lsqr:
        line["lsqr"] = lsqr_solves(kpp, torch, dev, ctx)
    if not args.no_flops:
        line["ablation"] = ablation(kpp, torch, dev, ctx)
    if not args.no_sparse:
        line["sparse"] = sparse_solves(kpp, torch, dev, ctx, ["sparse_kpp", "sparse_cd"])
    if not args.no_mixed:
        line["precisions_well_conditioned"] = precisions_well_conditioned(kpp, torch, dev, ctx)
    kpp.kpp_context_destroy(ctx)
    if not args.no_serving:
        line["serving"] = serving(kpp, torch, dev, args.serve_requests)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(A4h, b4h, 128, 1e-4, 1e-10, synth.CONFIGS["c4"]["schedule_seed"])
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
