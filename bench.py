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
FP64 factors and iterative refinement) and reported under "mixed".

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
    return ap.parse_args()


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
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
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

    for _ in range(args.warmup):
        one_mixed()
    torch.cuda.synchronize()
    mres = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mres.append(one_mixed())
    torch.cuda.synchronize()
    melapsed = time.perf_counter() - t0
    miters = sum(r.iters for _, r in mres)
    mlast = mres[-1][1]
    line["mixed"] = {
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
    kpp.kpp_system_destroy(h)
    kpp.kpp_context_destroy(ctx)
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
