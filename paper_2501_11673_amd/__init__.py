"""Python binding of libkpp (include/kpp.h): MI355X Kaczmarz++ / CD++ block step.

Argument marshalling only: every step of the solver runs in the HIP library.
The functions keep the C names.  Device buffers are passed as integer device
addresses (for example ``tensor.data_ptr()``); streams as ``hipStream_t``
handles (``torch.cuda.current_stream().cuda_stream``).  Import fails loudly if
the library has not been built (``python paper_2501_11673_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkpp.so")

KPP_OK = 0
KPP_NOT_CONVERGED = 1
KPP_ERR_INVALID_ARG = -1
KPP_ERR_SHAPE = -2
KPP_ERR_NOT_SPD = -3
KPP_ERR_NONFINITE = -4
KPP_ERR_OOM = -5
KPP_ERR_HIP = -6
KPP_ERR_REJECTED = -7
KPP_ERR_DEVICE = -8

KPP_KACZMARZ = 0
KPP_CD_PSD = 1

KPP_MEMO_OFF = 0
KPP_MEMO_ONLINE = 1
KPP_MEMO_FIXED = 2

KPP_FP64 = 0
KPP_MIXED_FP32 = 1
KPP_MIXED_BF16 = 2

KPP_ENGINE_AUTO = 0
KPP_ENGINE_LAUNCH = 1
KPP_ENGINE_FUSED = 2

KPP_PROJ_EXACT = 0
KPP_PROJ_LSQR = 1

_STATUS_NAMES = {v: k for k, v in globals().items() if k.startswith(("KPP_OK", "KPP_NOT", "KPP_ERR"))}


class kpp_params(ctypes.Structure):
    _fields_ = [
        ("block_size", ctypes.c_int32),
        ("memo", ctypes.c_int32),
        ("num_blocks", ctypes.c_int32),
        ("fixed_partition", ctypes.c_int32),
        ("accel", ctypes.c_int32),
        ("adaptive_rho", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("confirm_true_residual", ctypes.c_int32),
        ("lambda_", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("max_iters", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("keep_memo", ctypes.c_int32),
        ("refine_max_rounds", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("engine", ctypes.c_int32),
        ("team_groups", ctypes.c_int32),
        ("schedule", ctypes.c_void_p),
        ("schedule_len", ctypes.c_int64),
        ("block_rows", ctypes.c_void_p),
        ("block_rows_count", ctypes.c_int32),
        ("resume", ctypes.c_int32),
        ("rht", ctypes.c_int32),
        ("no_launch_timing", ctypes.c_int32),
        ("rht_seed", ctypes.c_uint64),
        ("projection", ctypes.c_int32),
        ("lsqr_iters", ctypes.c_int32),
        ("sketch_size", ctypes.c_int32),
        ("reserved3", ctypes.c_int32),
        ("sketch_seed", ctypes.c_uint64),
    ]


class kpp_result(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int64),
        ("memo_hits", ctypes.c_int64),
        ("memo_misses", ctypes.c_int64),
        ("factors_fp64", ctypes.c_int64),
        ("converged", ctypes.c_int32),
        ("refinements", ctypes.c_int32),
        ("checkpoints", ctypes.c_int32),
        ("engine_used", ctypes.c_int32),
        ("est_rel_res", ctypes.c_double),
        ("true_rel_res", ctypes.c_double),
        ("rho_final", ctypes.c_double),
        ("seconds_total", ctypes.c_double),
        ("seconds_factor", ctypes.c_double),
        ("flops", ctypes.c_double),
        ("bytes_algorithmic", ctypes.c_double),
        ("kernel_seconds", ctypes.c_double),
        ("kernel_launches", ctypes.c_double),
        ("seconds_queued", ctypes.c_double),
        ("team_groups", ctypes.c_int32),
        ("cols_per_lane", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KppError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class kpp_server_info(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("rejected", ctypes.c_int64),
        ("rounds", ctypes.c_int64),
        ("queued", ctypes.c_int32),
        ("active", ctypes.c_int32),
        ("peak_active", ctypes.c_int32),
        ("cu_budget", ctypes.c_int32),
        ("bytes_active", ctypes.c_uint64),
        ("peak_bytes", ctypes.c_uint64),
        ("busy_seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    # Device pointers and streams handed to the library come from torch, whose
    # wheel ships its own HIP runtime.  Loading torch first makes the
    # library's libamdhip64 dependency resolve to that same runtime instance
    # (two runtimes in one process do not share devices or streams).
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - the library also runs without torch
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python paper_2501_11673_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "kpp_abi_version": (i32, []),
        "kpp_last_error": (ctypes.c_char_p, []),
        "kpp_params_default": (i32, [P(kpp_params), i32]),
        "kpp_context_create": (i32, [i32, vp, P(vp)]),
        "kpp_context_destroy": (i32, [vp]),
        "kpp_system_create": (i32, [vp, i32, i64, i64, vp, i64, vp, P(vp)]),
        "kpp_system_create_csr": (i32, [vp, i32, i64, i64, i64, vp, vp, vp, vp, P(vp)]),
        "kpp_system_destroy": (i32, [vp]),
        "kpp_solve": (i32, [vp, P(kpp_params), vp, P(kpp_result)]),
        "kpp_schedule_generate": (i32, [i32, i64, i64, P(kpp_params), i64, P(i32), P(i32), P(i32),
                                        i32, P(i32)]),
        "kpp_block_factor": (i32, [vp, i32, f64, i32, P(i32), P(i32), vp]),
        "kpp_block_factor_noalloc": (i32, [vp, i32, f64, i32, P(i32), P(i32), vp]),
        "kpp_residual_norm": (i32, [vp, vp, P(f64)]),
        "kpp_request_footprint": (i32, [vp, P(kpp_params), P(ctypes.c_uint64)]),
        "kpp_server_create": (i32, [vp, ctypes.c_uint64, i32, P(vp)]),
        "kpp_server_submit": (i32, [vp, vp, P(kpp_params), vp, P(ctypes.c_uint64)]),
        "kpp_server_poll": (i32, [vp, i32, f64, P(ctypes.c_uint64), P(i32), P(kpp_result), P(i32)]),
        "kpp_server_stats": (i32, [vp, P(kpp_server_info)]),
        "kpp_server_destroy": (i32, [vp]),
        "kpp_state_export": (i32, [vp, vp, P(ctypes.c_size_t)]),
        "kpp_state_import": (i32, [vp, vp, ctypes.c_size_t]),
        "kpp_solve_multi": (i32, [vp, P(kpp_params), i32, vp, i64, vp, i64, P(kpp_result)]),
        "kpp_rht_signs": (i32, [ctypes.c_uint64, i64, P(ctypes.c_int8)]),
        "kpp_rht_general": (i32, [vp, i64, i64, vp, i64, vp, vp, i64, vp, i64, vp]),
        "kpp_rht_psd": (i32, [vp, i64, vp, i64, vp, vp, i64, vp, i64, vp, vp]),
        "kpp_rht_vector": (i32, [vp, i64, vp, vp, i64, vp, i32, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("kpp_abi_version", "kpp_last_error", "kpp_params_default", "kpp_context_create",
            "kpp_context_destroy", "kpp_system_create", "kpp_system_create_csr", "kpp_system_destroy", "kpp_solve",
            "kpp_schedule_generate", "kpp_block_factor", "kpp_block_factor_noalloc", "kpp_residual_norm", "kpp_request_footprint", "kpp_server_create",
            "kpp_server_submit", "kpp_server_poll", "kpp_server_stats", "kpp_server_destroy",
            "kpp_state_export", "kpp_state_import", "kpp_solve_multi", "kpp_rht_signs", "kpp_rht_general", "kpp_rht_psd",
            "kpp_rht_vector")


def _check(status):
    if status < 0:
        raise KppError(status, kpp_last_error())
    return status


def kpp_abi_version() -> int:
    return _lib.kpp_abi_version()


def kpp_last_error() -> str:
    return _lib.kpp_last_error().decode()


def kpp_params_default(kind: int) -> kpp_params:
    p = kpp_params()
    _check(_lib.kpp_params_default(ctypes.byref(p), kind))
    return p


def kpp_context_create(device: int = 0, hip_stream: int = 0) -> int:
    out = ctypes.c_void_p()
    _check(_lib.kpp_context_create(device, ctypes.c_void_p(hip_stream), ctypes.byref(out)))
    return out.value


def kpp_context_destroy(ctx: int) -> None:
    _check(_lib.kpp_context_destroy(ctypes.c_void_p(ctx)))


def kpp_system_create(ctx: int, kind: int, m: int, n: int, A_dev: int, lda: int, b_dev: int) -> int:
    out = ctypes.c_void_p()
    _check(_lib.kpp_system_create(ctypes.c_void_p(ctx), kind, m, n, ctypes.c_void_p(A_dev), lda,
                                  ctypes.c_void_p(b_dev), ctypes.byref(out)))
    return out.value


def kpp_system_create_csr(ctx: int, kind: int, m: int, n: int, nnz: int, row_ptr_dev: int, col_dev: int,
                          val_dev: int, b_dev: int) -> int:
    """Sparse system from device CSR arrays (int64 row pointers, int32
    columns ascending within each row, FP64 values), borrowed for its life."""
    out = ctypes.c_void_p()
    _check(_lib.kpp_system_create_csr(ctypes.c_void_p(ctx), kind, m, n, nnz, ctypes.c_void_p(row_ptr_dev),
                                      ctypes.c_void_p(col_dev), ctypes.c_void_p(val_dev), ctypes.c_void_p(b_dev),
                                      ctypes.byref(out)))
    return out.value


def kpp_system_destroy(sys_: int) -> None:
    _check(_lib.kpp_system_destroy(ctypes.c_void_p(sys_)))


def kpp_solve(sys_: int, params: kpp_params, x_dev: int):
    """Returns (status, kpp_result); raises KppError on a negative status."""
    res = kpp_result()
    st = _check(_lib.kpp_solve(ctypes.c_void_p(sys_), ctypes.byref(params), ctypes.c_void_p(x_dev),
                               ctypes.byref(res)))
    return st, res


def kpp_schedule_generate(kind: int, m: int, n: int, params: kpp_params, T: int, blocks_cap: int):
    """Returns (step_block[T], block_rows[nb][s], block_len[nb]) as Python lists."""
    s = params.block_size
    steps = (ctypes.c_int32 * max(T, 1))()
    rows = (ctypes.c_int32 * max(blocks_cap * s, 1))()
    lens = (ctypes.c_int32 * max(blocks_cap, 1))()
    nb = ctypes.c_int32()
    _check(_lib.kpp_schedule_generate(kind, m, n, ctypes.byref(params), T, steps, rows, lens,
                                      blocks_cap, ctypes.byref(nb)))
    k = nb.value
    return (list(steps[:T]), [list(rows[b * s:(b + 1) * s]) for b in range(k)], list(lens[:k]))


def kpp_set_schedule(params: kpp_params, step_block, block_rows):
    """Point params at a caller-given schedule: step_block[t] is the block of
    step t, block_rows a (blocks x block_size) table of row indices (ascending,
    -1 after the last row of a shorter block).  Returns the int32 arrays the
    pointers refer to; keep them alive until kpp_solve returns."""
    steps = (ctypes.c_int32 * max(len(step_block), 1))(*[int(v) for v in step_block])
    flat = [int(v) for row in block_rows for v in row]
    table = (ctypes.c_int32 * max(len(flat), 1))(*flat)
    params.schedule = ctypes.cast(steps, ctypes.c_void_p).value
    params.schedule_len = len(step_block)
    params.block_rows = ctypes.cast(table, ctypes.c_void_p).value
    params.block_rows_count = len(block_rows)
    return steps, table


def kpp_state_export(sys_: int) -> bytes:
    """The system's resumable solver state (see kpp.h) as bytes."""
    size = ctypes.c_size_t(0)
    _check(_lib.kpp_state_export(ctypes.c_void_p(sys_), None, ctypes.byref(size)))
    buf = (ctypes.c_uint8 * max(size.value, 1))()
    _check(_lib.kpp_state_export(ctypes.c_void_p(sys_), ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(size)))
    return bytes(buf[:size.value])


def kpp_state_import(sys_: int, state: bytes) -> None:
    buf = (ctypes.c_uint8 * max(len(state), 1)).from_buffer_copy(state if state else b"\0")
    _check(_lib.kpp_state_import(ctypes.c_void_p(sys_), ctypes.cast(buf, ctypes.c_void_p), len(state)))


def kpp_solve_multi(sys_: int, params: kpp_params, k: int, B_dev: int, ldb: int, X_dev: int, ldx: int):
    """k right-hand sides (B m x k, X n x k, row-major device arrays).
    Returns (status, [kpp_result] * k)."""
    res = (kpp_result * max(k, 1))()
    st = _check(_lib.kpp_solve_multi(ctypes.c_void_p(sys_), ctypes.byref(params), k, ctypes.c_void_p(B_dev), ldb,
                                     ctypes.c_void_p(X_dev), ldx, res))
    return st, [res[c] for c in range(k)]


def kpp_rht_signs(seed: int, N: int):
    """N signs (+1 / -1, a list of ints) drawn as kpp_solve draws them for rht_seed = seed."""
    out = (ctypes.c_int8 * max(N, 1))()
    _check(_lib.kpp_rht_signs(ctypes.c_uint64(seed), N, out))
    return list(out[:N])


def kpp_rht_general(ctx: int, m: int, n: int, A_dev: int, lda: int, b_dev: int, signs_dev: int, R: int,
                    At_dev: int, ldt: int, bt_dev: int) -> None:
    vp = ctypes.c_void_p
    _check(_lib.kpp_rht_general(vp(ctx), m, n, vp(A_dev), lda, vp(b_dev), vp(signs_dev), R, vp(At_dev), ldt,
                                vp(bt_dev)))


def kpp_rht_psd(ctx: int, n: int, A_dev: int, lda: int, b_dev: int, signs_dev: int, R: int, At_dev: int,
                ldt: int, bt_dev: int, work_dev: int = 0) -> None:
    vp = ctypes.c_void_p
    _check(_lib.kpp_rht_psd(vp(ctx), n, vp(A_dev), lda, vp(b_dev), vp(signs_dev), R, vp(At_dev), ldt, vp(bt_dev),
                            vp(work_dev or None)))


def kpp_rht_vector(ctx: int, R: int, signs_dev: int, x_dev: int, nx: int, y_dev: int, direction: int,
                   work_dev: int = 0) -> None:
    vp = ctypes.c_void_p
    _check(_lib.kpp_rht_vector(vp(ctx), R, vp(signs_dev), vp(x_dev), nx, vp(y_dev), direction,
                               vp(work_dev or None)))


def kpp_block_factor(sys_: int, s: int, lam: float, rows, lens, L_dev: int) -> None:
    nb = len(lens)
    r = (ctypes.c_int32 * max(nb * s, 1))(*[int(v) for v in rows])
    ln = (ctypes.c_int32 * max(nb, 1))(*[int(v) for v in lens])
    _check(_lib.kpp_block_factor(ctypes.c_void_p(sys_), s, lam, nb, r, ln, ctypes.c_void_p(L_dev)))


def kpp_block_factor_noalloc(sys_: int, s: int, lam: float, rows, lens, L_dev: int) -> None:
    nb = len(lens)
    r = (ctypes.c_int32 * max(nb * s, 1))(*[int(v) for v in rows])
    ln = (ctypes.c_int32 * max(nb, 1))(*[int(v) for v in lens])
    _check(_lib.kpp_block_factor_noalloc(ctypes.c_void_p(sys_), s, lam, nb, r, ln, ctypes.c_void_p(L_dev)))


def kpp_residual_norm(sys_: int, x_dev: int) -> float:
    out = ctypes.c_double()
    _check(_lib.kpp_residual_norm(ctypes.c_void_p(sys_), ctypes.c_void_p(x_dev), ctypes.byref(out)))
    return out.value


def kpp_request_footprint(sys_: int, params: kpp_params) -> int:
    out = ctypes.c_uint64()
    _check(_lib.kpp_request_footprint(ctypes.c_void_p(sys_), ctypes.byref(params), ctypes.byref(out)))
    return out.value


def kpp_server_create(ctx: int, hbm_budget_bytes: int, max_active: int) -> int:
    out = ctypes.c_void_p()
    _check(_lib.kpp_server_create(ctypes.c_void_p(ctx), int(hbm_budget_bytes), max_active, ctypes.byref(out)))
    return out.value


def kpp_server_submit(srv: int, sys_: int, params: kpp_params, x_dev: int) -> int:
    """Returns the request id; raises KppError (KPP_ERR_REJECTED, ...) if refused."""
    rid = ctypes.c_uint64()
    _check(_lib.kpp_server_submit(ctypes.c_void_p(srv), ctypes.c_void_p(sys_), ctypes.byref(params),
                                  ctypes.c_void_p(x_dev), ctypes.byref(rid)))
    return rid.value


def kpp_server_poll(srv: int, cap: int = 64, wait_seconds: float = 0.0):
    """Returns [(id, status, kpp_result), ...] of finished requests."""
    ids = (ctypes.c_uint64 * max(cap, 1))()
    sts = (ctypes.c_int32 * max(cap, 1))()
    res = (kpp_result * max(cap, 1))()
    n = ctypes.c_int32()
    _check(_lib.kpp_server_poll(ctypes.c_void_p(srv), cap, float(wait_seconds), ids, sts, res, ctypes.byref(n)))
    return [(ids[i], sts[i], res[i]) for i in range(n.value)]


def kpp_server_stats(srv: int) -> kpp_server_info:
    out = kpp_server_info()
    _check(_lib.kpp_server_stats(ctypes.c_void_p(srv), ctypes.byref(out)))
    return out


def kpp_server_destroy(srv: int) -> None:
    _check(_lib.kpp_server_destroy(ctypes.c_void_p(srv)))
