"""Thin ctypes binding of libgmrf.so (include/gmrf.h).

Functions keep the C names and take device buffers as integers (HIP device
addresses, e.g. ``tensor.data_ptr()``) or as torch tensors, whose
``data_ptr()`` is passed.  No computation happens here: every step runs in
the library's HIP kernels.  Importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from collections.abc import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GMRF_LIB selects another build of the library (the host-sanitized one)
LIB_PATH = os.environ.get("GMRF_LIB") or os.path.join(_HERE, "libgmrf.so")

GP_OK = 0
GP_ERR_INVALID_ARG = -1
GP_ERR_NOT_SPD = -2
GP_ERR_OOM = -3
GP_ERR_BUSY = -4
GP_ERR_NOT_CONVERGED = -5
GP_ERR_BREAKDOWN = -6
GP_ERR_DEVICE = -7
GP_ERR_TIMEOUT = -8
GP_ERR_CANCELLED = -9
GP_KMAX = 24          # largest K; length of gp_result's per-regressor arrays
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "NOT_SPD", -3: "OOM", -4: "BUSY",
                -5: "NOT_CONVERGED", -6: "BREAKDOWN", -7: "DEVICE", -8: "TIMEOUT", -9: "CANCELLED"}

GP_PRECOND_JACOBI = 0
GP_PRECOND_BLOCK_JACOBI = 1
GP_PRECOND_RB_IC0 = 2
GP_MATVEC_AUTO, GP_MATVEC_RASTER, GP_MATVEC_ZMARCH = 0, 1, 2
GP_PREC_FP64 = 0
GP_PREC_FP32_REFINE64 = 1

# every symbol the header declares
EXPORTS = [
    "gp_opts_default", "gp_last_error", "gp_version",
    "gp_ctx_create", "gp_ctx_set_stream", "gp_ctx_memory", "gp_ctx_destroy",
    "gp_ctx_profile", "gp_ctx_profile_read",
    "gp_op_create", "gp_op_set_blocks", "gp_op_set_alpha", "gp_op_query",
    "gp_op_voxel_index", "gp_op_destroy",
    "gp_apply", "gp_solve", "gp_solve_batch", "gp_perturb_rhs", "gp_sample",
    "gp_probe_rhs", "gp_trace_reduce", "gp_trace_reduce_static", "gp_trace",
    "gp_rng_normal", "gp_rng_rademacher", "gp_rng_raw",
    "gp_server_cfg_default", "gp_server_create", "gp_server_submit", "gp_server_poll",
    "gp_server_drain", "gp_server_get_stats", "gp_server_destroy", "gp_server_cancel", "gp_server_step",
    "gp_autotune", "gp_tune_save", "gp_tune_load",
    "gp_data_create", "gp_data_assemble", "gp_data_lambda", "gp_data_destroy", "gp_alpha_posterior",
    "gp_hyper_default", "gp_svb_step", "gp_data_assemble_ar", "gp_svb_step_ar", "gp_alpha_extrapolate",
    "gp_rng_gamma", "gp_gibbs_step",
]

GP_REQ_SOLVE, GP_REQ_SAMPLE, GP_REQ_TRACE = 0, 1, 2


class GpOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("max_outer", ctypes.c_int),
                ("precond", ctypes.c_int), ("precision", ctypes.c_int),
                ("rhs_tile", ctypes.c_int), ("chunk", ctypes.c_int),
                ("wg_per_cu", ctypes.c_int), ("matvec", ctypes.c_int),
                ("zero_guess", ctypes.c_int), ("seed", ctypes.c_uint64)]


class GpStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("outer_steps", ctypes.c_int), ("reserved", ctypes.c_int),
                ("relres", ctypes.c_double), ("time_us", ctypes.c_double)]


class GpProf(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("units", ctypes.c_int64),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


KERNEL_KINDS = ["refine", "matvec", "update", "addsol", "perturb", "precond", "pack",
                "probe", "trace", "apply", "data", "rb_red", "rb_matvec", "rb_update", "rb_refine",
                "rb_addsol", "rb_edge", "rb_red64"]


class GpItem(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("R", ctypes.c_int),
                ("b", ctypes.c_void_p), ("x", ctypes.c_void_p)]


class GpServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active_rhs", ctypes.c_int),
                ("chunk", ctypes.c_int), ("probes", ctypes.c_int), ("manual", ctypes.c_int),
                ("reserved", ctypes.c_int), ("opts", GpOpts)]


class GpRequest(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("op_index", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("out", ctypes.c_void_p), ("timeout_ms", ctypes.c_double)]


class GpResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("kind", ctypes.c_int), ("op_index", ctypes.c_int),
                ("status", ctypes.c_int), ("rhs", ctypes.c_int), ("iters_max", ctypes.c_int),
                ("reserved", ctypes.c_int), ("relres_max", ctypes.c_double),
                ("latency_us", ctypes.c_double), ("queue_us", ctypes.c_double),
                ("admit_round", ctypes.c_int64), ("retire_round", ctypes.c_int64),
                ("trace_total", ctypes.c_double), ("trace_kk", ctypes.c_double * GP_KMAX),
                ("trace_Gkk", ctypes.c_double * GP_KMAX)]


class GpServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rhs_solved", ctypes.c_int64), ("peak_active_rhs", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("elapsed_s", ctypes.c_double), ("solves_per_s", ctypes.c_double),
                ("requests_per_s", ctypes.c_double)]


class GpHyper(ctypes.Structure):
    _fields_ = [("q1", ctypes.c_double), ("q2", ctypes.c_double), ("u1", ctypes.c_double),
                ("u2", ctypes.c_double), ("r1", ctypes.c_double), ("r2", ctypes.c_double)]


class GmrfError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with "
                          "`python -m paper_1606_00980_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                             ctypes.c_double, ctypes.c_size_t)
    P = ctypes.POINTER
    sig = {
        "gp_opts_default": (None, [P(GpOpts)]),
        "gp_last_error": (ctypes.c_char_p, []),
        "gp_version": (i32, []),
        "gp_ctx_create": (i32, [i32, vp, sz, P(vp)]),
        "gp_ctx_set_stream": (i32, [vp, vp]),
        "gp_ctx_memory": (i32, [vp, P(sz), P(sz)]),
        "gp_ctx_destroy": (i32, [vp]),
        "gp_ctx_profile": (i32, [vp, i32]),
        "gp_ctx_profile_read": (i32, [vp, i32, P(GpProf)]),
        "gp_op_create": (i32, [vp, vp, i32, i32, i32, i32, i32, P(vp)]),
        "gp_op_set_blocks": (i32, [vp, vp, P(i64)]),
        "gp_op_set_alpha": (i32, [vp, P(dbl)]),
        "gp_op_query": (i32, [vp, P(i64), P(i64), P(i32), P(sz)]),
        "gp_op_voxel_index": (i32, [vp, vp]),
        "gp_op_destroy": (i32, [vp]),
        "gp_apply": (i32, [vp, i32, vp, vp]),
        "gp_solve": (i32, [vp, i32, vp, vp, P(GpOpts), P(GpStats)]),
        "gp_solve_batch": (i32, [vp, i32, P(GpItem), P(GpOpts), P(GpStats)]),
        "gp_perturb_rhs": (i32, [vp, i32, vp, vp, vp, vp]),
        "gp_sample": (i32, [vp, i32, vp, vp, vp, vp, P(GpOpts), P(GpStats)]),
        "gp_probe_rhs": (i32, [vp, i32, vp, vp]),
        "gp_trace_reduce": (i32, [vp, i32, vp, vp, P(dbl), P(dbl), P(dbl)]),
        "gp_trace_reduce_static": (i32, [vp, i32, vp, vp, P(dbl), P(dbl), P(dbl)]),
        "gp_trace": (i32, [vp, i32, vp, vp, P(dbl), P(dbl), P(dbl), P(GpOpts), P(GpStats)]),
        "gp_rng_normal": (i32, [vp, ctypes.c_uint64, ctypes.c_uint64, sz, vp]),
        "gp_rng_rademacher": (i32, [vp, ctypes.c_uint64, ctypes.c_uint64, sz, vp]),
        "gp_rng_raw": (i32, [vp, ctypes.c_uint64, ctypes.c_uint64, sz, vp]),
        "gp_server_cfg_default": (None, [P(GpServerCfg)]),
        "gp_server_create": (i32, [vp, i32, P(vp), P(vp), P(GpServerCfg), P(vp)]),
        "gp_server_submit": (i32, [vp, P(GpRequest), P(ctypes.c_uint64)]),
        "gp_server_poll": (i32, [vp, P(GpResult), i32, P(i32)]),
        "gp_server_drain": (i32, [vp, i32]),
        "gp_server_get_stats": (i32, [vp, P(GpServerStats)]),
        "gp_server_destroy": (i32, [vp]),
        "gp_server_cancel": (i32, [vp, ctypes.c_uint64]),
        "gp_server_step": (i32, [vp, i32]),
        "gp_autotune": (i32, [vp, i32, P(GpOpts), P(GpOpts)]),
        "gp_tune_save": (i32, [vp, ctypes.c_char_p]),
        "gp_tune_load": (i32, [vp, ctypes.c_char_p]),
        "gp_data_create": (i32, [vp, i32, i32, P(dbl), vp, P(vp)]),
        "gp_data_assemble": (i32, [vp, vp, i32, vp, vp, P(i64)]),
        "gp_data_destroy": (i32, [vp]),
        "gp_data_lambda": (i32, [vp, i32, vp, vp, dbl, dbl, vp, vp, vp]),
        "gp_alpha_posterior": (i32, [vp, i32, vp, dbl, dbl, P(dbl), P(dbl), P(dbl)]),
        "gp_hyper_default": (None, [P(GpHyper)]),
        "gp_svb_step": (i32, [vp, i32, vp, vp, vp, vp, vp, P(dbl), P(GpHyper), vp, P(GpOpts), P(GpStats)]),
        "gp_data_assemble_ar": (i32, [vp, vp, vp, i32, vp, vp, P(i64)]),
        "gp_alpha_extrapolate": (i32, [i32, P(dbl), P(dbl), P(dbl)]),
        "gp_rng_gamma": (i32, [vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_size_t, dbl, vp, vp]),
        "gp_gibbs_step": (i32, [vp, vp, vp, vp, vp, vp, P(dbl), P(GpHyper), vp, ctypes.c_uint64, ctypes.c_uint64,
                                P(GpOpts), P(GpStats)]),
        "gp_svb_step_ar": (i32, [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, P(dbl), P(dbl), P(GpHyper), vp, vp,
                                 P(GpOpts), P(GpStats), P(GpStats)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _ptr(buf) -> int | None:
    """Device address of a torch tensor (or an int passed through)."""
    if buf is None:
        return None
    if isinstance(buf, int):
        return buf
    return buf.data_ptr()


def _check(status: int, where: str) -> int:
    if status != GP_OK:
        raise GmrfError(status, where, lib.gp_last_error().decode())
    return status


def gp_opts_default(**overrides) -> GpOpts:
    o = GpOpts()
    lib.gp_opts_default(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def gp_last_error() -> str:
    return lib.gp_last_error().decode()


def gp_version() -> int:
    return lib.gp_version()


def gp_ctx_create(device: int = 0, stream: int | None = None, hbm_budget: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib.gp_ctx_create(device, stream, hbm_budget, ctypes.byref(h)), "gp_ctx_create")
    return h.value


def gp_ctx_set_stream(ctx: int, stream: int | None) -> None:
    _check(lib.gp_ctx_set_stream(ctx, stream), "gp_ctx_set_stream")


def gp_ctx_memory(ctx: int):
    used, budget = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.gp_ctx_memory(ctx, ctypes.byref(used), ctypes.byref(budget)), "gp_ctx_memory")
    return used.value, budget.value


def gp_ctx_destroy(ctx: int) -> None:
    _check(lib.gp_ctx_destroy(ctx), "gp_ctx_destroy")


def gp_ctx_profile(ctx: int, enable: bool) -> None:
    _check(lib.gp_ctx_profile(ctx, 1 if enable else 0), "gp_ctx_profile")


def gp_ctx_profile_read(ctx: int) -> dict:
    """{kind: {launches, units, ms, bytes}} for every kernel kind."""
    out = {}
    for i, name in enumerate(KERNEL_KINDS):
        p = GpProf()
        _check(lib.gp_ctx_profile_read(ctx, i, ctypes.byref(p)), "gp_ctx_profile_read")
        out[name] = {"launches": p.launches, "units": p.units, "ms": p.ms, "bytes": p.bytes}
    return out


def gp_op_create(ctx: int, mask: np.ndarray, conn: int, K: int) -> int:
    """mask: host array shaped (nz, ny, nx) (or (ny, nx)), nonzero = in mask."""
    m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
    if m.ndim == 2:
        m = m[None]
    nz, ny, nx = m.shape
    h = ctypes.c_void_p()
    _check(lib.gp_op_create(ctx, m.ctypes.data, nx, ny, nz, conn, K, ctypes.byref(h)),
           "gp_op_create")
    return h.value


def gp_op_set_blocks(op: int, B) -> None:
    bad = ctypes.c_int64(-1)
    st = lib.gp_op_set_blocks(op, _ptr(B), ctypes.byref(bad))
    if st != GP_OK:
        err = GmrfError(st, "gp_op_set_blocks", gp_last_error())
        err.bad_voxel = bad.value
        raise err


def gp_data_create(op: int, T: int, P: int, X, Y) -> int:
    """X: host (T, K) array; Y: device (T, N) FP64 tensor."""
    x = np.ascontiguousarray(X, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(lib.gp_data_create(op, T, P, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(Y),
                              ctypes.byref(h)), "gp_data_create")
    return h.value


def gp_data_assemble(d: int, lam, Ns: int, A, bw=None) -> None:
    bad = ctypes.c_int64(-1)
    st = lib.gp_data_assemble(d, _ptr(lam), Ns, _ptr(A), _ptr(bw), ctypes.byref(bad))
    if st != GP_OK:
        err = GmrfError(st, "gp_data_assemble", gp_last_error())
        err.bad_voxel = bad.value
        raise err


def gp_data_assemble_ar(d: int, op_a: int, lam, Ns: int, W, ba=None) -> None:
    bad = ctypes.c_int64(-1)
    st = lib.gp_data_assemble_ar(d, op_a, _ptr(lam), Ns, _ptr(W), _ptr(ba), ctypes.byref(bad))
    if st != GP_OK:
        err = GmrfError(st, "gp_data_assemble_ar", gp_last_error())
        err.bad_voxel = bad.value
        raise err


def gp_svb_step_ar(d: int, op_a: int, Ns: int, z1w, z2w, W, z1a, z2a, A, lam, alpha, beta, bw_work, ba_work,
                   prior: GpHyper | None = None, opts: GpOpts | None = None, check: bool = True):
    """One SVB iteration over W, A, alpha, beta and lambda; alpha and beta
    (numpy) and W, A, lam (device) are updated in place.  Returns (status,
    W-sampling stats, A-sampling stats)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    sw, sa = _stats_array(Ns), _stats_array(Ns)
    o = opts if opts is not None else gp_opts_default()
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.gp_svb_step_ar(d, op_a, Ns, _ptr(z1w), _ptr(z2w), _ptr(W), _ptr(z1a), _ptr(z2a), _ptr(A), _ptr(lam),
                            a.ctypes.data_as(dp), b.ctypes.data_as(dp),
                            ctypes.byref(prior) if prior is not None else None, _ptr(bw_work), _ptr(ba_work),
                            ctypes.byref(o), sw, sa)
    if check:
        _check(st, "gp_svb_step_ar")
    alpha[:] = a
    beta[:] = b
    return st, _stats_list(sw, Ns), _stats_list(sa, Ns)


def gp_rng_gamma(ctx: int, seed: int, stream: int, n: int, shape: float, scale, out) -> None:
    _check(lib.gp_rng_gamma(ctx, seed, stream, n, shape, _ptr(scale), _ptr(out)), "gp_rng_gamma")


def gp_gibbs_step(d: int, A, z1, z2, W, lam, alpha, bw_work, seed: int, iteration: int,
                  prior: GpHyper | None = None, opts: GpOpts | None = None, check: bool = True):
    """One Gibbs iteration for W, alpha, lambda; alpha (numpy) and W, lam
    (device) are updated in place.  Returns (status, stats of the W draw)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    st_arr = _stats_array(1)
    o = opts if opts is not None else gp_opts_default()
    st = lib.gp_gibbs_step(d, _ptr(A), _ptr(z1), _ptr(z2), _ptr(W), _ptr(lam),
                           a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           ctypes.byref(prior) if prior is not None else None, _ptr(bw_work), seed, iteration,
                           ctypes.byref(o), st_arr)
    if check:
        _check(st, "gp_gibbs_step")
    alpha[:] = a
    return st, _stats_list(st_arr, 1)


def gp_alpha_extrapolate(a_jm2, a_jm1, a_j) -> np.ndarray:
    """Returns the extrapolated a_j (numpy) from the last three posterior means."""
    dp = ctypes.POINTER(ctypes.c_double)
    x2 = np.ascontiguousarray(a_jm2, dtype=np.float64)
    x1 = np.ascontiguousarray(a_jm1, dtype=np.float64)
    x0 = np.array(a_j, dtype=np.float64)
    _check(lib.gp_alpha_extrapolate(x0.size, x2.ctypes.data_as(dp), x1.ctypes.data_as(dp), x0.ctypes.data_as(dp)),
           "gp_alpha_extrapolate")
    return x0


def gp_data_lambda(d: int, Ns: int, W, A, u1: float, u2: float, rss=None, scale=None, mean=None) -> None:
    _check(lib.gp_data_lambda(d, Ns, _ptr(W), _ptr(A), u1, u2, _ptr(rss), _ptr(scale), _ptr(mean)),
           "gp_data_lambda")


def gp_alpha_posterior(op: int, R: int, W, q1: float, q2: float, K: int):
    """Returns (qf (R, K), scale (K), mean (K)) as numpy arrays."""
    qf = np.empty(R * K); sc = np.empty(K); mn = np.empty(K)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.gp_alpha_posterior(op, R, _ptr(W), q1, q2, qf.ctypes.data_as(dp), sc.ctypes.data_as(dp),
                                  mn.ctypes.data_as(dp)), "gp_alpha_posterior")
    return qf.reshape(R, K), sc, mn


def gp_hyper_default(**overrides) -> GpHyper:
    h = GpHyper()
    lib.gp_hyper_default(ctypes.byref(h))
    for k, v in overrides.items():
        setattr(h, k, v)
    return h


def gp_svb_step(d: int, Ns: int, A, z1, z2, W, lam, alpha, bw_work, prior: GpHyper | None = None,
                opts: GpOpts | None = None, check: bool = True):
    """One SVB iteration; alpha (numpy, K) and lam / W (device) are updated in
    place.  Returns (status, per-sample stats)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    st_arr = _stats_array(Ns)
    o = opts if opts is not None else gp_opts_default()
    st = lib.gp_svb_step(d, Ns, _ptr(A), _ptr(z1), _ptr(z2), _ptr(W), _ptr(lam),
                         a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         ctypes.byref(prior) if prior is not None else None, _ptr(bw_work), ctypes.byref(o), st_arr)
    if check:
        _check(st, "gp_svb_step")
    alpha[:] = a
    return st, _stats_list(st_arr, Ns)


def gp_data_destroy(d: int) -> None:
    _check(lib.gp_data_destroy(d), "gp_data_destroy")


def gp_op_set_alpha(op: int, alpha) -> None:
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    _check(lib.gp_op_set_alpha(op, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "gp_op_set_alpha")


def gp_op_query(op: int) -> dict:
    N, E, K, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int(), ctypes.c_size_t()
    _check(lib.gp_op_query(op, ctypes.byref(N), ctypes.byref(E), ctypes.byref(K),
                           ctypes.byref(nb)), "gp_op_query")
    return {"N": N.value, "E": E.value, "K": K.value, "bytes": nb.value}


def gp_op_voxel_index(op: int, lin) -> None:
    _check(lib.gp_op_voxel_index(op, _ptr(lin)), "gp_op_voxel_index")


def gp_op_destroy(op: int) -> None:
    _check(lib.gp_op_destroy(op), "gp_op_destroy")


def gp_apply(op: int, R: int, x, y) -> None:
    _check(lib.gp_apply(op, R, _ptr(x), _ptr(y)), "gp_apply")


def _stats_array(n: int):
    return (GpStats * max(n, 1))()


_STATS_DTYPE = np.dtype([("status", np.int32), ("inner_iters", np.int32), ("outer_steps", np.int32),
                         ("reserved", np.int32), ("relres", np.float64), ("time_us", np.float64)])


class StatsList(Sequence):
    """Per-right-hand-side statistics as a read-only sequence of dicts with
    the fields of gp_stats; entries are built on access (a solve's caller
    often looks at few of them)."""

    __slots__ = ("_a",)

    def __init__(self, arr, n: int):
        self._a = np.frombuffer(arr, dtype=_STATS_DTYPE, count=n)

    def __len__(self):
        return len(self._a)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(len(self)))]
        e = self._a[i]
        return {"status": int(e["status"]), "inner_iters": int(e["inner_iters"]),
                "outer_steps": int(e["outer_steps"]), "relres": float(e["relres"]),
                "time_us": float(e["time_us"])}

    def __add__(self, other):
        return list(self) + list(other)

    def __radd__(self, other):
        return list(other) + list(self)

    def __eq__(self, other):
        if isinstance(other, (list, tuple, StatsList)):
            return list(self) == list(other)
        return NotImplemented

    __hash__ = None

    def __repr__(self):
        return repr(list(self))


def _stats_list(arr, n: int):
    return StatsList(arr, n)


def gp_solve(op: int, R: int, b, x, opts: GpOpts | None = None, check: bool = True):
    """Returns (status, per-RHS stats list)."""
    st_arr = _stats_array(R)
    o = opts if opts is not None else gp_opts_default()
    st = lib.gp_solve(op, R, _ptr(b), _ptr(x), ctypes.byref(o), st_arr)
    if check:
        _check(st, "gp_solve")
    return st, _stats_list(st_arr, R)


def gp_solve_batch(ctx: int, items, opts: GpOpts | None = None, check: bool = True):
    """items: list of (op, R, b, x)."""
    arr = (GpItem * max(len(items), 1))()
    total = 0
    for i, (op, R, b, x) in enumerate(items):
        arr[i].op, arr[i].R, arr[i].b, arr[i].x = op, R, _ptr(b), _ptr(x)
        total += R
    st_arr = _stats_array(total)
    o = opts if opts is not None else gp_opts_default()
    st = lib.gp_solve_batch(ctx, len(items), arr, ctypes.byref(o), st_arr)
    if check:
        _check(st, "gp_solve_batch")
    return st, _stats_list(st_arr, total)


def gp_perturb_rhs(op: int, R: int, bw, z1, z2, b) -> None:
    _check(lib.gp_perturb_rhs(op, R, _ptr(bw), _ptr(z1), _ptr(z2), _ptr(b)), "gp_perturb_rhs")


def gp_sample(op: int, R: int, bw, z1, z2, w, opts: GpOpts | None = None, check: bool = True):
    st_arr = _stats_array(R)
    o = opts if opts is not None else gp_opts_default()
    st = lib.gp_sample(op, R, _ptr(bw), _ptr(z1), _ptr(z2), _ptr(w), ctypes.byref(o), st_arr)
    if check:
        _check(st, "gp_sample")
    return st, _stats_list(st_arr, R)


def gp_probe_rhs(op: int, m: int, probes, b) -> None:
    _check(lib.gp_probe_rhs(op, m, _ptr(probes), _ptr(b)), "gp_probe_rhs")


def _trace_out(K: int):
    return (ctypes.c_double(), (ctypes.c_double * K)(), (ctypes.c_double * K)())


def gp_trace_reduce(op: int, m: int, probes, u, K: int):
    t, tk, gk = _trace_out(K)
    _check(lib.gp_trace_reduce(op, m, _ptr(probes), _ptr(u), ctypes.byref(t), tk, gk),
           "gp_trace_reduce")
    return t.value, np.array(tk[:]), np.array(gk[:])


def gp_trace_reduce_static(op: int, m: int, probes, u, K: int):
    t, tk, gk = _trace_out(K)
    _check(lib.gp_trace_reduce_static(op, m, _ptr(probes), _ptr(u), ctypes.byref(t), tk, gk),
           "gp_trace_reduce_static")
    return t.value, np.array(tk[:]), np.array(gk[:])


def gp_trace(op: int, m: int, probes, u, K: int, opts: GpOpts | None = None):
    t, tk, gk = _trace_out(K)
    st_arr = _stats_array(m)
    o = opts if opts is not None else gp_opts_default()
    _check(lib.gp_trace(op, m, _ptr(probes), _ptr(u), ctypes.byref(t), tk, gk,
                        ctypes.byref(o), st_arr), "gp_trace")
    return t.value, np.array(tk[:]), np.array(gk[:]), _stats_list(st_arr, m)


def gp_rng_normal(ctx: int, seed: int, stream: int, n: int, out) -> None:
    _check(lib.gp_rng_normal(ctx, seed, stream, n, _ptr(out)), "gp_rng_normal")


def gp_rng_rademacher(ctx: int, seed: int, stream: int, n: int, out) -> None:
    _check(lib.gp_rng_rademacher(ctx, seed, stream, n, _ptr(out)), "gp_rng_rademacher")


def gp_rng_raw(ctx: int, seed: int, stream: int, nblocks: int, out) -> None:
    _check(lib.gp_rng_raw(ctx, seed, stream, nblocks, _ptr(out)), "gp_rng_raw")


def gp_server_cfg_default(**overrides) -> GpServerCfg:
    c = GpServerCfg()
    lib.gp_server_cfg_default(ctypes.byref(c))
    for k, v in overrides.items():
        if k == "opts":
            c.opts = v
        else:
            setattr(c, k, v)
    return c


def gp_server_create(ctx: int, ops, bws, cfg: GpServerCfg | None = None) -> int:
    n = len(ops)
    oa = (ctypes.c_void_p * n)(*ops)
    ba = (ctypes.c_void_p * n)(*[_ptr(b) for b in bws])
    h = ctypes.c_void_p()
    c = cfg if cfg is not None else gp_server_cfg_default()
    _check(lib.gp_server_create(ctx, n, oa, ba, ctypes.byref(c), ctypes.byref(h)), "gp_server_create")
    return h.value


def gp_server_submit(srv: int, kind: int, op_index: int, seed: int, out=None, timeout_ms: float = 0.0) -> int:
    r = GpRequest(kind, op_index, seed, _ptr(out), timeout_ms)
    t = ctypes.c_uint64()
    _check(lib.gp_server_submit(srv, ctypes.byref(r), ctypes.byref(t)), "gp_server_submit")
    return t.value


def gp_server_cancel(srv: int, ticket: int) -> None:
    _check(lib.gp_server_cancel(srv, ticket), "gp_server_cancel")


def gp_server_step(srv: int, rounds: int = 1) -> None:
    _check(lib.gp_server_step(srv, rounds), "gp_server_step")


def _result_dict(r: GpResult) -> dict:
    return {"ticket": r.ticket, "kind": r.kind, "op_index": r.op_index, "status": r.status,
            "rhs": r.rhs, "iters_max": r.iters_max, "relres_max": r.relres_max,
            "latency_us": r.latency_us, "queue_us": r.queue_us, "admit_round": r.admit_round,
            "retire_round": r.retire_round, "trace_total": r.trace_total,
            "trace_kk": list(r.trace_kk), "trace_Gkk": list(r.trace_Gkk)}


def gp_server_poll(srv: int, max_results: int = 256) -> list:
    arr = (GpResult * max_results)()
    n = ctypes.c_int()
    _check(lib.gp_server_poll(srv, arr, max_results, ctypes.byref(n)), "gp_server_poll")
    return [_result_dict(arr[i]) for i in range(n.value)]


def gp_server_drain(srv: int, timeout_ms: int = -1) -> None:
    _check(lib.gp_server_drain(srv, timeout_ms), "gp_server_drain")


def gp_server_get_stats(srv: int) -> dict:
    s = GpServerStats()
    _check(lib.gp_server_get_stats(srv, ctypes.byref(s)), "gp_server_get_stats")
    return {f: getattr(s, f) for f, _ in GpServerStats._fields_}


def gp_server_destroy(srv: int) -> None:
    _check(lib.gp_server_destroy(srv), "gp_server_destroy")


def gp_autotune(op: int, R: int, base: GpOpts | None = None) -> GpOpts:
    b = base if base is not None else gp_opts_default()
    best = GpOpts()
    _check(lib.gp_autotune(op, R, ctypes.byref(b), ctypes.byref(best)), "gp_autotune")
    return best


def gp_tune_save(ctx: int, path: str) -> None:
    _check(lib.gp_tune_save(ctx, path.encode()), "gp_tune_save")


def gp_tune_load(ctx: int, path: str) -> None:
    _check(lib.gp_tune_load(ctx, path.encode()), "gp_tune_load")
