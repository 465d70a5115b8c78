"""Python binding of libctrace (include/ctrace.h): argument marshalling only.

Every entry point of the C ABI is exposed under the same name; the
`TraceContext` class bundles the context with a device arena and stream
taken from PyTorch (PyTorch is used for device memory and streams only).
The library must be built (paper_2010_08482_amd.build_lib); importing this
module without it raises immediately - there is no fallback path.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libctrace.so")

CTR_OK = 0
CTR_FP64 = 0
CTR_FP32_SPLIT = 1
CTR_FLAG_ZERO = 1
CTR_FLAG_REJECTED = 2
CTR_FLAG_INVALID = 4
CTR_KERNEL_AUTO = 0
CTR_KERNEL_WAVE = 1
CTR_KERNEL_BLOCK = 2
CTR_KERNEL_STREAM = 3
CTR_KERNEL_GROUPED = 4
CTR_KERNEL_GROUPED_ROWS = 5
CTR_OPT_GRAPH = 1


class ctr_value(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double), ("log_scale", ctypes.c_double),
                ("log_bound", ctypes.c_double), ("log_abs", ctypes.c_double), ("n_strings", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class ctr_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("slices", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class ctr_impurity(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("n_flavors", ctypes.c_int32), ("n_sectors", ctypes.c_int32),
                ("is_complex", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sector_dim", ctypes.POINTER(ctypes.c_int32)), ("energies", ctypes.POINTER(ctypes.c_double)),
                ("next", ctypes.POINTER(ctypes.c_int32)), ("blocks", ctypes.POINTER(ctypes.c_void_p)),
                ("block_norm", ctypes.POINTER(ctypes.c_double))]


class ctr_server_opts(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("max_pending", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t),
                ("grid_share", ctypes.POINTER(ctypes.c_double)), ("max_pass_flop", ctypes.c_double)]


class ctr_mc_opts(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int32), ("n_bath", ctypes.c_int32), ("bath_eps", ctypes.POINTER(ctypes.c_double)),
                ("bath_v", ctypes.POINTER(ctypes.c_double)), ("rebuild_every", ctypes.c_int32),
                ("full_traces", ctypes.c_int32)]


class ctr_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("impurity", ctypes.c_int32), ("status", ctypes.c_int32),
                ("value", ctr_value), ("latency_ms", ctypes.c_double), ("batch", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


VALUE_DTYPE = np.dtype([("re", "<f8"), ("im", "<f8"), ("log_scale", "<f8"), ("log_bound", "<f8"), ("log_abs", "<f8"),
                        ("n_strings", "<i4"), ("flags", "<i4")])
assert VALUE_DTYPE.itemsize == ctypes.sizeof(ctr_value)
RESULT_DTYPE = np.dtype([("tag", "<u8"), ("impurity", "<i4"), ("status", "<i4"), ("value", VALUE_DTYPE),
                         ("latency_ms", "<f8"), ("batch", "<i4"), ("reserved", "<i4")])
assert RESULT_DTYPE.itemsize == ctypes.sizeof(ctr_result)
CTR_ERR_BUSY = -8
CTR_STATIC_SCRATCH_BYTES = 64 << 20  # ctr_trace_batch_device_static: per-call scratch array per device


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2010_08482_amd.build_lib` "
                          "(the trace has no CPU or PyTorch fallback)")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "ctr_version": (ctypes.c_char_p, []),
        "ctr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "ctr_last_error": (ctypes.c_char_p, [vp]),
        "ctr_create": (ctypes.c_int, [ctypes.c_int, vp, ctypes.c_size_t, vp, P(vp)]),
        "ctr_destroy": (None, [vp]),
        "ctr_set_impurity": (ctypes.c_int, [vp, P(ctr_impurity)]),
        "ctr_arena_resident_bytes": (ctypes.c_size_t, [vp]),
        "ctr_trace": (ctypes.c_int, [vp, i32, P(f64), P(i32), P(ctr_opts), P(ctr_value)]),
        "ctr_trace_batch": (ctypes.c_int, [vp, i32, P(i64), P(f64), P(i32), P(ctr_opts), P(ctr_value)]),
        "ctr_trace_batch_device": (ctypes.c_int, [vp, i32, vp, vp, vp, P(ctr_opts), vp]),
        "ctr_trace_batch_device_static": (ctypes.c_int, [vp, i32, vp, vp, vp, P(ctr_opts), vp]),
        "ctr_trace_lazy_batch": (ctypes.c_int, [vp, i32, P(i64), P(f64), P(i32), P(f64), P(ctr_opts),
                                                P(ctr_value)]),
        "ctr_trace_lazy": (ctypes.c_int, [vp, i32, P(f64), P(i32), f64, P(ctr_opts), P(ctr_value)]),
        "ctr_trace_histogram": (ctypes.c_int, [vp, i32, P(i64), P(f64), P(i32), P(i32), i32, P(ctr_opts),
                                               P(ctr_value), P(f64)]),
        "ctr_bound": (ctypes.c_int, [vp, i32, P(f64), P(i32), P(f64)]),
        "ctr_density_matrix": (ctypes.c_int, [vp, i32, P(i64), P(f64), P(i32), P(f64), P(ctr_value), P(f64)]),
        "ctr_strings": (ctypes.c_int, [vp, i32, P(i32), P(i32), P(i32)]),
        "ctr_synchronize": (ctypes.c_int, [vp]),
        "ctr_last_kernel": (ctypes.c_int, [vp, P(i32), P(i32)]),
        "ctr_probe_peaks": (ctypes.c_int, [vp, P(f64)]),
        "ctr_kernel_timing": (ctypes.c_int, [vp, i32]),
        "ctr_kernel_timing_read": (ctypes.c_int, [vp, P(f64), P(i32)]),
        "ctr_tune": (ctypes.c_int, [vp, i32, P(i64), P(f64), P(i32), P(i32), P(f64)]),
        "ctr_server_create": (ctypes.c_int, [P(vp), i32, P(ctr_server_opts), P(vp)]),
        "ctr_server_submit": (ctypes.c_int, [vp, i32, ctypes.c_uint64, i32, P(f64), P(i32), f64]),
        "ctr_server_poll": (ctypes.c_int, [vp, vp, i32, P(i32), i32]),
        "ctr_server_drain": (ctypes.c_int, [vp]),
        "ctr_server_stats": (ctypes.c_int, [vp, P(i64), P(i64)]),
        "ctr_server_destroy": (None, [vp]),
        "ctr_mc_create": (ctypes.c_int, [vp, P(ctr_mc_opts), P(vp)]),
        "ctr_mc_set_config": (ctypes.c_int, [vp, i32, i32, P(f64), P(i32)]),
        "ctr_mc_step": (ctypes.c_int, [vp, P(f64), P(i32)]),
        "ctr_mc_config": (ctypes.c_int, [vp, i32, i32, P(f64), P(i32), P(i32), P(f64)]),
        "ctr_mc_stats": (ctypes.c_int, [vp, P(i64), P(i64), P(i64), P(i64)]),
        "ctr_mc_timing": (ctypes.c_int, [vp, P(f64), P(f64)]),
        "ctr_mc_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


class CtraceError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{ctr_status_string(status)}: {msg}")
        self.status = status


def ctr_version() -> str:
    return _lib.ctr_version().decode()


def ctr_status_string(status: int) -> str:
    return _lib.ctr_status_string(status).decode()


def ctr_last_error(ctx) -> str:
    return _lib.ctr_last_error(ctx).decode()


def _check(ctx, status):
    if status != CTR_OK:
        raise CtraceError(status, ctr_last_error(ctx) if ctx else "")


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def ctr_create(device: int, arena_ptr: int, arena_bytes: int, stream_ptr: int):
    out = ctypes.c_void_p()
    st = _lib.ctr_create(int(device), ctypes.c_void_p(arena_ptr), ctypes.c_size_t(arena_bytes),
                         ctypes.c_void_p(stream_ptr), ctypes.byref(out))
    if st != CTR_OK:
        raise CtraceError(st, "ctr_create failed")
    return out


def ctr_destroy(ctx) -> None:
    _lib.ctr_destroy(ctx)


def _opts(precision, kernel=CTR_KERNEL_AUTO, slices=0, flags=0):
    o = ctr_opts()
    o.precision = int(precision)
    o.kernel = int(kernel)
    o.slices = int(slices)
    o.flags = int(flags)
    return o


def ctr_set_impurity(ctx, table) -> None:
    """table: a SectorTable (dims, energies, next, blocks, beta, n_flavors, is_complex)."""
    nf, ns = int(table.n_flavors), int(table.n_sectors)
    dims = np.ascontiguousarray(table.dims, dtype=np.int32)
    energies = np.ascontiguousarray(np.concatenate(table.energies), dtype=np.float64)
    nxt = np.ascontiguousarray(table.next, dtype=np.int32).reshape(-1)
    cdt = np.complex128 if table.is_complex else np.float64
    keep = []
    ptrs = (ctypes.c_void_p * (ns * nf))()
    for q in range(ns):
        for f in range(nf):
            B = table.blocks[q][f]
            if B is None:
                ptrs[q * nf + f] = None
            else:
                arr = np.ascontiguousarray(B, dtype=cdt)
                keep.append(arr)
                ptrs[q * nf + f] = arr.ctypes.data
    imp = ctr_impurity()
    imp.beta = float(table.beta)
    imp.n_flavors = nf
    imp.n_sectors = ns
    imp.is_complex = 1 if table.is_complex else 0
    imp.reserved = 0
    imp.sector_dim = _ptr(dims, ctypes.c_int32)
    imp.energies = _ptr(energies, ctypes.c_double)
    imp.next = _ptr(nxt, ctypes.c_int32)
    imp.blocks = ptrs
    imp.block_norm = None
    _check(ctx, _lib.ctr_set_impurity(ctx, ctypes.byref(imp)))


def ctr_arena_resident_bytes(ctx) -> int:
    return int(_lib.ctr_arena_resident_bytes(ctx))


def _string_arrays(tau, op):
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    op = np.ascontiguousarray(op, dtype=np.int32)
    if tau.shape != op.shape:
        raise ValueError("tau and op differ in length")
    return tau, op


def ctr_trace(ctx, tau, op, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO):
    tau, op = _string_arrays(tau, op)
    v = ctr_value()
    o = _opts(precision, kernel)
    _check(ctx, _lib.ctr_trace(ctx, int(op.size), _ptr(tau, ctypes.c_double), _ptr(op, ctypes.c_int32),
                               ctypes.byref(o), ctypes.byref(v)))
    return np.array([(v.re, v.im, v.log_scale, v.log_bound, v.log_abs, v.n_strings, v.flags)], dtype=VALUE_DTYPE)[0]


def ctr_trace_batch(ctx, offsets, tau, op, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO, slices=0, flags=0):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    tau, op = _string_arrays(tau, op)
    n = offsets.size - 1
    out = np.zeros(n, dtype=VALUE_DTYPE)
    o = _opts(precision, kernel, slices, flags)
    _check(ctx, _lib.ctr_trace_batch(ctx, n, _ptr(offsets, ctypes.c_int64), _ptr(tau, ctypes.c_double),
                                     _ptr(op, ctypes.c_int32), ctypes.byref(o),
                                     out.ctypes.data_as(ctypes.POINTER(ctr_value))))
    return out


def ctr_trace_batch_device(ctx, n_cfg, d_offsets_ptr, d_tau_ptr, d_op_ptr, d_out_ptr, precision=CTR_FP64,
                           kernel=CTR_KERNEL_AUTO, slices=0, flags=0):
    """Device pointers (ints); enqueues on the context's stream."""
    o = _opts(precision, kernel, slices, flags)
    _check(ctx, _lib.ctr_trace_batch_device(ctx, int(n_cfg), ctypes.c_void_p(d_offsets_ptr),
                                            ctypes.c_void_p(d_tau_ptr), ctypes.c_void_p(d_op_ptr),
                                            ctypes.byref(o), ctypes.c_void_p(d_out_ptr)))


def ctr_trace_batch_device_static(ctx, n_cfg, d_offsets_ptr, d_tau_ptr, d_op_ptr, d_out_ptr, precision=CTR_FP64,
                                  kernel=CTR_KERNEL_AUTO, slices=0):
    """As ctr_trace_batch_device, per-call scratch in the library's fixed device array."""
    o = _opts(precision, kernel, slices)
    _check(ctx, _lib.ctr_trace_batch_device_static(ctx, int(n_cfg), ctypes.c_void_p(d_offsets_ptr),
                                                   ctypes.c_void_p(d_tau_ptr), ctypes.c_void_p(d_op_ptr),
                                                   ctypes.byref(o), ctypes.c_void_p(d_out_ptr)))


def ctr_trace_lazy_batch(ctx, offsets, tau, op, log_threshold, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    tau, op = _string_arrays(tau, op)
    thr = np.ascontiguousarray(log_threshold, dtype=np.float64)
    n = offsets.size - 1
    out = np.zeros(n, dtype=VALUE_DTYPE)
    o = _opts(precision, kernel)
    _check(ctx, _lib.ctr_trace_lazy_batch(ctx, n, _ptr(offsets, ctypes.c_int64), _ptr(tau, ctypes.c_double),
                                          _ptr(op, ctypes.c_int32), _ptr(thr, ctypes.c_double), ctypes.byref(o),
                                          out.ctypes.data_as(ctypes.POINTER(ctr_value))))
    return out


def ctr_trace_lazy(ctx, tau, op, log_threshold, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO):
    tau, op = _string_arrays(tau, op)
    v = ctr_value()
    o = _opts(precision, kernel)
    _check(ctx, _lib.ctr_trace_lazy(ctx, int(op.size), _ptr(tau, ctypes.c_double), _ptr(op, ctypes.c_int32),
                                    float(log_threshold), ctypes.byref(o), ctypes.byref(v)))
    return np.array([(v.re, v.im, v.log_scale, v.log_bound, v.log_abs, v.n_strings, v.flags)], dtype=VALUE_DTYPE)[0]


def ctr_trace_histogram(ctx, offsets, tau, op, sector_label, n_labels, precision=CTR_FP64,
                        kernel=CTR_KERNEL_AUTO, slices=0):
    """(values [n_cfg] VALUE_DTYPE, hist [n_cfg, n_labels] complex128)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    tau, op = _string_arrays(tau, op)
    lab = np.ascontiguousarray(sector_label, dtype=np.int32)
    n = offsets.size - 1
    out = np.zeros(n, dtype=VALUE_DTYPE)
    hist = np.zeros((max(n, 0), int(n_labels)), dtype=np.complex128)
    o = _opts(precision, kernel, slices)
    _check(ctx, _lib.ctr_trace_histogram(ctx, n, _ptr(offsets, ctypes.c_int64), _ptr(tau, ctypes.c_double),
                                         _ptr(op, ctypes.c_int32), _ptr(lab, ctypes.c_int32), int(n_labels),
                                         ctypes.byref(o), out.ctypes.data_as(ctypes.POINTER(ctr_value)),
                                         hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out, hist


def ctr_density_matrix(ctx, offsets, tau, op, sector_dims, weight=None):
    """(values [n_cfg] VALUE_DTYPE, list of per-sector complex blocks sum_C weight_C R(C))."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    tau, op = _string_arrays(tau, op)
    n = offsets.size - 1
    dims = [int(d) for d in sector_dims]
    out = np.zeros(n, dtype=VALUE_DTYPE)
    rho = np.zeros(sum(d * d for d in dims), dtype=np.complex128)
    w = None if weight is None else np.ascontiguousarray(weight, dtype=np.complex128)
    if w is not None and w.shape != (n,):
        raise ValueError("one weight per configuration")
    _check(ctx, _lib.ctr_density_matrix(ctx, n, _ptr(offsets, ctypes.c_int64), _ptr(tau, ctypes.c_double),
                                        _ptr(op, ctypes.c_int32),
                                        w.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                                        if w is not None else None,
                                        out.ctypes.data_as(ctypes.POINTER(ctr_value)),
                                        rho.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    blocks, o = [], 0
    for d in dims:
        blocks.append(rho[o:o + d * d].reshape(d, d))
        o += d * d
    return out, blocks


def ctr_bound(ctx, tau, op) -> float:
    tau, op = _string_arrays(tau, op)
    lb = ctypes.c_double()
    _check(ctx, _lib.ctr_bound(ctx, int(op.size), _ptr(tau, ctypes.c_double), _ptr(op, ctypes.c_int32),
                               ctypes.byref(lb)))
    return float(lb.value)


def ctr_strings(ctx, op, n_sectors: int):
    op = np.ascontiguousarray(op, dtype=np.int32)
    q0 = np.zeros(max(n_sectors, 1), dtype=np.int32)
    n = ctypes.c_int32()
    _check(ctx, _lib.ctr_strings(ctx, int(op.size), _ptr(op, ctypes.c_int32), _ptr(q0, ctypes.c_int32),
                                 ctypes.byref(n)))
    return q0[: n.value].copy()


def ctr_probe_peaks(ctx):
    """Measured TFLOP/s of FP64 MFMA 16x16x4 and 4x4x4, FP32 MFMA 16x16x4; clock MHz; compute units."""
    out = np.zeros(5)
    _check(ctx, _lib.ctr_probe_peaks(ctx, _ptr(out, ctypes.c_double)))
    return {"fp64_mfma_16x16x4_tflops": float(out[0]), "fp64_mfma_4x4x4_tflops": float(out[1]),
            "fp32_mfma_16x16x4_tflops": float(out[2]), "clock_mhz": float(out[3]), "compute_units": int(out[4])}


def ctr_last_kernel(ctx):
    """(CTR_KERNEL_* the last trace call ran, FP32-split slices or 0)."""
    k, sl = ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, _lib.ctr_last_kernel(ctx, ctypes.byref(k), ctypes.byref(sl)))
    return int(k.value), int(sl.value)


def ctr_synchronize(ctx) -> None:
    _check(ctx, _lib.ctr_synchronize(ctx))


def ctr_kernel_timing(ctx, on: bool) -> None:
    _check(ctx, _lib.ctr_kernel_timing(ctx, 1 if on else 0))


def ctr_kernel_timing_read(ctx):
    """(summed chain-kernel milliseconds, number of launches) since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int32()
    _check(ctx, _lib.ctr_kernel_timing_read(ctx, ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def ctr_tune(ctx, offsets, tau, op):
    """Times every applicable FP64 chain kernel on the sample; returns
    (chosen CTR_KERNEL_*, {kernel: milliseconds})."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    tau, op = _string_arrays(tau, op)
    chosen = ctypes.c_int32()
    ms = np.full(5, -1.0)
    _check(ctx, _lib.ctr_tune(ctx, offsets.size - 1, _ptr(offsets, ctypes.c_int64), _ptr(tau, ctypes.c_double),
                              _ptr(op, ctypes.c_int32), ctypes.byref(chosen), _ptr(ms, ctypes.c_double)))
    return int(chosen.value), {k: float(ms[k]) for k in range(1, 5) if ms[k] >= 0}


def ctr_server_create(ctxs, max_batch: int = 4096, max_pending: int = 1 << 20, hbm_budget: int = 0,
                      grid_share=None, max_pass_flop: float = 0.0):
    """grid_share: optional per-context fractions in (0, 1] of each persistent grid."""
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    share = None if grid_share is None else np.ascontiguousarray(grid_share, dtype=np.float64)
    if share is not None and share.size != len(ctxs):
        raise ValueError("one grid share per context")
    o = ctr_server_opts(int(max_batch), int(max_pending), int(hbm_budget),
                        _ptr(share, ctypes.c_double) if share is not None else None, float(max_pass_flop))
    out = ctypes.c_void_p()
    st = _lib.ctr_server_create(arr, len(ctxs), ctypes.byref(o), ctypes.byref(out))
    if st != CTR_OK:
        raise CtraceError(st, "ctr_server_create failed")
    return out


def ctr_server_submit(srv, impurity: int, tag: int, tau, op, log_threshold: float = -math.inf) -> int:
    """Returns the status (CTR_OK or CTR_ERR_BUSY); raises on any other error."""
    tau, op = _string_arrays(tau, op)
    st = _lib.ctr_server_submit(srv, int(impurity), int(tag), int(op.size), _ptr(tau, ctypes.c_double),
                                _ptr(op, ctypes.c_int32), float(log_threshold))
    if st not in (CTR_OK, CTR_ERR_BUSY):
        raise CtraceError(st, "ctr_server_submit")
    return st


def ctr_server_poll(srv, max_results: int = 4096, wait: bool = False) -> np.ndarray:
    out = np.zeros(max_results, dtype=RESULT_DTYPE)
    n = ctypes.c_int32()
    st = _lib.ctr_server_poll(srv, out.ctypes.data, int(max_results), ctypes.byref(n), 1 if wait else 0)
    if st != CTR_OK:
        raise CtraceError(st, "ctr_server_poll")
    return out[: n.value]


def ctr_server_drain(srv) -> None:
    st = _lib.ctr_server_drain(srv)
    if st != CTR_OK:
        raise CtraceError(st, "ctr_server_drain")


def ctr_server_stats(srv):
    """(device passes, requests evaluated)."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    st = _lib.ctr_server_stats(srv, ctypes.byref(a), ctypes.byref(b))
    if st != CTR_OK:
        raise CtraceError(st, "ctr_server_stats")
    return int(a.value), int(b.value)


def ctr_server_destroy(srv) -> None:
    _lib.ctr_server_destroy(srv)


def ctr_mc_create(ctx, n_chains, bath_eps, bath_v, rebuild_every=0, full_traces=False):
    """bath_eps, bath_v: [n_flavors, n_bath] arrays."""
    eps = np.ascontiguousarray(bath_eps, dtype=np.float64)
    v = np.ascontiguousarray(bath_v, dtype=np.float64)
    o = ctr_mc_opts(int(n_chains), int(eps.shape[1]) if eps.ndim == 2 else 0, _ptr(eps, ctypes.c_double),
                    _ptr(v, ctypes.c_double), int(rebuild_every), 1 if full_traces else 0)
    out = ctypes.c_void_p()
    _check(ctx, _lib.ctr_mc_create(ctx, ctypes.byref(o), ctypes.byref(out)))
    return out


def ctr_mc_set_config(mc, chain, tau, op):
    tau, op = _string_arrays(tau, op)
    _check(None, _lib.ctr_mc_set_config(mc, int(chain), int(op.size), _ptr(tau, ctypes.c_double),
                                        _ptr(op, ctypes.c_int32)))


def ctr_mc_step(mc, u, n_chains=None):
    """u: [n_chains, 6] uniforms in [0, 1); returns the decisions (int32 [n_chains]).
    The library reads n_chains x 6 values: a u of another shape raises ValueError
    when n_chains is given (MarkovChains.step always passes it)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    if u.ndim != 2 or u.shape[1] != 6 or (n_chains is not None and u.shape[0] != int(n_chains)):
        raise ValueError(f"u must have shape (n_chains, 6), got {u.shape}")
    dec = np.zeros(u.shape[0], dtype=np.int32)
    _check(None, _lib.ctr_mc_step(mc, _ptr(u, ctypes.c_double), _ptr(dec, ctypes.c_int32)))
    return dec


def ctr_mc_config(mc, chain, cap=512):
    """(tau, op, log|w_loc|, log|w_hyb|) of one chain."""
    tau = np.zeros(cap)
    op = np.zeros(cap, dtype=np.int32)
    n = ctypes.c_int32()
    lw = np.zeros(2)
    _check(None, _lib.ctr_mc_config(mc, int(chain), int(cap), _ptr(tau, ctypes.c_double), _ptr(op, ctypes.c_int32),
                                    ctypes.byref(n), _ptr(lw, ctypes.c_double)))
    return tau[: n.value].copy(), op[: n.value].copy(), float(lw[0]), float(lw[1])


def ctr_mc_stats(mc):
    v = [ctypes.c_int64() for _ in range(4)]
    _check(None, _lib.ctr_mc_stats(mc, *[ctypes.byref(x) for x in v]))
    return {"steps": v[0].value, "proposed": v[1].value, "lazy_rejected": v[2].value, "accepted": v[3].value}


def ctr_mc_timing(mc):
    """(host ms, trace ms) accumulated by ctr_mc_step."""
    h, t = ctypes.c_double(), ctypes.c_double()
    _check(None, _lib.ctr_mc_timing(mc, ctypes.byref(h), ctypes.byref(t)))
    return h.value, t.value


def ctr_mc_destroy(mc) -> None:
    _lib.ctr_mc_destroy(mc)


class MarkovChains:
    """Markov chains over one TraceContext's impurity with a discrete bath per flavor."""

    def __init__(self, context, n_chains, bath_eps, bath_v, rebuild_every=0, full_traces=False):
        self.context = context
        self.n_chains = int(n_chains)
        self.mc = ctr_mc_create(context.ctx, n_chains, bath_eps, bath_v, rebuild_every, full_traces)

    def set_config(self, chain, tau, op):
        ctr_mc_set_config(self.mc, chain, tau, op)

    def step(self, u):
        return ctr_mc_step(self.mc, u, self.n_chains)

    def config(self, chain):
        return ctr_mc_config(self.mc, chain)

    def stats(self):
        return ctr_mc_stats(self.mc)

    def timing(self):
        return ctr_mc_timing(self.mc)

    def close(self):
        if getattr(self, "mc", None):
            ctr_mc_destroy(self.mc)
            self.mc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TraceServer:
    """Continuous-batching server over TraceContexts (one worker per context)."""

    def __init__(self, contexts, max_batch: int = 4096, max_pending: int = 1 << 20, hbm_budget: int = 0,
                 grid_share=None, max_pass_flop: float = 0.0):
        self.contexts = list(contexts)
        self.srv = ctr_server_create([c.ctx for c in self.contexts], max_batch, max_pending, hbm_budget,
                                     grid_share, max_pass_flop)

    def submit(self, impurity, tag, tau, op, log_threshold=-math.inf):
        return ctr_server_submit(self.srv, impurity, tag, tau, op, log_threshold)

    def poll(self, max_results=4096, wait=False):
        return ctr_server_poll(self.srv, max_results, wait)

    def drain(self):
        ctr_server_drain(self.srv)

    def stats(self):
        return ctr_server_stats(self.srv)

    def close(self):
        if getattr(self, "srv", None):
            ctr_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def value_pair(v):
    """(mantissa, log_scale) of a ctr_value record, complex mantissa if im != 0."""
    m = complex(v["re"], v["im"]) if v["im"] != 0 else float(v["re"])
    return m, float(v["log_scale"])


class TraceContext:
    """A ctrace context with its arena and stream taken from PyTorch.

    stream: the torch.cuda.Stream the context enqueues on (default: the current
    stream).  Contexts served together by a TraceServer overlap on the device
    only when each has a stream of its own."""

    def __init__(self, table, arena_bytes: int | None = None, device: int = 0, scratch_bytes: int = 1 << 30,
                 stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the trace library runs on the GPU only")
        self.device = int(device)
        self.table = table
        if arena_bytes is None:
            arena_bytes = self.default_arena_bytes(table, scratch_bytes)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{self.device}")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = ctr_create(self.device, self.arena.data_ptr(), self.arena.numel(), self.stream.cuda_stream)
        ctr_set_impurity(self.ctx, table)

    @staticmethod
    def default_arena_bytes(table, scratch_bytes: int = 1 << 30) -> int:
        """Operator blocks and kernel buffers of `table` plus `scratch_bytes` of
        per-call scratch (batches larger than the scratch run in chunks)."""
        es = 16 if table.is_complex else 8
        blocks = 0
        d = np.asarray(table.dims)
        for q in range(table.n_sectors):
            for o in range(2 * table.n_flavors):
                t = table.next[q, o]
                if t >= 0:
                    blocks += ((int(d[t]) + 15) // 16 * 16) * ((int(d[q]) + 3) // 4 * 4) * es + 256
        xr = (int(d.max()) + 15) // 16 * 16
        stream_buffers = 2 * (2 if table.is_complex else 1) * xr * 16 * 8 * 1024
        return int(blocks + stream_buffers + scratch_bytes)

    def close(self):
        if getattr(self, "ctx", None):
            ctr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def trace(self, tau, op, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO):
        return ctr_trace(self.ctx, tau, op, precision, kernel)

    def trace_batch(self, strings, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO, slices=0):
        """strings: sequence of (tau, op) pairs or objects with .tau and .op."""
        taus = [np.asarray(getattr(s, "tau", s[0] if isinstance(s, tuple) else None), dtype=np.float64)
                for s in strings]
        ops = [np.asarray(getattr(s, "op", s[1] if isinstance(s, tuple) else None), dtype=np.int32)
               for s in strings]
        offs = np.zeros(len(strings) + 1, dtype=np.int64)
        offs[1:] = np.cumsum([o.size for o in ops])
        tau = np.concatenate(taus) if taus else np.zeros(0)
        op = np.concatenate(ops) if ops else np.zeros(0, np.int32)
        return ctr_trace_batch(self.ctx, offs, tau, op, precision, kernel, slices)

    def trace_packed(self, offsets, tau, op, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO, slices=0, flags=0):
        return ctr_trace_batch(self.ctx, offsets, tau, op, precision, kernel, slices, flags)

    def lazy_batch(self, offsets, tau, op, log_threshold, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO):
        return ctr_trace_lazy_batch(self.ctx, offsets, tau, op, log_threshold, precision, kernel)

    def lazy(self, tau, op, log_threshold, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO):
        return ctr_trace_lazy(self.ctx, tau, op, log_threshold, precision, kernel)

    def tune(self, offsets, tau, op):
        return ctr_tune(self.ctx, offsets, tau, op)

    def histogram(self, offsets, tau, op, sector_label, n_labels, precision=CTR_FP64, kernel=CTR_KERNEL_AUTO,
                  slices=0):
        return ctr_trace_histogram(self.ctx, offsets, tau, op, sector_label, n_labels, precision, kernel, slices)

    def density_matrix(self, offsets, tau, op, weight=None):
        return ctr_density_matrix(self.ctx, offsets, tau, op, self.table.dims, weight)

    def bound(self, tau, op) -> float:
        return ctr_bound(self.ctx, tau, op)

    def strings(self, op):
        return ctr_strings(self.ctx, op, self.table.n_sectors)

    def synchronize(self):
        ctr_synchronize(self.ctx)


def log_abs(v) -> float:
    """log|trace| of a ctr_value record (-inf for zero)."""
    a = math.hypot(float(v["re"]), float(v["im"]))
    return math.log(a) + float(v["log_scale"]) if a > 0 else -math.inf
