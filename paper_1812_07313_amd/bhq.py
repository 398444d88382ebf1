"""Thin ctypes binding of libbhq (include/bhq.h), same names as the C ABI.

Argument marshalling only: every step of the force evaluation runs in the
library's HIP kernels.  Non-zero return codes raise :class:`BhqError`.
The library is built in-tree by ``paper_1812_07313_amd.build`` and loaded
from this package directory; a missing or unloadable library is an error
(there is no fallback path).
"""
import ctypes
import os

import numpy as np

MONO, QUAD, SPLIT_QUAD, SPLIT_MONO, QUAD_SOFT = 0, 1, 2, 3, 4
FP32_OFS64, FP64 = 0, 1
ORDER_COST, ORDER_XCD = 0, 1
ORDER_WINDOW, ORDER_TAIL = 256, 1024
XCDS = 8

OK = 0
E_ARG, E_RANGE, E_NODEV, E_HIP, E_NOMEM, E_STATE, E_NONFINITE = (
    -1, -2, -3, -4, -5, -6, -7)

KERNEL_NAMES = {MONO: "mono", QUAD: "quad", SPLIT_QUAD: "split_quad",
                SPLIT_MONO: "split_mono", QUAD_SOFT: "quad_soft"}
PRECISION_NAMES = {FP32_OFS64: "fp32_ofs64", FP64: "fp64"}

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbhq.so")

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_P = ctypes.c_void_p

# name -> (restype, argtypes); every exported symbol of include/bhq.h
SIGNATURES = {
    "bhq_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int]),
    "bhq_destroy": (ctypes.c_int, [_P]),
    "bhq_set_kernel": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
    "bhq_set_eps": (ctypes.c_int, [_P, ctypes.c_double]),
    "bhq_set_eps2_i": (ctypes.c_int, [_P, ctypes.c_int64, _D]),
    "bhq_set_split": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double]),
    "bhq_set_groups": (ctypes.c_int, [_P, ctypes.c_int64, _I64, _D, _I64,
                                      _I64]),
    "bhq_set_i": (ctypes.c_int, [_P, ctypes.c_int64, _D]),
    "bhq_set_jp": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _D,
                                  _D]),
    "bhq_set_jc": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _D, _D,
                                  _D, _D]),
    "bhq_set_groups_dev": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P, _P, _P]),
    "bhq_set_i_dev": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P]),
    "bhq_set_eps2_i_dev": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P]),
    "bhq_set_jp_dev": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P, _P]),
    "bhq_set_jc_dev": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P, _P, _P,
                                      _P]),
    "bhq_set_pool_particles_dev": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P]),
    "bhq_set_pool_cells_dev": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P, _P, _P]),
    "bhq_set_jp_idx_dev": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P]),
    "bhq_set_jc_idx_dev": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P]),
    "bhq_count_live": (ctypes.c_int, [_P, _I64, _I64]),
    "bhq_clock_begin": (ctypes.c_int, [_P, ctypes.c_double, _P]),
    "bhq_clock_end": (ctypes.c_int, [_P, _D]),
    "bhq_compute": (ctypes.c_int, [_P, _P]),
    "bhq_compute_noalloc": (ctypes.c_int, [_P, _P, _P, _P]),
    "bhq_get_result": (ctypes.c_int, [_P, _D, _D]),
    "bhq_get_counts": (ctypes.c_int, [_P, _I64, _I64]),
    "bhq_get_kernel_ms": (ctypes.c_int, [_P, _D]),
    "bhq_last_error": (ctypes.c_char_p, [_P]),
    "bhq_set_tuning": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int]),
    "bhq_get_tuning": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)]),
    "bhq_set_group_order": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int]),
    "bhq_get_group_order": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)]),
    "bhq_get_order": (ctypes.c_int, [_P, _I32, ctypes.c_int64, _I64]),
    "bhq_get_build_info": (ctypes.c_int, [_P, _I64]),
    "bhq_plan_order": (ctypes.c_int, [ctypes.c_int64, _I64, _I64, _I64,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _I32, ctypes.c_int64,
                                      _I64]),
    "bhq_build_lists_batch": (ctypes.c_int, [ctypes.c_int64, _I64, _D, _D,
                                             ctypes.c_double, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(_P)]),
    "bhq_build_lists": (ctypes.c_int, [ctypes.c_int64, _D, _D,
                                       ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int,
                                       ctypes.POINTER(_P)]),
    "bhq_lists_sizes": (ctypes.c_int, [_P, _I64]),
    "bhq_lists_export": (ctypes.c_int, [_P, _I64, _I64, _D, _D, _I64, _I64,
                                        _I64, _I32]),
    "bhq_lists_cells": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "bhq_set_lists": (ctypes.c_int, [_P, _P, _D, _D]),
    "bhq_lists_free": (ctypes.c_int, [_P]),
    "bhq_set_pool_particles": (ctypes.c_int, [_P, ctypes.c_int64, _D, _D]),
    "bhq_set_pool_cells": (ctypes.c_int, [_P, ctypes.c_int64, _D, _D, _D, _D]),
    "bhq_set_jp_idx": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _I32]),
    "bhq_set_jc_idx": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _I32]),
    "bhq_set_lists_indexed": (ctypes.c_int, [_P, _P, _D, _D]),
    "bhq_build_lists_device": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P,
                                              ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_double,
                                              ctypes.c_double, _P]),
    "bhq_build_lists_device_batch": (ctypes.c_int, [_P, ctypes.c_int64, _I64, _P, _P, _P,
                                                    ctypes.c_double, ctypes.c_int,
                                                    ctypes.c_int, _P]),
    "bhq_get_lists_sizes": (ctypes.c_int, [_P, _I64]),
    "bhq_get_lists": (ctypes.c_int, [_P, _I64, _I64, _I64, _I64, _I64, _I32]),
    "bhq_get_cells": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "bhq_get_result_device": (ctypes.c_int, [_P, _P, _P, _P]),
    "bhq_kick_drift": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P,
                                      ctypes.c_double, ctypes.c_double, _P]),
    "bhq_energies": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P,
                                    ctypes.c_double, _D, _P]),
    "bhq_wrap_periodic": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_double, _P]),
    "bhq_sort_to_tree_order": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int,
                                               ctypes.POINTER(_P),
                                               ctypes.POINTER(ctypes.c_int), _P]),
    "bhq_pm_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double]),
    "bhq_pm_destroy": (ctypes.c_int, [_P]),
    "bhq_pm_compute": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P, _P, ctypes.c_int,
                                      _P]),
    "bhq_pm_get_ms": (ctypes.c_int, [_P, _D]),
    "bhq_pm_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


class BhqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libbhq error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load libbhq.so; build it first only if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        # PyTorch ships its own HIP runtime.  Importing it first lets libbhq
        # bind to that runtime, so the process runs one HIP runtime; a
        # second one started by libbhq before torch leaves torch without a
        # device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != OK:
        msg = lib().bhq_last_error(ctx)
        raise BhqError(rc, msg.decode() if msg else "")


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _ip(a):
    return None if a is None else a.ctypes.data_as(_I64)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


# --- contexts ---------------------------------------------------------------

def bhq_create(device=0, kernel=QUAD, precision=FP32_OFS64):
    h = _P()
    _check(lib().bhq_create(ctypes.byref(h), int(device), int(kernel),
                            int(precision)))
    return h


def bhq_destroy(ctx):
    _check(lib().bhq_destroy(ctx), ctx)


def bhq_set_kernel(ctx, kernel, precision):
    _check(lib().bhq_set_kernel(ctx, int(kernel), int(precision)), ctx)


def bhq_set_eps(ctx, eps):
    _check(lib().bhq_set_eps(ctx, float(eps)), ctx)


def bhq_set_eps2_i(ctx, eps2):
    e = _f64(eps2)
    _check(lib().bhq_set_eps2_i(ctx, e.shape[0], _dp(e)), ctx)


def bhq_set_split(ctx, rs, rcut, box=0.0):
    _check(lib().bhq_set_split(ctx, float(rs), float(rcut), float(box)), ctx)


def bhq_set_groups(ctx, i_off, center, jp_off, jc_off):
    i_off, jp_off, jc_off = _i64(i_off), _i64(jp_off), _i64(jc_off)
    ng = i_off.shape[0] - 1
    c = _f64(center, (-1, 3))
    if not (c.shape[0] == ng == jp_off.shape[0] - 1 == jc_off.shape[0] - 1):
        raise BhqError(E_ARG, "group array lengths disagree")
    _check(lib().bhq_set_groups(ctx, ng, _ip(i_off), _dp(c), _ip(jp_off),
                                _ip(jc_off)), ctx)


def bhq_set_i(ctx, x):
    x = _f64(x, (-1, 3))
    _check(lib().bhq_set_i(ctx, x.shape[0], _dp(x)), ctx)


def bhq_set_jp(ctx, adr, x, m):
    x = _f64(x, (-1, 3))
    m = _f64(m)
    if m.shape[0] != x.shape[0]:
        raise BhqError(E_ARG, "x and m lengths disagree")
    _check(lib().bhq_set_jp(ctx, int(adr), x.shape[0], _dp(x), _dp(m)), ctx)


def bhq_set_jc(ctx, adr, x, m, q, trace=None):
    x = _f64(x, (-1, 3))
    m = _f64(m)
    q = _f64(q, (-1, 6))
    t = None if trace is None else _f64(trace)
    n = x.shape[0]
    if m.shape[0] != n or q.shape[0] != n or (t is not None and t.shape[0] != n):
        raise BhqError(E_ARG, "j-cell array lengths disagree")
    _check(lib().bhq_set_jc(ctx, int(adr), n, _dp(x), _dp(m), _dp(q), _dp(t)),
           ctx)


def bhq_set_pool_particles(ctx, x, m):
    x = _f64(x, (-1, 3))
    m = _f64(m)
    if m.shape[0] != x.shape[0]:
        raise BhqError(E_ARG, "x and m lengths disagree")
    _check(lib().bhq_set_pool_particles(ctx, x.shape[0], _dp(x), _dp(m)), ctx)


def bhq_set_pool_cells(ctx, x, m, q, trace=None):
    x = _f64(x, (-1, 3))
    m = _f64(m)
    q = _f64(q, (-1, 6))
    t = None if trace is None else _f64(trace)
    n = x.shape[0]
    if m.shape[0] != n or q.shape[0] != n or (t is not None and t.shape[0] != n):
        raise BhqError(E_ARG, "cell pool array lengths disagree")
    _check(lib().bhq_set_pool_cells(ctx, n, _dp(x), _dp(m), _dp(q), _dp(t)), ctx)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def bhq_set_jp_idx(ctx, adr, idx):
    i = _i32(idx)
    _check(lib().bhq_set_jp_idx(ctx, int(adr), i.shape[0],
                                i.ctypes.data_as(_I32)), ctx)


def bhq_set_jc_idx(ctx, adr, idx):
    i = _i32(idx)
    _check(lib().bhq_set_jc_idx(ctx, int(adr), i.shape[0],
                                i.ctypes.data_as(_I32)), ctx)


def bhq_compute(ctx, stream=None):
    _check(lib().bhq_compute(ctx, _stream_handle(stream)), ctx)


def bhq_compute_noalloc(ctx, a, pot=None, stream=None):
    """Force evaluation into caller GPU tensors a (ni, 3) and pot (ni,) or
    None, float64, group order; allocates nothing."""
    n = int(a.shape[0])
    pa = _device_ptr(a, (n, 3), "a")
    pp = None if pot is None else _device_ptr(pot, (n,), "pot")
    _check(lib().bhq_compute_noalloc(ctx, pa, pp, _stream_handle(stream)), ctx)


def bhq_count_live(ctx):
    """(particle pairs, cell pairs) of the split kernels' lists inside the
    cutoff."""
    pp, pc = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().bhq_count_live(ctx, ctypes.byref(pp), ctypes.byref(pc)), ctx)
    return pp.value, pc.value


def bhq_clock_begin(ctx, wall_ms, stream=None):
    _check(lib().bhq_clock_begin(ctx, float(wall_ms), _stream_handle(stream)), ctx)


def bhq_clock_end(ctx):
    mhz = ctypes.c_double()
    _check(lib().bhq_clock_end(ctx, ctypes.byref(mhz)), ctx)
    return mhz.value


def bhq_get_result(ctx, ni):
    a = np.zeros((ni, 3))
    pot = np.zeros(ni)
    _check(lib().bhq_get_result(ctx, _dp(a), _dp(pot)), ctx)
    return a, pot


def bhq_get_counts(ctx):
    pp, pc = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().bhq_get_counts(ctx, ctypes.byref(pp), ctypes.byref(pc)), ctx)
    return pp.value, pc.value


def bhq_get_kernel_ms(ctx):
    ms = ctypes.c_double()
    _check(lib().bhq_get_kernel_ms(ctx, ctypes.byref(ms)), ctx)
    return ms.value


def bhq_set_tuning(ctx, block=256, i_per_thread=2, blocks_per_cu=0,
                   persistent=0, use_graph=0, jsplit=1, waves_per_eu=0):
    _check(lib().bhq_set_tuning(ctx, int(block), int(i_per_thread),
                                int(blocks_per_cu), int(persistent),
                                int(use_graph), int(jsplit), int(waves_per_eu)), ctx)


def bhq_get_tuning(ctx):
    out = (ctypes.c_int * 7)()
    _check(lib().bhq_get_tuning(ctx, out), ctx)
    return dict(block=out[0], i_per_thread=out[1], blocks_per_cu=out[2],
                persistent=out[3], use_graph=out[4], jsplit=out[5],
                waves_per_eu=out[6])


def bhq_set_group_order(ctx, mode=ORDER_XCD, window=ORDER_WINDOW,
                        tail=ORDER_TAIL):
    _check(lib().bhq_set_group_order(ctx, int(mode), int(window), int(tail)),
           ctx)


def bhq_get_group_order(ctx):
    out = (ctypes.c_int * 3)()
    _check(lib().bhq_get_group_order(ctx, out), ctx)
    return dict(mode=out[0], window=out[1], tail=out[2])


def bhq_get_build_info(ctx):
    """(one_walk, longest particle list, longest cell list) of the last
    device build."""
    out = np.zeros(3, np.int64)
    _check(lib().bhq_get_build_info(ctx, _ip(out)), ctx)
    return bool(out[0]), int(out[1]), int(out[2])


def bhq_get_order(ctx):
    """The launch slot table in use (int32, -1 for empty slots)."""
    n = ctypes.c_int64()
    _check(lib().bhq_get_order(ctx, None, 0, ctypes.byref(n)), ctx)
    out = np.zeros(n.value, np.int32)
    _check(lib().bhq_get_order(ctx, out.ctypes.data_as(_I32), out.shape[0],
                               ctypes.byref(n)), ctx)
    return out


def bhq_plan_order(i_off, jp_off, jc_off, mode=ORDER_XCD, window=ORDER_WINDOW,
                   tail=ORDER_TAIL, xcds=XCDS):
    """Slot table of a group dispatch order: order[b] = group of launch
    slot b, -1 for an empty slot."""
    i_off, jp_off, jc_off = _i64(i_off), _i64(jp_off), _i64(jc_off)
    ng = i_off.shape[0] - 1
    n = ctypes.c_int64()
    args = (ng, _ip(i_off), _ip(jp_off), _ip(jc_off), int(mode), int(window),
            int(tail), int(xcds))
    _check(lib().bhq_plan_order(*args, None, 0, ctypes.byref(n)))
    out = np.empty(n.value, dtype=np.int32)
    _check(lib().bhq_plan_order(*args, out.ctypes.data_as(_I32), out.shape[0],
                                ctypes.byref(n)))
    return out


def bhq_last_error(ctx=None):
    msg = lib().bhq_last_error(ctx)
    return msg.decode() if msg else ""


# --- host list builder --------------------------------------------------------

def bhq_build_lists(x, m, theta, ncrit, nleaf=8, box=0.0, rcut=0.0,
                    nthreads=0):
    x = _f64(x, (-1, 3))
    m = _f64(m)
    h = _P()
    _check(lib().bhq_build_lists(x.shape[0], _dp(x), _dp(m), float(theta),
                                 int(ncrit), int(nleaf), float(box),
                                 float(rcut), int(nthreads), ctypes.byref(h)))
    return h


def bhq_build_lists_batch(sys_off, x, m, theta, ncrit, nleaf=8, nthreads=0):
    off = _i64(sys_off)
    x = _f64(x, (-1, 3))
    m = _f64(m)
    h = _P()
    _check(lib().bhq_build_lists_batch(off.shape[0] - 1, _ip(off), _dp(x),
                                       _dp(m), float(theta), int(ncrit),
                                       int(nleaf), int(nthreads),
                                       ctypes.byref(h)))
    return h


def bhq_lists_sizes(L):
    s = np.zeros(4, np.int64)
    _check(lib().bhq_lists_sizes(L, _ip(s)))
    return tuple(int(v) for v in s)


def bhq_lists_export(L, n):
    ng, njp, njc, _ = bhq_lists_sizes(L)
    out = dict(i_idx=np.zeros(n, np.int64), i_off=np.zeros(ng + 1, np.int64),
               center=np.zeros((ng, 3)), side=np.zeros(ng),
               jp_off=np.zeros(ng + 1, np.int64), jp_idx=np.zeros(njp, np.int64),
               jc_off=np.zeros(ng + 1, np.int64),
               jc_cell=np.zeros(njc, np.int32))
    _check(lib().bhq_lists_export(
        L, _ip(out["i_idx"]), _ip(out["i_off"]), _dp(out["center"]),
        _dp(out["side"]), _ip(out["jp_off"]), _ip(out["jp_idx"]),
        _ip(out["jc_off"]), out["jc_cell"].ctypes.data_as(_I32)))
    return out


def bhq_lists_cells(L):
    nc = bhq_lists_sizes(L)[3]
    out = dict(com=np.zeros((nc, 3)), mass=np.zeros(nc), q=np.zeros((nc, 6)),
               trace=np.zeros(nc))
    _check(lib().bhq_lists_cells(L, _dp(out["com"]), _dp(out["mass"]),
                                 _dp(out["q"]), _dp(out["trace"])))
    return out


def bhq_set_lists(ctx, L, x, m):
    x = _f64(x, (-1, 3))
    m = _f64(m)
    _check(lib().bhq_set_lists(ctx, L, _dp(x), _dp(m)), ctx)


def bhq_set_lists_indexed(ctx, L, x, m):
    x = _f64(x, (-1, 3))
    m = _f64(m)
    _check(lib().bhq_set_lists_indexed(ctx, L, _dp(x), _dp(m)), ctx)


def bhq_lists_free(L):
    _check(lib().bhq_lists_free(L))


# --- device list builder -------------------------------------------------------

def _device_ptr(t, shape, name):
    """Address of a contiguous float64 GPU tensor of the given shape."""
    if not (hasattr(t, "is_cuda") and t.is_cuda):
        raise TypeError("%s must be a GPU tensor" % name)
    if str(t.dtype) != "torch.float64" or not t.is_contiguous():
        raise TypeError("%s must be a contiguous float64 tensor" % name)
    if tuple(t.shape) != shape:
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), shape))
    return t.data_ptr()


def _dev_arg(t, shape, dtype, name):
    """Address of a contiguous GPU tensor of the given dtype ("float64",
    "int64", "int32") and shape, or None for t None."""
    if t is None:
        return None
    if not (hasattr(t, "is_cuda") and t.is_cuda):
        raise TypeError("%s must be a GPU tensor" % name)
    if str(t.dtype) != "torch." + dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (name, dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t.data_ptr()


def bhq_set_groups_dev(ctx, i_off, center, jp_off, jc_off, stream=None):
    """Offsets (ng+1,) int64 and centres (ng, 3) float64 GPU tensors."""
    ng = int(center.shape[0])
    _check(lib().bhq_set_groups_dev(
        ctx, ng, _dev_arg(i_off, (ng + 1,), "int64", "i_off"),
        _dev_arg(center, (ng, 3), "float64", "center"),
        _dev_arg(jp_off, (ng + 1,), "int64", "jp_off"),
        _dev_arg(jc_off, (ng + 1,), "int64", "jc_off"), _stream_handle(stream)), ctx)


def bhq_set_i_dev(ctx, x, stream=None):
    n = int(x.shape[0])
    _check(lib().bhq_set_i_dev(ctx, n, _dev_arg(x, (n, 3), "float64", "x"),
                               _stream_handle(stream)), ctx)


def bhq_set_eps2_i_dev(ctx, eps2, stream=None):
    n = int(eps2.shape[0])
    _check(lib().bhq_set_eps2_i_dev(ctx, n, _dev_arg(eps2, (n,), "float64", "eps2"),
                                    _stream_handle(stream)), ctx)


def bhq_set_jp_dev(ctx, adr, x, m, stream=None):
    n = int(m.shape[0])
    _check(lib().bhq_set_jp_dev(ctx, int(adr), n, _dev_arg(x, (n, 3), "float64", "x"),
                                _dev_arg(m, (n,), "float64", "m"), _stream_handle(stream)),
           ctx)


def bhq_set_jc_dev(ctx, adr, x, m, q, trace=None, stream=None):
    n = int(m.shape[0])
    _check(lib().bhq_set_jc_dev(ctx, int(adr), n, _dev_arg(x, (n, 3), "float64", "x"),
                                _dev_arg(m, (n,), "float64", "m"),
                                _dev_arg(q, (n, 6), "float64", "q"),
                                _dev_arg(trace, (n,), "float64", "trace"),
                                _stream_handle(stream)), ctx)


def bhq_set_pool_particles_dev(ctx, x, m, stream=None):
    n = int(m.shape[0])
    _check(lib().bhq_set_pool_particles_dev(ctx, n, _dev_arg(x, (n, 3), "float64", "x"),
                                            _dev_arg(m, (n,), "float64", "m"),
                                            _stream_handle(stream)), ctx)


def bhq_set_pool_cells_dev(ctx, x, m, q, trace=None, stream=None):
    n = int(m.shape[0])
    _check(lib().bhq_set_pool_cells_dev(ctx, n, _dev_arg(x, (n, 3), "float64", "x"),
                                        _dev_arg(m, (n,), "float64", "m"),
                                        _dev_arg(q, (n, 6), "float64", "q"),
                                        _dev_arg(trace, (n,), "float64", "trace"),
                                        _stream_handle(stream)), ctx)


def bhq_set_jp_idx_dev(ctx, adr, idx, stream=None):
    n = int(idx.shape[0])
    _check(lib().bhq_set_jp_idx_dev(ctx, int(adr), n, _dev_arg(idx, (n,), "int32", "idx"),
                                    _stream_handle(stream)), ctx)


def bhq_set_jc_idx_dev(ctx, adr, idx, stream=None):
    n = int(idx.shape[0])
    _check(lib().bhq_set_jc_idx_dev(ctx, int(adr), n, _dev_arg(idx, (n,), "int32", "idx"),
                                    _stream_handle(stream)), ctx)


def bhq_build_lists_device(ctx, x, m, theta, ncrit, nleaf=8, box=0.0, rcut=0.0,
                           stream=None):
    """x: (n, 3) and m: (n,) float64 torch tensors on the context's GPU."""
    n = int(m.shape[0])
    px = _device_ptr(x, (n, 3), "x")
    pm = _device_ptr(m, (n,), "m")
    _check(lib().bhq_build_lists_device(ctx, n, px, pm, float(theta), int(ncrit),
                                        int(nleaf), float(box), float(rcut),
                                        _stream_handle(stream)), ctx)


def bhq_build_lists_device_batch(ctx, sys_off, x, m, theta, ncrit, nleaf=8, eps2=None,
                                 stream=None):
    """Independent systems (host sys_off[nsys+1]); x, m, eps2 (optional)
    GPU tensors in input order."""
    so = _i64(sys_off)
    nsys = so.shape[0] - 1
    n = int(m.shape[0])
    _check(lib().bhq_build_lists_device_batch(
        ctx, nsys, _ip(so), _device_ptr(x, (n, 3), "x"), _device_ptr(m, (n,), "m"),
        None if eps2 is None else _device_ptr(eps2, (n,), "eps2"), float(theta),
        int(ncrit), int(nleaf), _stream_handle(stream)), ctx)


def bhq_get_lists_sizes(ctx):
    out = np.zeros(4, np.int64)
    _check(lib().bhq_get_lists_sizes(ctx, _ip(out)), ctx)
    return tuple(int(v) for v in out)


def bhq_get_lists(ctx, n=None):
    """The context's index lists on the host (bhq_lists_export's layout);
    i_idx only when n (the particle count) is given."""
    ng, njp, njc, _ = bhq_get_lists_sizes(ctx)
    out = dict(i_off=np.zeros(ng + 1, np.int64), jp_off=np.zeros(ng + 1, np.int64),
               jp_idx=np.zeros(njp, np.int64), jc_off=np.zeros(ng + 1, np.int64),
               jc_cell=np.zeros(njc, np.int32))
    if n is not None:
        out["i_idx"] = np.zeros(n, np.int64)
    _check(lib().bhq_get_lists(
        ctx, _ip(out.get("i_idx")), _ip(out["i_off"]), _ip(out["jp_off"]),
        _ip(out["jp_idx"]), _ip(out["jc_off"]),
        out["jc_cell"].ctypes.data_as(_I32)), ctx)
    return out


def bhq_get_cells(ctx):
    nc = bhq_get_lists_sizes(ctx)[3]
    out = dict(com=np.zeros((nc, 3)), mass=np.zeros(nc), q=np.zeros((nc, 6)),
               trace=np.zeros(nc))
    _check(lib().bhq_get_cells(ctx, _dp(out["com"]), _dp(out["mass"]),
                               _dp(out["q"]), _dp(out["trace"])), ctx)
    return out


# --- time-step helpers (device arrays as torch tensors) ------------------------

def _dptr(t, shape, name):
    return None if t is None else _device_ptr(t, shape, name)


def bhq_get_result_device(ctx, a, pot=None, stream=None):
    """a: (n, 3) float64 GPU tensor, pot: (n,) or None; input order."""
    n = int(a.shape[0])
    _check(lib().bhq_get_result_device(ctx, _dptr(a, (n, 3), "a"),
                                       _dptr(pot, (n,), "pot"),
                                       _stream_handle(stream)), ctx)


def bhq_kick_drift(ctx, x, v, a, dt_kick, dt_drift, stream=None):
    n = int(v.shape[0])
    _check(lib().bhq_kick_drift(ctx, n, _dptr(x, (n, 3), "x"),
                                _dptr(v, (n, 3), "v"), _dptr(a, (n, 3), "a"),
                                float(dt_kick), float(dt_drift),
                                _stream_handle(stream)), ctx)


def bhq_wrap_periodic(ctx, x, box, stream=None):
    n = int(x.shape[0])
    _check(lib().bhq_wrap_periodic(ctx, n, _dptr(x, (n, 3), "x"), float(box),
                                   _stream_handle(stream)), ctx)


def bhq_sort_to_tree_order(ctx, fields, stream=None):
    """Permute GPU tensors (each with n rows of 8 to 64 bytes, contiguous,
    8-byte elements) in place into the tree order of the current lists."""
    fields = list(fields)
    if not fields:
        raise ValueError("no fields")
    n = int(fields[0].shape[0])
    ptrs, rb = [], []
    for k, t in enumerate(fields):
        if not (hasattr(t, "is_cuda") and t.is_cuda) or not t.is_contiguous():
            raise TypeError("field %d must be a contiguous GPU tensor" % k)
        if int(t.shape[0]) != n or t.element_size() != 8:
            raise ValueError("field %d must have %d rows of 8-byte elements" % (k, n))
        ptrs.append(t.data_ptr())
        rb.append(int(t.numel() // max(n, 1)) * 8)
    arr = (_P * len(ptrs))(*ptrs)
    rba = (ctypes.c_int * len(rb))(*rb)
    _check(lib().bhq_sort_to_tree_order(ctx, n, len(ptrs), arr, rba,
                                        _stream_handle(stream)), ctx)


def bhq_energies(ctx, m, v, pot=None, eps=0.0, stream=None):
    """(K, W) with W = 1/2 sum m (pot + m/eps); W = 0 without pot."""
    n = int(m.shape[0])
    out = np.zeros(2)
    _check(lib().bhq_energies(ctx, n, _dptr(m, (n,), "m"), _dptr(v, (n, 3), "v"),
                              _dptr(pot, (n,), "pot"), float(eps), _dp(out),
                              _stream_handle(stream)), ctx)
    return float(out[0]), float(out[1])


# --- particle-mesh long-range force ----------------------------------------------

def _pm_check(rc, pm=None):
    if rc != OK:
        msg = lib().bhq_pm_last_error(pm)
        raise BhqError(rc, msg.decode() if msg else "")


def bhq_pm_create(nmesh, box, rs, device=0):
    h = _P()
    _pm_check(lib().bhq_pm_create(ctypes.byref(h), int(device), int(nmesh), float(box),
                                  float(rs)))
    return h


def bhq_pm_destroy(pm):
    _pm_check(lib().bhq_pm_destroy(pm), pm)


def bhq_pm_compute(pm, x, m, a, pot=None, accumulate=False, stream=None):
    """x, a: (n, 3), m, pot: (n,) float64 GPU tensors."""
    n = int(m.shape[0])
    _pm_check(lib().bhq_pm_compute(pm, n, _dptr(x, (n, 3), "x"), _dptr(m, (n,), "m"),
                                   _dptr(a, (n, 3), "a"), _dptr(pot, (n,), "pot"),
                                   int(bool(accumulate)), _stream_handle(stream)), pm)


def bhq_pm_get_ms(pm):
    ms = ctypes.c_double()
    _pm_check(lib().bhq_pm_get_ms(pm, ctypes.byref(ms)), pm)
    return ms.value
