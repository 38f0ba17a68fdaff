"""ctypes wrapper around the plain serial C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and this package never imports the GPU library.

Every function takes and returns numpy arrays; see ``oracle.h`` for the
definitions and the paper passages each one follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

NPARAM = 32 + 32 + 32 * 32 + 32 + 32 + 1
H = 32


_STAMP = _SO + ".cpu"


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc -O2 -march=native
    (the paper's flags, Section 4).  -march=native ties the library to the
    host CPU, so it is rebuilt when loaded on a different CPU model."""
    src = os.path.join(_HERE, "oracle.c")
    stale = (not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src)
             or not os.path.exists(_STAMP) or open(_STAMP).read() != _cpu_model())
    if force or stale:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-march=native", "-std=c99", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
        with open(_STAMP, "w") as f:
            f.write(_cpu_model())
    return _SO


class Counters(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("stages", ctypes.c_int64),
                ("merge_splits", ctypes.c_int64), ("local_sorts", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        vp, sz, i, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int64
        cp = ctypes.POINTER(Counters)
        dp = ctypes.POINTER(ctypes.c_double)
        L.o_count_round.argtypes = [vp, vp, vp, vp, sz, i, i, vp]
        L.o_lsd.argtypes = [vp, vp, vp, vp, sz, i, i, i, vp, cp]
        L.o_lsd_rounds.argtypes = [i, i]
        L.o_merge_split.argtypes = [vp, vp, sz, vp, vp]
        L.o_bitonic_block.argtypes = [vp, vp, sz, i, sz, cp]
        L.o_oet_block.argtypes = [vp, vp, sz, i, sz, i, cp]
        L.o_bitonic.argtypes = [vp, vp, sz, i, cp]
        L.o_oet.argtypes = [vp, vp, sz, i, i, cp]
        L.o_segmented.argtypes = [vp, vp, vp, sz, i, i]
        L.o_is_sorted.argtypes = [vp, sz, i]
        L.o_check_stable_kv.argtypes = [vp, vp, vp, sz, i, i]
        L.o_mlp_forward_f64.argtypes = [dp, ctypes.c_double]
        L.o_mlp_forward_f64.restype = ctypes.c_double
        L.o_mlp_loss_grad_f64.argtypes = [dp, dp, dp, sz, dp]
        L.o_mlp_loss_grad_f64.restype = ctypes.c_double
        L.o_adam_step_f64.argtypes = [dp, dp, dp, dp, sz, i64, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.o_adam_step_f64.restype = None
        L.o_mlp_forward_f32.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_float]
        L.o_mlp_forward_f32.restype = ctypes.c_float
        L.o_midrank_targets.argtypes = [vp, sz, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _kb(a):
    if a.dtype == np.uint32:
        return 4
    if a.dtype == np.uint64:
        return 8
    raise TypeError("keys must be uint32 or uint64, got %s" % a.dtype)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("oracle %s failed with %d" % (what, rc))


def count_round(keys, shift, bits, vals=None):
    """One stable count-sort round; returns (keys_out, vals_out, hist)."""
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    ko = np.empty_like(k)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint64)
    vo = None if v is None else np.empty_like(v)
    h = np.zeros(1 << bits, dtype=np.uint64)
    _check(lib().o_count_round(_p(k), _p(ko), _p(v), _p(vo), k.size, shift, bits, _p(h)), "count_round")
    return ko, vo, h


def lsd(keys, radix_bits=8, vals=None, want_hist=False):
    """Stable LSD radix sort.  Returns keys_out, or (keys_out, vals_out), plus
    the per-round histograms and the counters when want_hist."""
    keys = np.ascontiguousarray(keys)
    kb = _kb(keys)
    out = np.empty_like(keys)
    vb = 0
    vo = None
    if vals is not None:
        vals = np.ascontiguousarray(vals)
        vb = vals.dtype.itemsize
        vo = np.empty_like(vals)
    rounds = lib().o_lsd_rounds(kb, radix_bits)
    hist = np.zeros((rounds, 1 << radix_bits), dtype=np.uint64) if want_hist else None
    cnt = Counters()
    _check(lib().o_lsd(_p(keys), _p(out), _p(vals), _p(vo), keys.size, kb, vb, radix_bits,
                       _p(hist), ctypes.byref(cnt)), "lsd")
    res = out if vals is None else (out, vo)
    if want_hist:
        return res, hist, cnt
    return res


def lsd_rounds(key_bytes, radix_bits):
    return lib().o_lsd_rounds(key_bytes, radix_bits)


def merge_split(A, B):
    A = np.ascontiguousarray(A, dtype=np.uint64)
    B = np.ascontiguousarray(B, dtype=np.uint64)
    assert A.size == B.size
    lo = np.empty_like(A)
    hi = np.empty_like(A)
    _check(lib().o_merge_split(_p(A), _p(B), A.size, _p(lo), _p(hi)), "merge_split")
    return lo, hi


def bitonic_block(keys, p):
    keys = np.ascontiguousarray(keys)
    out = np.empty_like(keys)
    cnt = Counters()
    _check(lib().o_bitonic_block(_p(keys), _p(out), keys.size, _kb(keys), p, ctypes.byref(cnt)),
           "bitonic_block")
    return out, cnt


def oet_block(keys, p, first_parity=0):
    keys = np.ascontiguousarray(keys)
    out = np.empty_like(keys)
    cnt = Counters()
    _check(lib().o_oet_block(_p(keys), _p(out), keys.size, _kb(keys), p, first_parity,
                             ctypes.byref(cnt)), "oet_block")
    return out, cnt


def bitonic(keys):
    keys = np.ascontiguousarray(keys)
    out = np.empty_like(keys)
    cnt = Counters()
    _check(lib().o_bitonic(_p(keys), _p(out), keys.size, _kb(keys), ctypes.byref(cnt)), "bitonic")
    return out, cnt


def oet(keys, first_parity=0):
    keys = np.ascontiguousarray(keys)
    out = np.empty_like(keys)
    cnt = Counters()
    _check(lib().o_oet(_p(keys), _p(out), keys.size, _kb(keys), first_parity, ctypes.byref(cnt)),
           "oet")
    return out, cnt


def segmented(keys, offsets, radix_bits=8):
    keys = np.ascontiguousarray(keys)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    out = np.empty_like(keys)
    _check(lib().o_segmented(_p(keys), _p(out), _p(offsets), offsets.size - 1, _kb(keys),
                             radix_bits), "segmented")
    return out


def is_sorted(keys):
    keys = np.ascontiguousarray(keys)
    return bool(lib().o_is_sorted(_p(keys), keys.size, _kb(keys)))


def check_stable_kv(keys_in, keys_out, idx_out):
    """0 if (keys_out, idx_out) is the stable sort of keys_in, else 1..4."""
    keys_in = np.ascontiguousarray(keys_in)
    keys_out = np.ascontiguousarray(keys_out)
    idx_out = np.ascontiguousarray(idx_out)
    assert keys_in.dtype == keys_out.dtype and keys_in.size == keys_out.size == idx_out.size
    return lib().o_check_stable_kv(_p(keys_in), _p(keys_out), _p(idx_out), keys_in.size,
                                   _kb(keys_in), idx_out.dtype.itemsize)


def mlp_forward_f64(params, x):
    params = np.ascontiguousarray(params, dtype=np.float64)
    assert params.size == NPARAM
    return lib().o_mlp_forward_f64(_dp(params), float(x))


def mlp_loss_grad_f64(params, xs, ts):
    params = np.ascontiguousarray(params, dtype=np.float64)
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    ts = np.ascontiguousarray(ts, dtype=np.float64)
    g = np.zeros(NPARAM, dtype=np.float64)
    loss = lib().o_mlp_loss_grad_f64(_dp(params), _dp(xs), _dp(ts), xs.size, _dp(g))
    return loss, g


def adam_step_f64(params, grad, m1, m2, t, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (params, grad, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().o_adam_step_f64(_dp(params), _dp(grad), _dp(m1), _dp(m2), params.size, int(t),
                          lr, beta1, beta2, eps)


def mlp_forward_f32(params, x):
    params = np.ascontiguousarray(params, dtype=np.float32)
    return lib().o_mlp_forward_f32(params.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   ctypes.c_float(x))


def midrank_targets(sorted_sample):
    s = np.ascontiguousarray(sorted_sample, dtype=np.uint64)
    t = np.empty(s.size, dtype=np.float64)
    _check(lib().o_midrank_targets(_p(s), s.size, _dp(t)), "midrank_targets")
    return t
