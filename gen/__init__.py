"""Seeded synthetic inputs (host C with OpenMP, plus a HIP twin for uniform
keys).  Shared by the tests, the smoke check and the benchmark; holds no
sorting arithmetic.  See ``gen.h`` for the definitions."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgen.so")
_DEV_SO = os.path.join(_HERE, "libgen_dev.so")
_lib = None
_dev = None

# Seeds: S0 for the whole study, config c uses S0 + c.
S0 = 0x170809495


def _stale(so, srcs):
    return not os.path.exists(so) or any(os.path.getmtime(so) < os.path.getmtime(s) for s in srcs)


def build(force: bool = False, device: bool = True) -> None:
    src = os.path.join(_HERE, "gen.c")
    if force or _stale(_SO, [src]):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    dsrc = os.path.join(_HERE, "gen_dev.hip")
    if device and (force or _stale(_DEV_SO, [dsrc])):
        tmp = _DEV_SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-o", tmp, dsrc])
        os.replace(tmp, _DEV_SO)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(device=False)
        L = ctypes.CDLL(_SO)
        u64, vp, sz, d = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double
        L.gen_splitmix64.argtypes = [u64, u64]
        L.gen_splitmix64.restype = u64
        L.gen_uniform_u32.argtypes = [u64, vp, sz]
        L.gen_uniform_u64.argtypes = [u64, vp, sz]
        L.gen_uniform_u32_range.argtypes = [u64, vp, sz, sz]
        L.gen_zipf_u64.argtypes = [u64, vp, sz, d, d]
        L.gen_lognormal_u64.argtypes = [u64, vp, sz]
        L.gen_gauss_mix_u64.argtypes = [u64, vp, sz, ctypes.c_int, ctypes.c_int]
        L.gen_loguniform_lengths.argtypes = [u64, vp, sz, d, d]
        L.gen_sample_indices.argtypes = [u64, vp, sz, u64]
        for f in ("gen_uniform_u32", "gen_uniform_u64", "gen_uniform_u32_range", "gen_zipf_u64",
                  "gen_lognormal_u64", "gen_gauss_mix_u64", "gen_loguniform_lengths",
                  "gen_sample_indices"):
            getattr(L, f).restype = None
        _lib = L
    return _lib


def dev():
    """The device twin (needs a GPU at call time)."""
    global _dev
    if _dev is None:
        if not os.path.exists(_DEV_SO):
            raise RuntimeError("libgen_dev.so is not built; run __graft_entry__.build()")
        import torch  # noqa: F401  (bind to torch's HIP runtime: one runtime per process)
        L = ctypes.CDLL(_DEV_SO)
        u64, vp = ctypes.c_uint64, ctypes.c_void_p
        L.gen_dev_uniform_u32.argtypes = [u64, vp, u64, u64, vp]
        L.gen_dev_uniform_u64.argtypes = [u64, vp, u64, u64, vp]
        L.gen_dev_iota.argtypes = [vp, u64, ctypes.c_int, vp]
        _dev = L
    return _dev


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def splitmix64(seed, i):
    return lib().gen_splitmix64(seed & (2**64 - 1), i)


def uniform_u32(seed, n, start=0):
    out = np.empty(n, dtype=np.uint32)
    lib().gen_uniform_u32_range(seed & (2**64 - 1), _p(out), start, n)
    return out


def uniform_u64(seed, n):
    out = np.empty(n, dtype=np.uint64)
    lib().gen_uniform_u64(seed & (2**64 - 1), _p(out), n)
    return out


def zipf_u64(seed, n, s=1.1, N=2.0**32):
    out = np.empty(n, dtype=np.uint64)
    lib().gen_zipf_u64(seed & (2**64 - 1), _p(out), n, s, N)
    return out


def lognormal_u64(seed, n):
    out = np.empty(n, dtype=np.uint64)
    lib().gen_lognormal_u64(seed & (2**64 - 1), _p(out), n)
    return out


def gauss_mix_u64(seed, n, comps=16, sigma_log2=50):
    out = np.empty(n, dtype=np.uint64)
    lib().gen_gauss_mix_u64(seed & (2**64 - 1), _p(out), n, comps, sigma_log2)
    return out


def loguniform_lengths(seed, S, lo_log2=4.0, hi_log2=20.0):
    out = np.empty(S, dtype=np.int64)
    lib().gen_loguniform_lengths(seed & (2**64 - 1), _p(out), S, lo_log2, hi_log2)
    return out


def sample_indices(seed, m, n):
    out = np.empty(m, dtype=np.uint64)
    lib().gen_sample_indices(seed & (2**64 - 1), _p(out), m, n)
    return out


def instances_u32(seed, n, count):
    """`count` independent uniform u32 arrays of length n, instance i drawn
    from seed mix(seed, n, i); returned as one (count, n) array."""
    out = np.empty((count, n), dtype=np.uint32)
    for i in range(count):
        s = splitmix64(splitmix64(seed, n), i)
        lib().gen_uniform_u32_range(s, _p(out[i]), 0, n)
    return out


def uniform_u32_dev(seed, tensor, start=0, stream=None):
    """Fill a CUDA uint32/int32 tensor with uniform_u32(seed, len, start)."""
    rc = dev().gen_dev_uniform_u32(seed & (2**64 - 1), tensor.data_ptr(), start, tensor.numel(),
                                   stream)
    if rc:
        raise RuntimeError("gen_dev_uniform_u32 failed")


def uniform_u64_dev(seed, tensor, start=0, stream=None):
    rc = dev().gen_dev_uniform_u64(seed & (2**64 - 1), tensor.data_ptr(), start, tensor.numel(),
                                   stream)
    if rc:
        raise RuntimeError("gen_dev_uniform_u64 failed")


def iota_dev(tensor, stream=None):
    rc = dev().gen_dev_iota(tensor.data_ptr(), tensor.numel(), tensor.element_size(), stream)
    if rc:
        raise RuntimeError("gen_dev_iota failed")
