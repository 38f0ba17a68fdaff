"""Python binding of librs (include/rs.h): argument marshalling only.

Every function has the name of the C entry point it calls and forwards
device pointers, sizes and the HIP stream.  PyTorch supplies device memory
(tensors) and streams; every step of every sort runs in librs's HIP kernels.
If librs.so is missing the binding raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librs.so")

RS_OK, RS_ERR_INVALID, RS_ERR_UNSUPPORTED, RS_ERR_WORKSPACE, RS_ERR_HIP = range(5)
RS_ALGO_AUTO, RS_ALGO_LSD, RS_ALGO_BTN, RS_ALGO_OET, RS_ALGO_LEARNED, RS_ALGO_LDS_RADIX = range(6)
RS_OP_SORT, RS_OP_SORT_KV, RS_OP_BATCH, RS_OP_SEGMENTED, RS_OP_TUNE, RS_OP_BLOCKS = range(6)

EXPORTS = ["rs_sort_u32", "rs_sort_u64", "rs_sort_kv", "rs_sort_batch_u32", "rs_sort_segmented",
           "rs_sort_blocks_u32", "rs_sort_u32_noalloc", "rs_stream_copy", "rs_blocks_set_model", "rs_blocks_get_model", "rs_blocks_default_p",
           "rs_workspace_bytes", "rs_small_capacity", "rs_status_string", "rs_get_stats",
           "rs_tune_set", "rs_tune_get", "rs_tune_run", "rs_tune_run_model", "rs_tune_save", "rs_tune_load", "rs_profile_enable", "rs_profile_read",
           "rs_learned_set_opts", "rs_learned_get_opts", "rs_mlp_num_params", "rs_mlp_forward",
           "rs_mlp_loss_grad", "rs_mlp_adam_step", "rs_mlp_set_weights", "rs_learned_debug_fault",
           "rs_learned_debug_ids"]


class RsError(RuntimeError):
    def __init__(self, code, where):
        msg = "%s failed: %s (%d)" % (where, rs_status_string(code), code)
        if code == RS_ERR_HIP:
            try:
                msg += ", hipError %d" % rs_get_stats().hip_error
            except Exception:
                pass
        super().__init__(msg)
        self.code = code


class rs_stats(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("radix_bits", ctypes.c_int32),
                ("passes", ctypes.c_int32), ("runs_p", ctypes.c_int32),
                ("network_stages", ctypes.c_int64), ("tile_keys", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("buckets_overflowed", ctypes.c_int64),
                ("keys_overflowed", ctypes.c_int64), ("train_loss", ctypes.c_double),
                ("device_error", ctypes.c_uint32), ("hip_error", ctypes.c_int32),
                ("passes_skipped", ctypes.c_int32)]


class rs_block_model(ctypes.Structure):
    _fields_ = [("local_ns_per_key", ctypes.c_double), ("stage_ps_per_key", ctypes.c_double),
                ("stage_fixed_us", ctypes.c_double), ("resident_runs", ctypes.c_int32)]


class rs_tune_entry(ctypes.Structure):
    _fields_ = [("size_log2", ctypes.c_int32), ("algo", ctypes.c_int32), ("p", ctypes.c_int32),
                ("radix_bits", ctypes.c_int32), ("tile_items", ctypes.c_int32),
                ("seg_tile_items", ctypes.c_int32)]


class rs_tune_result(ctypes.Structure):
    _fields_ = [("size_log2", ctypes.c_int32), ("algo", ctypes.c_int32), ("p", ctypes.c_int32),
                ("radix_bits", ctypes.c_int32), ("tile_items", ctypes.c_int32),
                ("seg_tile_items", ctypes.c_int32), ("chosen", ctypes.c_int32),
                ("us_per_array", ctypes.c_double), ("us_single", ctypes.c_double),
                ("us_model", ctypes.c_double)]


class rs_learned_opts(ctypes.Structure):
    _fields_ = [("train_steps", ctypes.c_int32), ("lr", ctypes.c_float), ("use_network", ctypes.c_int32),
                ("bucket_cap", ctypes.c_int32), ("feature_mode", ctypes.c_int32),
                ("fallback_frac", ctypes.c_double), ("train_blocks", ctypes.c_int32),
                ("max_fallback_buckets", ctypes.c_int32)]


class rs_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


_lib = None


def lib():
    """The loaded librs (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librs.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        # PyTorch ships its own libamdhip64 with the same soname as the
        # system one librs links.  Loading torch first makes librs bind to
        # that already-loaded runtime, so the process has one HIP runtime
        # (two copies cannot share the device).
        _torch()
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        L.rs_sort_u32.argtypes = [vp, vp, sz, i, i, vp, sz, vp]
        L.rs_sort_u64.argtypes = [vp, vp, sz, i, i, vp, sz, vp]
        L.rs_sort_kv.argtypes = [vp, vp, vp, vp, sz, i, i, i, i, vp, sz, vp]
        L.rs_sort_batch_u32.argtypes = [vp, vp, sz, sz, i, i, vp, sz, vp]
        L.rs_sort_segmented.argtypes = [vp, vp, vp, sz, ctypes.c_int64, i, vp, sz, vp]
        L.rs_sort_blocks_u32.argtypes = [vp, vp, sz, i, i, vp, sz, vp]
        L.rs_sort_u32_noalloc.argtypes = [vp, vp, sz, i, i, vp]
        L.rs_sort_u32_noalloc.restype = i
        L.rs_stream_copy.argtypes = [vp, vp, sz, vp]
        L.rs_stream_copy.restype = i
        L.rs_blocks_set_model.argtypes = [ctypes.POINTER(rs_block_model)]
        L.rs_blocks_get_model.argtypes = [ctypes.POINTER(rs_block_model)]
        L.rs_blocks_default_p.argtypes = [sz, i]
        L.rs_blocks_default_p.restype = ctypes.c_int32
        L.rs_workspace_bytes.argtypes = [i, sz, i, i, i, i, sz]
        L.rs_workspace_bytes.restype = sz
        L.rs_small_capacity.argtypes = [i]
        L.rs_small_capacity.restype = sz
        L.rs_status_string.argtypes = [i]
        L.rs_status_string.restype = ctypes.c_char_p
        L.rs_get_stats.argtypes = [ctypes.POINTER(rs_stats)]
        L.rs_tune_set.argtypes = [ctypes.POINTER(rs_tune_entry), i]
        L.rs_tune_set.restype = i
        L.rs_tune_get.argtypes = [ctypes.POINTER(rs_tune_entry), i]
        L.rs_tune_get.restype = i
        L.rs_tune_run.argtypes = [vp, sz, i, vp, ctypes.POINTER(rs_tune_result), i]
        L.rs_tune_run.restype = i
        L.rs_tune_run_model.argtypes = [vp, sz, i, vp, ctypes.POINTER(rs_tune_result), i]
        L.rs_tune_run_model.restype = i
        L.rs_tune_save.argtypes = [ctypes.c_char_p]
        L.rs_tune_save.restype = i
        L.rs_tune_load.argtypes = [ctypes.c_char_p]
        L.rs_tune_load.restype = i
        L.rs_learned_set_opts.argtypes = [ctypes.POINTER(rs_learned_opts)]
        L.rs_learned_set_opts.restype = i
        L.rs_learned_get_opts.argtypes = [ctypes.POINTER(rs_learned_opts)]
        L.rs_learned_get_opts.restype = i
        L.rs_mlp_num_params.argtypes = []
        L.rs_mlp_num_params.restype = sz
        L.rs_mlp_forward.argtypes = [vp, vp, vp, sz, vp]
        L.rs_mlp_forward.restype = i
        L.rs_mlp_loss_grad.argtypes = [vp, vp, vp, sz, vp, vp]
        L.rs_mlp_loss_grad.restype = i
        f32 = ctypes.c_float
        L.rs_mlp_adam_step.argtypes = [vp, vp, vp, vp, ctypes.c_int32, f32, f32, f32, f32, vp]
        L.rs_mlp_adam_step.restype = i
        L.rs_mlp_set_weights.argtypes = [vp, sz]
        L.rs_mlp_set_weights.restype = i
        L.rs_learned_debug_fault.argtypes = [i, vp, sz]
        L.rs_learned_debug_fault.restype = i
        L.rs_learned_debug_ids.argtypes = [vp, vp]
        L.rs_learned_debug_ids.restype = i
        L.rs_profile_enable.argtypes = [i]
        L.rs_profile_read.argtypes = [ctypes.POINTER(rs_kernel_time), i]
        L.rs_profile_read.restype = i
        for f in ("rs_profile_enable", "rs_sort_u32", "rs_sort_u64", "rs_sort_kv", "rs_sort_batch_u32",
                  "rs_sort_segmented", "rs_get_stats"):
            getattr(L, f).restype = i
        _lib = L
    return _lib


# ---- marshalling helpers -------------------------------------------------

def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_dev(t, bytes_, what):
    if not t.is_cuda or not t.is_contiguous() or t.element_size() != bytes_:
        raise ValueError("%s must be a contiguous CUDA tensor of %d-byte elements" % (what, bytes_))


# rs_get_stats reads the device status word in the most recent call's
# workspace: a workspace this binding allocates for a call is kept (per
# thread) until the thread's next call, so that the stats stay readable
# whatever is allocated in between.
_tls = threading.local()


def _workspace(need, ws, device):
    if ws is None:
        ws = _torch().empty(max(int(need), 1), dtype=_torch().uint8, device=device)
        _tls.ws = ws
    else:
        _tls.ws = None
    return ws


def _call(rc, where):
    if rc != RS_OK:
        raise RsError(rc, where)


# ---- the C entry points --------------------------------------------------

def rs_workspace_bytes(op, n, key_bytes=4, val_bytes=0, radix_bits=0, algo=RS_ALGO_AUTO,
                       num_segments=0):
    return lib().rs_workspace_bytes(op, n, key_bytes, val_bytes, radix_bits, algo, num_segments)


def rs_small_capacity(key_bytes=4):
    return lib().rs_small_capacity(key_bytes)


def rs_status_string(code):
    return lib().rs_status_string(code).decode()


def rs_get_stats():
    s = rs_stats()
    _call(lib().rs_get_stats(ctypes.byref(s)), "rs_get_stats")
    return s


TUNE_FIELDS = ("size_log2", "algo", "p", "radix_bits", "tile_items", "seg_tile_items")


def rs_tune_set(entries):
    """entries: iterable of (size_log2, algo, p) or (size_log2, algo, p,
    radix_bits, tile_items, seg_tile_items); missing fields are 0."""
    entries = list(entries)
    arr = (rs_tune_entry * max(1, len(entries)))()
    for k, e in enumerate(entries):
        e = tuple(e) + (0,) * (len(TUNE_FIELDS) - len(e))
        for f, v in zip(TUNE_FIELDS, e):
            setattr(arr[k], f, int(v))
    _call(lib().rs_tune_set(arr, len(entries)), "rs_tune_set")


def rs_tune_save(path):
    _call(lib().rs_tune_save(os.fsencode(path)), "rs_tune_save")


def rs_tune_load(path):
    _call(lib().rs_tune_load(os.fsencode(path)), "rs_tune_load")


def rs_blocks_get_model():
    """The MBSP cost model that picks p for the device-scale networks, as a dict."""
    m = rs_block_model()
    _call(lib().rs_blocks_get_model(ctypes.byref(m)), "rs_blocks_get_model")
    return {k: getattr(m, k) for k, _ in rs_block_model._fields_}


def rs_blocks_set_model(local_ns_per_key, stage_ps_per_key, stage_fixed_us, resident_runs):
    m = rs_block_model(local_ns_per_key, stage_ps_per_key, stage_fixed_us, resident_runs)
    _call(lib().rs_blocks_set_model(ctypes.byref(m)), "rs_blocks_set_model")


def rs_blocks_default_p(n, algo):
    """The p that p = 0 selects for n keys (0 for n = 0 or an algo other than BTN/OET)."""
    return int(lib().rs_blocks_default_p(n, algo))


def rs_tune_get():
    """The table as tuples (size_log2, algo, p, radix_bits, tile_items,
    seg_tile_items), classes 0..32."""
    arr = (rs_tune_entry * 64)()
    k = lib().rs_tune_get(arr, 64)
    return [tuple(getattr(arr[i], f) for f in TUNE_FIELDS) for i in range(k)]


def rs_tune_run(instances=1024, ws=None, stream=None, model=False):
    """Runs the autotuner on the current device (model=True: the small
    classes guided by the fitted cost model, rs_tune_run_model); returns a
    list of dicts (the fields of rs_tune_result)."""
    torch = _torch()
    need = rs_workspace_bytes(RS_OP_TUNE, instances)
    ws = _workspace(need, ws, torch.device("cuda", torch.cuda.current_device()))
    buf = (rs_tune_result * 1024)()
    fn = lib().rs_tune_run_model if model else lib().rs_tune_run
    k = fn(_ptr(ws), ws.numel(), instances, _stream(stream), buf, 1024)
    if k < 0:
        raise RsError(-k, "rs_tune_run_model" if model else "rs_tune_run")
    return [{f: getattr(buf[i], f) for f, _ in rs_tune_result._fields_} for i in range(k)]


def rs_learned_get_opts():
    o = rs_learned_opts()
    _call(lib().rs_learned_get_opts(ctypes.byref(o)), "rs_learned_get_opts")
    return {f: getattr(o, f) for f, _ in rs_learned_opts._fields_}


def rs_learned_set_opts(**kw):
    """Sets the named options (others keep their value); returns the old ones."""
    old = rs_learned_get_opts()
    new = dict(old)
    new.update(kw)
    o = rs_learned_opts(**new)
    _call(lib().rs_learned_set_opts(ctypes.byref(o)), "rs_learned_set_opts")
    return old


def rs_mlp_num_params():
    return lib().rs_mlp_num_params()


def rs_mlp_forward(params, x, y=None, stream=None):
    _check_dev(params, 4, "params")
    _check_dev(x, 4, "x")
    y = x.new_empty(x.shape) if y is None else y
    _call(lib().rs_mlp_forward(_ptr(params), _ptr(x), _ptr(y), x.numel(), _stream(stream)),
          "rs_mlp_forward")
    return y


def rs_mlp_loss_grad(params, x, t, grad=None, stream=None):
    """Returns a float32 tensor of 1154: the gradient (1153) and the summed
    squared error."""
    _check_dev(params, 4, "params")
    _check_dev(x, 4, "x")
    _check_dev(t, 4, "t")
    grad = params.new_empty(rs_mlp_num_params() + 1) if grad is None else grad
    _call(lib().rs_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(t), x.numel(), _ptr(grad),
                                 _stream(stream)), "rs_mlp_loss_grad")
    return grad


def rs_mlp_adam_step(params, m1, m2, grad, step, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One Adam step on device float32 tensors of 1153 (params, m1, m2 are
    updated in place; grad is read)."""
    np_ = rs_mlp_num_params()
    for name, t in (("params", params), ("m1", m1), ("m2", m2), ("grad", grad)):
        _check_dev(t, 4, name)
        if t.numel() < np_:
            raise ValueError("%s holds fewer than %d floats" % (name, np_))
    _call(lib().rs_mlp_adam_step(_ptr(params), _ptr(m1), _ptr(m2), _ptr(grad), int(step), float(lr),
                                 float(beta1), float(beta2), float(eps), _stream(stream)), "rs_mlp_adam_step")


def rs_mlp_set_weights(params):
    """Host float32 array of 1153 raw parameters the learned path uses
    instead of training; None goes back to training."""
    if params is None:
        _call(lib().rs_mlp_set_weights(None, 0), "rs_mlp_set_weights")
        return
    import numpy as np
    a = np.ascontiguousarray(params, dtype=np.float32)
    _call(lib().rs_mlp_set_weights(a.ctypes.data, a.size), "rs_mlp_set_weights")


RS_LEARNED_FAULT_NONE, RS_LEARNED_FAULT_SPLITTERS, RS_LEARNED_FAULT_SWAP = range(3)


def rs_learned_debug_fault(kind, splitters=None):
    """Plants a fault in the following learned sorts (RS_LEARNED_FAULT_*);
    splitters: host uint64 array of 65,535 for RS_LEARNED_FAULT_SPLITTERS."""
    if splitters is None:
        _call(lib().rs_learned_debug_fault(int(kind), None, 0), "rs_learned_debug_fault")
        return
    import numpy as np
    a = np.ascontiguousarray(splitters, dtype=np.uint64)
    _call(lib().rs_learned_debug_fault(int(kind), a.ctypes.data, a.size), "rs_learned_debug_fault")


def rs_learned_debug_ids(direct=None, assigned=None):
    """Has the following learned sorts write every key's bucket from the
    network directly into `direct` and from the splitter search into
    `assigned` (device int16 tensors of at least n entries); no arguments
    turn it off."""
    if direct is None and assigned is None:
        _call(lib().rs_learned_debug_ids(None, None), "rs_learned_debug_ids")
        return
    _check_dev(direct, 2, "direct")
    _check_dev(assigned, 2, "assigned")
    _call(lib().rs_learned_debug_ids(_ptr(direct), _ptr(assigned)), "rs_learned_debug_ids")


def rs_stream_copy(src, dst, stream=None):
    """Copies device tensor src into dst (same byte size) with the library's
    streaming copy kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not src.is_contiguous() or not dst.is_contiguous():
        raise ValueError("src and dst must be contiguous and of the same byte size")
    _call(lib().rs_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)), "rs_stream_copy")


def rs_profile_enable(on=True):
    _call(lib().rs_profile_enable(1 if on else 0), "rs_profile_enable")


def rs_profile_read():
    """{kernel name: (launches, total ms)} since the last read (waits on the
    recorded events)."""
    buf = (rs_kernel_time * 32)()
    k = lib().rs_profile_read(buf, 32)
    if k < 0:
        raise RsError(RS_ERR_HIP, "rs_profile_read")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(k)}


def rs_sort_u32(keys_in, keys_out=None, radix_bits=0, algo=RS_ALGO_AUTO, ws=None, stream=None):
    """Sort a CUDA tensor of 4-byte keys (read as uint32) ascending."""
    _check_dev(keys_in, 4, "keys_in")
    keys_out = keys_in.new_empty(keys_in.shape) if keys_out is None else keys_out
    _check_dev(keys_out, 4, "keys_out")
    n = keys_in.numel()
    ws = _workspace(rs_workspace_bytes(RS_OP_SORT, n, 4, 0, radix_bits, algo), ws, keys_in.device)
    _call(lib().rs_sort_u32(_ptr(keys_in), _ptr(keys_out), n, radix_bits, algo, _ptr(ws),
                            ws.numel(), _stream(stream)), "rs_sort_u32")
    return keys_out


def rs_sort_u64(keys_in, keys_out=None, radix_bits=0, algo=RS_ALGO_AUTO, ws=None, stream=None):
    """Sort a CUDA tensor of 8-byte keys (read as uint64) ascending."""
    _check_dev(keys_in, 8, "keys_in")
    keys_out = keys_in.new_empty(keys_in.shape) if keys_out is None else keys_out
    _check_dev(keys_out, 8, "keys_out")
    n = keys_in.numel()
    ws = _workspace(rs_workspace_bytes(RS_OP_SORT, n, 8, 0, radix_bits, algo), ws, keys_in.device)
    _call(lib().rs_sort_u64(_ptr(keys_in), _ptr(keys_out), n, radix_bits, algo, _ptr(ws),
                            ws.numel(), _stream(stream)), "rs_sort_u64")
    return keys_out


def rs_sort_kv(keys_in, vals_in, keys_out=None, vals_out=None, radix_bits=0, algo=RS_ALGO_AUTO,
               ws=None, stream=None):
    """Stable key-value sort; keys and values of 4 or 8 bytes."""
    kb, vb = keys_in.element_size(), vals_in.element_size()
    _check_dev(keys_in, kb, "keys_in")
    _check_dev(vals_in, vb, "vals_in")
    keys_out = keys_in.new_empty(keys_in.shape) if keys_out is None else keys_out
    vals_out = vals_in.new_empty(vals_in.shape) if vals_out is None else vals_out
    _check_dev(keys_out, kb, "keys_out")
    _check_dev(vals_out, vb, "vals_out")
    n = keys_in.numel()
    if vals_in.numel() != n:
        raise ValueError("keys and values differ in length")
    ws = _workspace(rs_workspace_bytes(RS_OP_SORT_KV, n, kb, vb, radix_bits, algo), ws,
                    keys_in.device)
    _call(lib().rs_sort_kv(_ptr(keys_in), _ptr(vals_in), _ptr(keys_out), _ptr(vals_out), n, kb, vb,
                           radix_bits, algo, _ptr(ws), ws.numel(), _stream(stream)), "rs_sort_kv")
    return keys_out, vals_out


RS_NOALLOC_SCRATCH_BYTES = 40 << 20
RS_NOALLOC_MAX_KEYS = 1 << 22


def rs_sort_u32_noalloc(keys_in, keys_out=None, radix_bits=0, algo=RS_ALGO_LSD, stream=None):
    """rs_sort_u32 with the library's static scratch instead of a workspace
    (n <= RS_NOALLOC_MAX_KEYS; LSD or AUTO)."""
    _check_dev(keys_in, 4, "keys_in")
    keys_out = keys_in.new_empty(keys_in.shape) if keys_out is None else keys_out
    _check_dev(keys_out, 4, "keys_out")
    if keys_out.numel() != keys_in.numel():
        raise ValueError("keys_out must hold as many keys as keys_in")
    _call(lib().rs_sort_u32_noalloc(_ptr(keys_in), _ptr(keys_out), keys_in.numel(), radix_bits, algo,
                                    _stream(stream)), "rs_sort_u32_noalloc")
    return keys_out


def rs_sort_batch_u32(keys_in, n, count, keys_out=None, algo=RS_ALGO_AUTO, p=0, ws=None,
                      stream=None):
    """Sort `count` back-to-back arrays of n uint32 keys each."""
    _check_dev(keys_in, 4, "keys_in")
    if keys_in.numel() != n * count:
        raise ValueError("keys_in must hold n * count keys")
    keys_out = keys_in.new_empty(keys_in.shape) if keys_out is None else keys_out
    _check_dev(keys_out, 4, "keys_out")
    ws = _workspace(rs_workspace_bytes(RS_OP_BATCH, n, 4, 0, 0, algo, count), ws, keys_in.device)
    _call(lib().rs_sort_batch_u32(_ptr(keys_in), _ptr(keys_out), n, count, algo, p, _ptr(ws),
                                  ws.numel(), _stream(stream)), "rs_sort_batch_u32")
    return keys_out


def rs_sort_blocks_u32(keys_in, keys_out=None, algo=RS_ALGO_BTN, p=0, ws=None, stream=None):
    """Sort a uint32 tensor with BTN or OET on p runs in device memory."""
    _check_dev(keys_in, 4, "keys_in")
    keys_out = keys_in.new_empty(keys_in.shape) if keys_out is None else keys_out
    _check_dev(keys_out, 4, "keys_out")
    n = keys_in.numel()
    ws = _workspace(rs_workspace_bytes(RS_OP_BLOCKS, n, 4, 0, 0, algo, p), ws, keys_in.device)
    _call(lib().rs_sort_blocks_u32(_ptr(keys_in), _ptr(keys_out), n, algo, p, _ptr(ws), ws.numel(),
                                   _stream(stream)), "rs_sort_blocks_u32")
    return keys_out


def rs_sort_segmented(keys_in, offsets, keys_out=None, algo=RS_ALGO_AUTO, ws=None, stream=None):
    """Sort each segment [offsets[s], offsets[s+1]) of a uint32 tensor."""
    _check_dev(keys_in, 4, "keys_in")
    _check_dev(offsets, 8, "offsets")
    keys_out = keys_in.new_empty(keys_in.shape) if keys_out is None else keys_out
    _check_dev(keys_out, 4, "keys_out")
    S = offsets.numel() - 1
    total = keys_in.numel()
    ws = _workspace(rs_workspace_bytes(RS_OP_SEGMENTED, total, 4, 0, 0, algo, S), ws,
                    keys_in.device)
    _call(lib().rs_sort_segmented(_ptr(keys_in), _ptr(keys_out), _ptr(offsets), S, total, algo,
                                  _ptr(ws), ws.numel(), _stream(stream)), "rs_sort_segmented")
    return keys_out
