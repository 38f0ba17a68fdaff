"""The C ABI: librs.so loads on a machine without a GPU and exports every
function include/*.h declares; argument checks that return before any device
work behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("rs.h", "rs_learned.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(rs_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    so = os.path.join(ROOT, "paper_1708_09495_amd", "librs.so")
    if not os.path.exists(so):
        from paper_1708_09495_amd import build
        build.build()
    return ctypes.CDLL(so)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"rs_sort_u32", "rs_sort_u64", "rs_sort_kv", "rs_sort_batch_u32", "rs_sort_segmented",
            "rs_workspace_bytes", "rs_get_stats", "rs_tune_run", "rs_mlp_loss_grad"} <= names
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    import paper_1708_09495_amd as rs
    assert set(rs.EXPORTS) == _declared()


def test_host_side_queries(lib):
    lib.rs_workspace_bytes.restype = ctypes.c_size_t
    lib.rs_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_size_t]
    lib.rs_status_string.restype = ctypes.c_char_p
    lib.rs_small_capacity.restype = ctypes.c_size_t
    n = 1 << 20
    ws = lib.rs_workspace_bytes(0, n, 4, 0, 8, 1, 0)
    assert ws >= 4 * n and ws % 256 == 0                # one n-key copy plus tables
    assert lib.rs_workspace_bytes(0, n, 4, 0, 17, 1, 0) == 0   # no such radix
    assert lib.rs_workspace_bytes(0, n, 4, 0, 16, 1, 0) >= 4 * n + 4 * 65536   # wide digits
    assert lib.rs_workspace_bytes(0, 1 << 32, 4, 0, 16, 1, 0) == 0  # 32-bit cursors
    assert lib.rs_workspace_bytes(1, n, 8, 8, 8, 4, 0) > 16 * n  # learned kv u64
    assert lib.rs_workspace_bytes(3, 1000, 4, 0, 0, 0, 10) >= 4000
    assert lib.rs_small_capacity(4) == 16384
    assert lib.rs_status_string(3) == b"workspace missing, too small or misaligned"


def test_argument_errors_return_before_device_work(lib):
    vp = ctypes.c_void_p
    lib.rs_sort_u32.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, vp,
                                ctypes.c_size_t, vp]
    # a null key pointer with n > 0, an out-of-range radix and bad algorithms
    # are rejected on the host, with no GPU needed to get there
    assert lib.rs_sort_u32(None, vp(256), 10, 8, 1, None, 0, None) == 1
    assert lib.rs_sort_u32(vp(256), vp(4096), 10, 17, 1, None, 0, None) == 1
    assert lib.rs_sort_u32(vp(256), vp(4096), 10, 8, 9, None, 0, None) == 2
    assert lib.rs_sort_u32(None, None, 0, 8, 1, None, 0, None) == 0
    lib.rs_sort_kv.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp]
    assert lib.rs_sort_kv(vp(256), vp(4096), vp(8192), vp(16384), 10, 4, 2, 8, 1, None, 0, None) == 1


def test_block_network_queries_and_errors(lib):
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.rs_workspace_bytes.restype = ctypes.c_size_t
    lib.rs_workspace_bytes.argtypes = [ctypes.c_int, sz, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, sz]
    n = 1_000_003
    # two padded copies of the keys plus the runs' local-sort tables
    for algo, p in ((2, 256), (2, 2), (3, 7), (3, 256)):
        pn = p * -(-n // p)
        ws = lib.rs_workspace_bytes(5, n, 4, 0, 0, algo, p)
        assert ws >= 8 * pn and ws % 256 == 0, (algo, p, ws)
    assert lib.rs_workspace_bytes(5, n, 4, 0, 0, 2, 3) == 0       # BTN needs a power of two
    assert lib.rs_workspace_bytes(5, n, 4, 0, 0, 2, 8192) == 0    # p above 4096
    assert lib.rs_workspace_bytes(5, n, 8, 0, 0, 2, 256) == 0     # uint32 keys only
    assert lib.rs_workspace_bytes(5, n, 4, 0, 0, 1, 256) == 0     # BTN or OET only
    assert lib.rs_workspace_bytes(5, n, 4, 0, 0, 2, 0) == lib.rs_workspace_bytes(5, n, 4, 0, 0, 2, 256)
    # rs_sort_u32 with BTN above one workgroup's capacity takes the same path
    assert lib.rs_workspace_bytes(0, n, 4, 0, 0, 2, 0) == lib.rs_workspace_bytes(5, n, 4, 0, 0, 2, 0)
    assert lib.rs_workspace_bytes(0, 1000, 4, 0, 0, 2, 0) == 256
    lib.rs_sort_blocks_u32.argtypes = [vp, vp, sz, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    assert lib.rs_sort_blocks_u32(None, vp(256), 10, 2, 4, None, 0, None) == 1   # null input
    assert lib.rs_sort_blocks_u32(vp(256), vp(4096), 10, 2, 3, None, 0, None) == 1  # p not 2^k
    assert lib.rs_sort_blocks_u32(vp(256), vp(4096), 10, 3, 1, None, 0, None) == 1  # p = 1
    assert lib.rs_sort_blocks_u32(vp(256), vp(4096), 10, 3, 5000, None, 0, None) == 1
    assert lib.rs_sort_blocks_u32(vp(256), vp(4096), 10, 1, 4, None, 0, None) == 2  # LSD
    assert lib.rs_sort_blocks_u32(None, None, 0, 2, 0, None, 0, None) == 0
