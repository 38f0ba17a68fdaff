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


def test_segmented_workspace_grows_with_keys_not_segments(lib):
    # the shared rounds' tables (look-back words and block sums, tile
    # descriptors, per-segment histograms) are bounded by the keys: at most
    # n / 10,241 segments can be long enough to use them
    lib.rs_workspace_bytes.restype = ctypes.c_size_t
    lib.rs_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_size_t]
    n = 1 << 24
    few = lib.rs_workspace_bytes(3, n, 4, 0, 0, 0, 64)
    many = lib.rs_workspace_bytes(3, n, 4, 0, 0, 0, 1 << 20)
    assert 4 * n < few < many < 8 * n + 32 * (1 << 20)
    # RS_ALGO_LSD (one workgroup per segment) needs none of those tables
    assert lib.rs_workspace_bytes(3, n, 4, 0, 0, 1, 1 << 20) < many


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
    # keys sorted in place but values not (and the reverse): the rounds pick
    # their buffers from the keys, so the mixed case is refused, for every
    # algorithm that takes values
    for algo in (0, 1, 4):
        assert lib.rs_sort_kv(vp(256), vp(1 << 20), vp(256), vp(1 << 24), 10, 8, 8, 8, algo,
                              None, 0, None) == 1
        assert lib.rs_sort_kv(vp(256), vp(1 << 20), vp(1 << 24), vp(1 << 20), 10, 8, 8, 8, algo,
                              None, 0, None) == 1


def test_lsd_key_count_limit(lib):
    """Digit counts and prefixes of the LSD rounds are 32-bit words: n = 2^32
    is refused (unsupported), n = 2^32 - 1 is planned."""
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.rs_workspace_bytes.restype = ctypes.c_size_t
    lib.rs_workspace_bytes.argtypes = [ctypes.c_int, sz, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, sz]
    big = 1 << 32
    for kb in (4, 8):
        for bits in (8, 11):
            assert lib.rs_workspace_bytes(0, big, kb, 0, bits, 1, 0) == 0
            assert lib.rs_workspace_bytes(0, big - 1, kb, 0, bits, 1, 0) > (big - 1) * kb
        assert lib.rs_workspace_bytes(1, big, kb, 4, 8, 1, 0) == 0
    assert lib.rs_workspace_bytes(0, big, 8, 0, 8, 4, 0) == 0     # learned path
    lib.rs_sort_u32.argtypes = [vp, vp, sz, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    lib.rs_sort_u64.argtypes = [vp, vp, sz, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    # in place, so no overlap check stops it first; refused before any device work
    assert lib.rs_sort_u32(vp(256), vp(256), big, 8, 1, None, 0, None) == 2
    assert lib.rs_sort_u32(vp(256), vp(256), big, 8, 0, None, 0, None) == 2
    assert lib.rs_sort_u64(vp(256), vp(256), big, 8, 4, None, 0, None) == 2


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
    lib.rs_blocks_default_p.restype = ctypes.c_int32
    lib.rs_blocks_default_p.argtypes = [sz, ctypes.c_int]
    pd = lib.rs_blocks_default_p(n, 2)
    assert lib.rs_workspace_bytes(5, n, 4, 0, 0, 2, 0) == lib.rs_workspace_bytes(5, n, 4, 0, 0, 2, pd)
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


class _Model(ctypes.Structure):
    _fields_ = [("local_ns_per_key", ctypes.c_double), ("stage_ps_per_key", ctypes.c_double),
                ("stage_fixed_us", ctypes.c_double), ("resident_runs", ctypes.c_int32)]


def _model_ns(m, n, algo, p):
    """T(p) as include/rs.h states it (ns)."""
    N = -(-n // p)
    waves = -(-p // m.resident_runs)
    lg = p.bit_length() - 1
    stages = lg * (lg + 1) // 2 if algo == 2 else p
    return (m.local_ns_per_key * N * waves
            + stages * (m.stage_ps_per_key * 1e-3 * p * N + m.stage_fixed_us * 1e3))


def test_block_model_default_p(lib):
    """p = 0 of the device-scale networks: the minimum of the MBSP cost model
    (Section 3, Eqs. TbG and ToG) over the valid p, by brute force here."""
    lib.rs_blocks_default_p.restype = ctypes.c_int32
    lib.rs_blocks_default_p.argtypes = [ctypes.c_size_t, ctypes.c_int]
    lib.rs_blocks_get_model.argtypes = [ctypes.POINTER(_Model)]
    lib.rs_blocks_set_model.argtypes = [ctypes.POINTER(_Model)]
    dflt = _Model()
    assert lib.rs_blocks_get_model(ctypes.byref(dflt)) == 0
    assert (dflt.local_ns_per_key, dflt.stage_ps_per_key, dflt.stage_fixed_us, dflt.resident_runs) == \
        (3.74, 1.67, 17.2, 512)
    BTN, OET = 2, 3
    try:
        models = [dflt, _Model(10.0, 0.5, 5.0, 64), _Model(1.0, 20.0, 100.0, 4096)]
        for m in models:
            assert lib.rs_blocks_set_model(ctypes.byref(m)) == 0
            for n in (100, 1000, 70_001, 1 << 20, 12_345_678, 1 << 27, 3 << 29):
                for algo in (BTN, OET):
                    p = lib.rs_blocks_default_p(n, algo)
                    pmax = max(2, min(4096, n // 64))
                    cands = [q for q in range(2, pmax + 1) if algo == OET or q & (q - 1) == 0]
                    assert p in cands, (n, algo, p)
                    t = [_model_ns(m, n, algo, q) for q in cands]
                    best = cands[min(range(len(cands)), key=lambda i: (t[i], cands[i]))]
                    assert abs(_model_ns(m, n, algo, p) - t[cands.index(best)]) <= 1e-9 * t[cands.index(best)], \
                        (n, algo, p, best)
        # the balance the model strikes: OET's optimum grows like sqrt(local / stage)
        assert lib.rs_blocks_set_model(ctypes.byref(_Model(1.0, 1e6, 0.0, 512))) == 0
        assert lib.rs_blocks_default_p(1 << 24, OET) == 2 and lib.rs_blocks_default_p(1 << 24, BTN) == 2
        assert lib.rs_blocks_set_model(ctypes.byref(_Model(1e6, 0.0, 0.0, 1 << 30))) == 0
        assert lib.rs_blocks_default_p(1 << 24, OET) == 4096 and lib.rs_blocks_default_p(1 << 24, BTN) == 4096
        # ceil(10000/p) = 65 for p = 154..156: the smaller p of a tie
        assert lib.rs_blocks_default_p(10_000, OET) == 154 and lib.rs_blocks_default_p(10_000, BTN) == 128
        # out-of-range models are refused and leave the model as it was
        cur = _Model()
        lib.rs_blocks_get_model(ctypes.byref(cur))
        for bad in (_Model(0.0, 1.0, 1.0, 1), _Model(1.0, -1.0, 1.0, 1), _Model(1.0, 1.0, -1.0, 1),
                    _Model(float("nan"), 1.0, 1.0, 1), _Model(1.0, float("inf"), 1.0, 1),
                    _Model(1.0, 1.0, 1.0, 0)):
            assert lib.rs_blocks_set_model(ctypes.byref(bad)) == 1
        assert lib.rs_blocks_set_model(None) == 1 and lib.rs_blocks_get_model(None) == 1
        after = _Model()
        lib.rs_blocks_get_model(ctypes.byref(after))
        assert bytes(after) == bytes(cur)
        assert lib.rs_blocks_default_p(0, OET) == 0 and lib.rs_blocks_default_p(1000, 1) == 0
    finally:
        assert lib.rs_blocks_set_model(ctypes.byref(dflt)) == 0


def test_noalloc_limits_on_the_host(lib):
    """The no-allocation sort refuses, before any device call, sizes above
    its limit, wide radices and algorithms other than LSD / AUTO; the
    largest accepted plan at every radix fits its static scratch."""
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.rs_sort_u32_noalloc.argtypes = [vp, vp, sz, ctypes.c_int, ctypes.c_int, vp]
    lib.rs_sort_u32_noalloc.restype = ctypes.c_int
    lib.rs_workspace_bytes.restype = ctypes.c_size_t
    lib.rs_workspace_bytes.argtypes = [ctypes.c_int, sz, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, sz]
    nmax, scratch = 1 << 22, 40 << 20
    assert lib.rs_sort_u32_noalloc(vp(256), vp(256), nmax + 1, 8, 1, None) == 2
    assert lib.rs_sort_u32_noalloc(vp(256), vp(256), 1000, 16, 1, None) == 2
    assert lib.rs_sort_u32_noalloc(vp(256), vp(256), 1000, 8, 2, None) == 2
    assert lib.rs_sort_u32_noalloc(vp(256), vp(256), 1000, 17, 1, None) == 1
    assert lib.rs_sort_u32_noalloc(None, vp(256), 1000, 8, 1, None) == 1
    for bits in range(1, 12):
        need = lib.rs_workspace_bytes(0, nmax, 4, 0, bits, 1, 0)
        assert 0 < need <= scratch, (bits, need)


class _TuneEntry(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("size_log2", "algo", "p", "radix_bits", "tile_items",
                                               "seg_tile_items")]


def test_tuning_table_on_the_host(lib, tmp_path):
    """The tuning table's checks and file format, host side: classes 0..32,
    small-array choices only up to class 14, radix 0..16, tiles 16/28 and
    8/16; a file that does not parse (or holds a bad entry) is refused before
    any device call; a well-formed file needs the device it was written for
    (none here)."""
    E = _TuneEntry
    lib.rs_tune_set.argtypes = [ctypes.POINTER(E), ctypes.c_int]
    lib.rs_tune_get.argtypes = [ctypes.POINTER(E), ctypes.c_int]
    lib.rs_tune_load.argtypes = [ctypes.c_char_p]
    arr = (E * 64)()
    assert lib.rs_tune_get(arr, 64) == 33
    old = [tuple(getattr(arr[i], f) for f, _ in E._fields_) for i in range(33)]
    assert all(e[1] == 0 and e[2] == 0 for e in old[15:])

    def put(*e):
        one = (E * 1)(E(*e))
        return lib.rs_tune_set(one, 1)
    try:
        assert put(20, 0, 0, 11, 0, 8) == 0
        assert put(12, 2, 64, 8, 28, 16) == 0
        assert lib.rs_tune_get(arr, 64) == 33
        assert tuple(getattr(arr[20], f) for f, _ in E._fields_) == (20, 0, 0, 11, 0, 8)
        for bad in ((33, 0, 0, 8, 0, 0), (20, 2, 4, 8, 0, 0), (20, 0, 0, 17, 0, 0), (20, 0, 0, 8, 20, 0),
                    (20, 0, 0, 8, 4, 0),
                    (20, 0, 0, 8, 0, 12), (12, 2, 3, 8, 0, 0)):
            assert put(*bad) == 1, bad
        good = ('{"format": "rs-tuning-1", "arch": "gfx950", "cus": 256, "classes": '
                '[{"size_log2": 20, "algo": 0, "p": 0, "radix_bits": 11, "tile_items": 0, "seg_tile_items": 8}]}')
        for text, rc in ((good, 4), (good.replace("rs-tuning-1", "other"), 1), ("{", 1), ("[]", 1),
                         (good.replace('"radix_bits": 11', '"radix_bits": 99'), 1),
                         (good.replace('"algo": 0', '"algo": 2'), 1), (good.replace('"cus"', '"cuz"'), 1)):
            f = tmp_path / "t.json"
            f.write_text(text)
            assert lib.rs_tune_load(str(f).encode()) == rc, text
        assert lib.rs_tune_load(str(tmp_path / "missing.json").encode()) == 1
    finally:
        restore = (E * 33)(*[E(*e) for e in old])
        assert lib.rs_tune_set(restore, 33) == 0
