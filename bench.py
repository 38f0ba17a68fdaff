#!/usr/bin/env python3
"""Benchmark of the integer-sorting hot path on one MI355X.  Prints ONE JSON
line per invocation.

Default workload (the headline): one step = one complete rs_sort_u32 call
(all count-sort rounds: the fill, the all-round histogram and the four
rank-and-scatter rounds) over 2^28 uint32 keys drawn uniform on [0, 2^32)
by SplitMix64, radix 2^8, with the input already resident in HBM.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
                  [--workload lsd|small|segmented|learned|blocks]
                  lsd:       [--log2n 28] [--radix-bits 8|11|16] [--key-bytes 4|8] [--kv]
                  small:     [--small-n 4096] [--algo btn|oet|lds_radix|auto] [--p P]
                  blocks:    [--log2n 27] [--algo btn|oet] [--p P] (0: the MBSP model's p)
                  learned:   [--dist zipf|lognormal|mixture]

The roofline object covers the dominant kernel of the workload: its
algorithmic bytes (or operations) per launch over its mean launch time,
timed with HIP events that the library records on the launch stream during
the timed steps.  The cpu_baseline object times the serial C oracle on a
bounded sample of the same input on one host core (mean of four runs, as
the paper reports its timings).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gkeys/s + HBM GB/s, uint32 n=2^28; batched/learned vs plain radix"
HBM_PEAK_GBS = 8000.0    # MI355X HBM3E, 8 TB/s
VALU_PEAK_TOPS = 39.3    # 256 CUs x 64 lanes x 2.4 GHz, one 32-bit op per lane per clock


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lsd",
                    choices=["lsd", "small", "segmented", "learned", "blocks", "crossover"])
    ap.add_argument("--log2n", type=int, default=None, help="lsd, learned: 28; blocks: 27")
    ap.add_argument("--radix-bits", type=int, default=8)
    ap.add_argument("--key-bytes", type=int, default=4, choices=[4, 8])
    ap.add_argument("--kv", action="store_true", help="stable sort with a payload = index")
    ap.add_argument("--small-n", type=int, default=4096)
    ap.add_argument("--instances", type=int, default=10000)
    ap.add_argument("--batch-only", action="store_true",
                    help="small: time only the batched launch (no single-instance timings)")
    ap.add_argument("--algo", default="auto", choices=["auto", "btn", "oet", "lds_radix"])
    ap.add_argument("--p", type=int, default=0)
    ap.add_argument("--segments", type=int, default=65536)
    ap.add_argument("--plain-sample", type=int, default=512,
                    help="segments timed one plain-radix call each (segmented workload)")
    ap.add_argument("--dist", default="zipf", choices=["zipf", "lognormal", "mixture"])
    ap.add_argument("--feature-mode", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="learned: the key feature (-1 automatic, 0 linear, 1 log2, 2 sample quantiles)")
    ap.add_argument("--mbsp-radix", action="store_true",
                    help="lsd: the MBSP check of the parallel radix sort (Eqs. TsG, Tp4, Tp2; Observation 7)")
    ap.add_argument("--mbsp", action="store_true",
                    help="blocks: also time OET and one workgroup's radix sort of the whole array and "
                         "report the MBSP model's g, G and predictions (Section 3, Eqs. TsG, ToG, TbG)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tune", type=int, default=0,
                    help="run the autotuner with this many instances first (0: no)")
    ap.add_argument("--tuning-file", default=None, help="load a saved tuning table first")
    ap.add_argument("--save-tuning", default=None, help="save the tuning table after --tune")
    ap.add_argument("--cross-lo", type=int, default=10, help="crossover: smallest lg n")
    ap.add_argument("--cross-hi", type=int, default=22, help="crossover: largest lg n")
    ap.add_argument("--cpu-log2n", type=int, default=28)
    return ap.parse_args()


# ---- shared helpers ----------------------------------------------------------

def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1708_09495_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_traffic(kernel, workload, src_hash):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary
    (profiles/pmc_<kernel>_<workload>.txt, "key: value" lines), if one exists
    for this kernel, workload and kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.txt" % (kernel, workload))
    try:
        with open(path) as f:
            d = dict(line.split(": ", 1) for line in f.read().splitlines() if ": " in line)
    except OSError:
        return None
    if d.get("source_sha256", "").strip() != src_hash:
        return None
    try:
        return int(d["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pin_one_core():
    """Pin this process to one host core for the oracle timing; returns the
    previous affinity set (or None where affinity is not available)."""
    try:
        old = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(old)})
        return old
    except (AttributeError, OSError):
        return None


def time_oracle(fn, runs=4):
    old = pin_one_core()
    try:
        times = []
        for _ in range(runs):
            t0 = time.perf_counter()
            fn()
            times.append(time.perf_counter() - t0)
    finally:
        if old is not None:
            os.sched_setaffinity(0, old)
    return sum(times) / len(times)


def timed_steps(step, steps, warmup, rs, torch, launch_timing=False):
    """Warm-up, then exactly `steps` steps between device synchronisations
    (ms per step, with nothing recorded between the launches), then, when
    launch_timing is set, the same number of steps again with the library's
    launch events on, for the per-kernel averages (each event pair adds a
    few microseconds between launches, so they stay out of ms per step).
    Returns (ms per step, profile)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    rs.rs_profile_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {}
    if launch_timing:
        rs.rs_profile_read()          # drop anything recorded before
        rs.rs_profile_enable(True)
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        rs.rs_profile_enable(False)
        prof = rs.rs_profile_read()
    return (t1 - t0) * 1e3 / steps, prof


def copy_ceiling_gbs(torch, nbytes, rs=None):
    """Read+write bandwidth of a device-to-device copy of nbytes: with rs,
    the library's own streaming copy kernel (timed by the library's launch
    events), else torch's copy_."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    reps = 10
    if rs is not None:
        ms, prof = timed_steps(lambda: rs.rs_stream_copy(a, b), reps, 2, rs, torch, launch_timing=True)
        launches, tot = prof.get("stream_copy", (0, 0.0))
        ms = tot / launches if launches else ms
    else:
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def kernels_of(prof):
    return {k: {"launches": c, "avg_ms": (t / c if c else None)} for k, (c, t) in prof.items()}


def hbm_roofline(prof, kname, bytes_per_launch, traffic=None):
    launches, tot_ms = prof.get(kname, (0, 0.0))
    avg_ms = tot_ms / launches if launches else float("nan")
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if launches else None
    return {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
        "kernel": kname, "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms,
    }


def line(args, value, ms_per_step, dtype, data, config, roofline, prof, extra=None):
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": data,
        "config": config,
        "roofline": roofline,
        "kernels": kernels_of(prof),
        "timing": "ms_per_step over the timed steps with no launch events; kernel averages "
                  "(roofline.achieved, kernels) from the same number of steps run again with "
                  "the library's launch events on",
    }
    if extra:
        res.update(extra)
    return res


# ---- plain LSD (the headline) --------------------------------------------------

def bench_lsd(args, torch, rs, gen, np):
    n = 1 << args.log2n
    kb = args.key_bytes
    bits = args.radix_bits
    seed = gen.S0 + 2
    kdt = torch.int32 if kb == 4 else torch.int64
    keys = torch.empty(n, dtype=kdt, device="cuda")
    (gen.uniform_u32_dev if kb == 4 else gen.uniform_u64_dev)(seed, keys)
    out = torch.empty_like(keys)
    vals = vout = None
    vb = 0
    if args.kv:
        vb = 4
        vals = torch.empty(n, dtype=torch.int32, device="cuda")
        gen.iota_dev(vals)
        vout = torch.empty_like(vals)
    op = rs.RS_OP_SORT_KV if args.kv else rs.RS_OP_SORT
    ws = torch.empty(rs.rs_workspace_bytes(op, n, kb, vb, bits, rs.RS_ALGO_LSD), dtype=torch.uint8,
                     device="cuda")
    torch.cuda.synchronize()

    def step():
        if args.kv:
            rs.rs_sort_kv(keys, vals, out, vout, radix_bits=bits, algo=rs.RS_ALGO_LSD, ws=ws)
        elif kb == 4:
            rs.rs_sort_u32(keys, out, radix_bits=bits, algo=rs.RS_ALGO_LSD, ws=ws)
        else:
            rs.rs_sort_u64(keys, out, radix_bits=bits, algo=rs.RS_ALGO_LSD, ws=ws)

    step()
    torch.cuda.synchronize()
    st = rs.rs_get_stats()
    assert st.device_error == 0, "device reported a bounded-wait or range error"
    passes = st.passes
    ms, prof = timed_steps(step, args.steps, args.warmup, rs, torch, launch_timing=True)
    gkeys = n / (ms * 1e-3) / 1e9
    wide = bits >= 12
    # whole-call algorithmic bytes: one histogram read (wide digits: a
    # counting read in every round), then one read + write of keys (and
    # values) per round
    call_bytes = (passes if wide else 1) * n * kb + passes * 2 * n * (kb + vb)
    kname = "wide_scatter" if wide else "onesweep"
    workload = "lsd_%s%s_n2p%d_b%d" % ("u32" if kb == 4 else "u64", "_kv32" if args.kv else "",
                                        args.log2n, bits)
    srcs = ("rs_wide.hip", "rs_dev.h") if wide else ("rs_lsd.hip", "rs_dev.h")
    roof = hbm_roofline(prof, kname, 2 * n * (kb + vb), pmc_traffic(kname, workload, source_hash(srcs)))
    config = {
        "workload": "plain LSD radix sort, %s keys%s, n=2^%d, radix 2^%d (%d count-sort rounds)"
                    % ("uint32" if kb == 4 else "uint64",
                       " + uint32 payload (stable)" if args.kv else " only", args.log2n, bits, passes),
        "n": n, "key_bytes": kb, "val_bytes": vb, "radix_bits": bits, "passes": passes,
        "tile_keys": st.tile_keys,
    }
    del ws, out, vout
    torch.cuda.empty_cache()
    extra = {
        "hbm_gbs": call_bytes / (ms * 1e-3) / 1e9,
        "copy_ceiling_gbs": copy_ceiling_gbs(torch, 1 << 30, rs),
        "copy_ceiling_torch_gbs": copy_ceiling_gbs(torch, 1 << 30),
    }
    if args.mbsp_radix and kb == 4 and not args.kv:
        extra["mbsp_radix"] = mbsp_radix_check(args, torch, rs, keys, n, bits, ms)
    res = line(args, gkeys, ms, "u32" if kb == 4 else "u64",
               "synthetic: SplitMix64 uniform keys on the full range, seed S0+2"
               + (", payload = original index (u32)" if args.kv else ""), config, roof, prof, extra)
    if not args.no_cpu:
        import oracle
        m = min(n, 1 << args.cpu_log2n)
        kh = np.ascontiguousarray(keys[:m].cpu().numpy().view(np.uint32 if kb == 4 else np.uint64))
        vh = np.arange(m, dtype=np.uint32) if args.kv else None
        sec = time_oracle(lambda: oracle.lsd(kh, bits, vals=vh))
        res["cpu_baseline"] = {
            "value": m / sec / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": "first 2^%d keys of the same input, serial C oracle o_lsd radix 2^%d%s, "
                      "pinned to one host core, mean of 4 runs"
                      % (m.bit_length() - 1, bits, ", payload = index" if args.kv else ""),
            "seconds_per_run": sec,
        }
    return res


# ---- small-n single arrays (BTN / OET / LDS radix) ---------------------------------

def network_ops(algo, n, p):
    """32-bit min/max operations one instance of the block network executes:
    a register bitonic sort of each N-run (N = n_pad/p), then per merge-split
    stage one min or max per key against the partner run and a bitonic merge
    of the kept N keys.  Stages: lg p (lg p + 1)/2 (BTN) or p (OET)."""
    import math
    npad = 1 << (n - 1).bit_length()
    N = npad // p
    lgN = int(math.log2(N))
    lgp = int(math.log2(p))
    local = p * 2 * (N // 2) * lgN * (lgN + 1) // 2
    stages = lgp * (lgp + 1) // 2 if algo == "btn" else (p if p > 1 else 0)
    per_stage = p * (N + 2 * (N // 2) * lgN)
    return local + stages * per_stage


def bench_small(args, torch, rs, gen, np):
    n = args.small_n
    count = args.instances
    algo = {"auto": rs.RS_ALGO_AUTO, "btn": rs.RS_ALGO_BTN, "oet": rs.RS_ALGO_OET,
            "lds_radix": rs.RS_ALGO_LDS_RADIX}[args.algo]
    host = gen.instances_u32(gen.S0 + 3, n, count)
    keys = torch.from_numpy(host.reshape(-1).view(np.int32)).cuda()
    out = torch.empty_like(keys)

    def step():
        rs.rs_sort_batch_u32(keys, n, count, out, algo=algo, p=args.p)

    step()
    torch.cuda.synchronize()
    st = rs.rs_get_stats()
    ms, prof = timed_steps(step, args.steps, args.warmup, rs, torch, launch_timing=True)
    used = {rs.RS_ALGO_BTN: "btn", rs.RS_ALGO_OET: "oet", rs.RS_ALGO_LDS_RADIX: "lds_radix"}[st.algo]
    p = st.runs_p
    # one instance alone, and the device-wide LSD sort of one instance
    single_ms = lsd_ms = float("nan")
    if not args.batch_only:
        one = keys[:n].clone()
        one_out = torch.empty_like(one)
        single_ms, _ = timed_steps(lambda: rs.rs_sort_batch_u32(one, n, 1, one_out, algo=algo, p=args.p),
                                   20, 3, rs, torch)
        ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SORT, n, 4, 0, 8, rs.RS_ALGO_LSD), dtype=torch.uint8,
                         device="cuda")
        lsd_ms, _ = timed_steps(lambda: rs.rs_sort_u32(one, one_out, radix_bits=8, algo=rs.RS_ALGO_LSD, ws=ws),
                                20, 3, rs, torch)
    total = n * count
    launches, tot_ms = prof.get("batch", (0, 0.0))
    avg = tot_ms / launches if launches else float("nan")
    if used in ("btn", "oet"):
        ops = network_ops(used, n, p) * count
        achieved = ops / (avg * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": None, "kernel": "batch",
                "ops_per_launch": ops, "avg_launch_ms": avg}
    else:
        roof = hbm_roofline(prof, "batch", 8 * total)
    res = line(args, total / (ms * 1e-3) / 1e9, ms, "u32",
               "synthetic: %d instances of %d SplitMix64 uniform u32 keys, instance seeds from S0+3"
               % (count, n),
               {"workload": "small-n single arrays, %d instances of n=%d in one launch, %s p=%d"
                            % (count, n, used, p), "n": n, "instances": count, "algo": used, "p": p},
               roof, prof,
               {"us_per_instance_batched": ms * 1e3 / count, "us_single_instance": single_ms * 1e3,
                "us_device_lsd_one_instance": lsd_ms * 1e3})
    if not args.no_cpu:
        import oracle
        k = max(1, min(count, (1 << 22) // n))

        def run():
            for i in range(k):
                if used == "btn":
                    oracle.bitonic_block(host[i], p)
                elif used == "oet":
                    oracle.oet_block(host[i], p)
                else:
                    oracle.lsd(host[i], 8)
        sec = time_oracle(run)
        res["cpu_baseline"] = {
            "value": k * n / sec / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": "first %d instances, serial C oracle %s, pinned to one host core, mean of 4 runs"
                      % (k, {"btn": "o_bitonic_block", "oet": "o_oet_block"}.get(used, "o_lsd")),
            "seconds_per_run": sec,
        }
    return res


# ---- batched segmented ----------------------------------------------------------

def bench_segmented(args, torch, rs, gen, np):
    S = args.segments
    lens = gen.loguniform_lengths(gen.S0 + 4, S, 4.0, 20.0)
    off = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    total = int(off[-1])
    keys = torch.empty(total, dtype=torch.int32, device="cuda")
    gen.uniform_u32_dev(gen.S0 + 4, keys)
    offd = torch.from_numpy(off).cuda()
    out = torch.empty_like(keys)
    ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SEGMENTED, total, 4, 0, 0, rs.RS_ALGO_AUTO, S),
                     dtype=torch.uint8, device="cuda")

    def step():
        rs.rs_sort_segmented(keys, offd, out, ws=ws)

    step()
    torch.cuda.synchronize()
    assert rs.rs_get_stats().device_error == 0
    ms, prof = timed_steps(step, args.steps, args.warmup, rs, torch, launch_timing=True)
    # algorithmic bytes: a segment sorted in LDS is read and written once;
    # the others take four radix-2^8 rounds through HBM, the device-wide
    # rounds shared by the segments of 10,241 .. 14,336 and 16,385 .. 2^30 -
    # 1 keys ("seg_round", four launches a step, each reading and writing
    # their keys once), which dominate.
    shared = ((lens >= 10241) & (lens <= 14336)) | ((lens > 16384) & (lens < (1 << 30)))
    small = ~shared & (lens <= 16384)
    alg = 8 * int(lens[small].sum()) + 32 * int(lens[~small].sum())
    roof = hbm_roofline(prof, "seg_round", 8 * int(lens[shared].sum()))
    # one plain LSD call per array, on a seeded sample of the segments
    rng = np.random.default_rng(int(gen.S0 + 4))
    pick = rng.choice(S, size=min(args.plain_sample, S), replace=False)
    lws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SORT, int(lens.max()), 4, 0, 8, rs.RS_ALGO_LSD),
                      dtype=torch.uint8, device="cuda")
    views = [(keys[off[i]:off[i + 1]], out[off[i]:off[i + 1]]) for i in pick]

    def plain():
        for a, b in views:
            rs.rs_sort_u32(a, b, radix_bits=8, algo=rs.RS_ALGO_LSD, ws=lws)

    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) * S / len(pick)   # scaled to all segments
    res = line(args, total / (ms * 1e-3) / 1e9, ms, "u32",
               "synthetic: %d segments, lengths log-uniform in [16, 2^20) (seed S0+4), "
               "SplitMix64 uniform u32 keys (seed S0+4)" % S,
               {"workload": "batched segmented sort, %d segments, %d keys: four shared radix-2^8 rounds "
                            "for the segments of 10,241 .. 14,336 and 16,385 .. 2^30 - 1 keys, one persistent "
                            "launch (in LDS) for the others"
                            % (S, total), "segments": S, "total_keys": total,
                "keys_in_shared_rounds": int(lens[shared].sum())},
               roof, prof,
               {"hbm_gbs": alg / (ms * 1e-3) / 1e9,
                "plain_per_array_gkeys": total / plain_s / 1e9,
                "plain_per_array_sample": "%d seeded segments, one rs_sort_u32 (LSD, radix 2^8) each, "
                                          "time scaled by %d/%d" % (len(pick), S, len(pick)),
                "speedup_vs_plain_per_array": plain_s / (ms * 1e-3)})
    del ws, lws, views
    if not args.no_cpu:
        import oracle
        k = int(np.searchsorted(off, 1 << 24))
        k = max(1, min(S, k))
        hostk = keys[:off[k]].cpu().numpy().view(np.uint32)
        sub = off[:k + 1].copy()
        sec = time_oracle(lambda: oracle.segmented(hostk, sub))
        res["cpu_baseline"] = {
            "value": int(off[k]) / sec / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": "first %d segments (%d keys), serial C oracle o_segmented, pinned to one host "
                      "core, mean of 4 runs" % (k, int(off[k])),
            "seconds_per_run": sec,
        }
    return res


# ---- learned-CDF buckets ---------------------------------------------------------

def bench_learned(args, torch, rs, gen, np):
    n = 1 << args.log2n
    if args.feature_mode != -1:
        rs.rs_learned_set_opts(feature_mode=args.feature_mode)
    host = {"zipf": gen.zipf_u64, "lognormal": gen.lognormal_u64,
            "mixture": gen.gauss_mix_u64}[args.dist](gen.S0 + 5, n)
    keys = torch.from_numpy(host.view(np.int64)).cuda()
    vals = torch.empty(n, dtype=torch.int64, device="cuda")
    gen.iota_dev(vals)
    ko, vo = torch.empty_like(keys), torch.empty_like(vals)
    ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SORT_KV, n, 8, 8, 0, rs.RS_ALGO_LEARNED),
                     dtype=torch.uint8, device="cuda")

    def step():
        rs.rs_sort_kv(keys, vals, ko, vo, algo=rs.RS_ALGO_LEARNED, ws=ws)

    step()
    torch.cuda.synchronize()
    st = rs.rs_get_stats()
    assert st.device_error == 0
    ms, prof = timed_steps(step, args.steps, args.warmup, rs, torch, launch_timing=True)

    def plain():
        rs.rs_sort_kv(keys, vals, ko, vo, radix_bits=8, algo=rs.RS_ALGO_LSD, ws=ws)

    plain_ms, _ = timed_steps(plain, max(3, args.steps // 2), 1, rs, torch)

    def plain_skip():
        rs.rs_sort_kv(keys, vals, ko, vo, radix_bits=8, algo=rs.RS_ALGO_AUTO, ws=ws)

    # the same rounds, skipping those whose digit is the same for every key
    skip_ms, _ = timed_steps(plain_skip, max(3, args.steps // 2), 1, rs, torch)
    skipped = rs.rs_get_stats().passes_skipped
    # the same learned path with the network off (buckets from the feature
    # and the calibration alone): what the network costs in time
    old_opts = rs.rs_learned_set_opts(use_network=0)
    try:
        nonet_ms, _ = timed_steps(step, max(3, args.steps // 2), 1, rs, torch)
        st_nonet = rs.rs_get_stats()
    finally:
        rs.rs_learned_set_opts(**old_opts)
    # dominant kernel: the two stable bucket-id rounds, each reading and
    # writing the 2-byte id, the key and the payload
    roof = hbm_roofline(prof, "learn_pass", 2 * n * (2 + 8 + 8))
    res = line(args, n / (ms * 1e-3) / 1e9, ms, "u64",
               "synthetic: %s u64 keys (seed S0+5), u64 payload = original index" % args.dist,
               {"workload": "learned-CDF buckets, n=2^%d u64 keys + u64 payload, %s" % (args.log2n, args.dist),
                "n": n, "dist": args.dist, "feature_mode": rs.rs_learned_get_opts()["feature_mode"]},
               roof, prof,
               {"plain_lsd_gkeys": n / (plain_ms * 1e-3) / 1e9, "plain_lsd_ms": plain_ms,
                "speedup_vs_plain": plain_ms / ms,
                "plain_skip_gkeys": n / (skip_ms * 1e-3) / 1e9, "plain_skip_rounds_skipped": skipped,
                "speedup_vs_plain_skip": skip_ms / ms,
                "feature_only_gkeys": n / (nonet_ms * 1e-3) / 1e9, "network_cost_ms": ms - nonet_ms,
                "feature_only_keys_overflowed": st_nonet.keys_overflowed,
                "fallback": st.fallback, "buckets_overflowed": st.buckets_overflowed,
                "keys_overflowed": st.keys_overflowed, "train_loss": st.train_loss})
    del ws
    if not args.no_cpu:
        import oracle
        m = min(n, 1 << 25)
        kh = np.ascontiguousarray(host[:m])
        vh = np.arange(m, dtype=np.uint64)
        sec = time_oracle(lambda: oracle.lsd(kh, 8, vals=vh))
        res["cpu_baseline"] = {
            "value": m / sec / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": "first 2^%d keys, serial C oracle o_lsd (stable kv, radix 2^8): the oracle "
                      "of the learned path is the stable sort; pinned to one core, mean of 4 runs"
                      % (m.bit_length() - 1),
            "seconds_per_run": sec,
        }
    return res


# ---- BTN / OET at device scale: p runs in HBM -----------------------------------------

def bench_blocks(args, torch, rs, gen, np):
    n = 1 << args.log2n
    name = "oet" if args.algo == "oet" else "btn"
    algo = rs.RS_ALGO_OET if name == "oet" else rs.RS_ALGO_BTN
    p = args.p if args.p else rs.rs_blocks_default_p(n, algo)  # the MBSP model's p
    keys = torch.empty(n, dtype=torch.int32, device="cuda")
    gen.uniform_u32_dev(gen.S0 + 2, keys)
    out = torch.empty_like(keys)
    ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_BLOCKS, n, 4, 0, 0, algo, p), dtype=torch.uint8,
                     device="cuda")

    def step():
        rs.rs_sort_blocks_u32(keys, out, algo=algo, p=p, ws=ws)

    step()
    torch.cuda.synchronize()
    st = rs.rs_get_stats()
    assert st.device_error == 0, "device reported a bounded-wait or range error"
    stages = st.network_stages
    ms, prof = timed_steps(step, args.steps, args.warmup, rs, torch, launch_timing=True)
    # one merge-split stage reads and writes every key of the p runs once
    N = -(-n // p)
    roof = hbm_roofline(prof, "block_merge", 2 * 4 * p * N)
    del ws
    # the plain LSD sort of the same keys, for the comparison the paper draws
    lws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SORT, n, 4, 0, 8, rs.RS_ALGO_LSD), dtype=torch.uint8,
                      device="cuda")
    lsd_ms, _ = timed_steps(lambda: rs.rs_sort_u32(keys, out, algo=rs.RS_ALGO_LSD, ws=lws),
                            max(2, args.steps // 2), 1, rs, torch)
    del lws, out
    torch.cuda.empty_cache()
    config = {
        "workload": "%s on p=%d runs of ceil(n/p) keys in HBM, uint32 keys, n=2^%d: local sort per "
                    "workgroup, then %d merge-split stages" % (name.upper(), p, args.log2n, stages),
        "n": n, "p": p, "stages": stages,
    }
    extra = {"plain_lsd_ms": lsd_ms, "plain_lsd_gkeys": n / (lsd_ms * 1e-3) / 1e9,
             "vs_plain_lsd": lsd_ms / ms}
    if args.mbsp:
        extra["mbsp"] = mbsp_check(args, torch, rs, keys, n, p, name, ms, stages, prof)
    res = line(args, n / (ms * 1e-3) / 1e9, ms, "u32", "synthetic: SplitMix64 uniform keys on the full "
               "range, seed S0+2", config, roof, prof, extra)
    if not args.no_cpu:
        import oracle
        m = min(n, 1 << min(args.cpu_log2n, 22 if name == "oet" else 24))  # OET: p rounds over the sample
        kh = np.ascontiguousarray(keys[:m].cpu().numpy().view(np.uint32))
        fn = (lambda: oracle.oet_block(kh, p)) if name == "oet" else (lambda: oracle.bitonic_block(kh, p))
        sec = time_oracle(fn, runs=2)
        res["cpu_baseline"] = {
            "value": m / sec / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": "first 2^%d keys of the same input, serial C oracle o_%s_block with the same "
                      "p, pinned to one host core, mean of 2 runs"
                      % (m.bit_length() - 1, "oet" if name == "oet" else "bitonic"),
            "seconds_per_run": sec,
        }
    return res


def mbsp_check(args, torch, rs, keys, n, p, name, ms, stages, prof):
    """The MBSP model of Section 3 on this GPU, with a processor read as a
    workgroup.  A run's local sort costs 68 (n/p) G (Eq. TsG: four rounds of
    3 + 2 accesses per key at G, with g = 5G folded in as the paper does,
    here measured instead) and one merge-split stage 4 (n/p) g; G and g are
    calibrated on the network just timed, then used to predict the other
    network (Eqs. ToG, TbG) and the serial sort, T_s = 68 n G (Eq. TsG):
    one workgroup's radix sort of the whole array."""
    import math
    N = -(-n // p)
    local_ms = prof["seg"][1] / prof["seg"][0] if prof.get("seg", (0, 0))[0] else float("nan")
    stage_ms = prof["block_merge"][1] / prof["block_merge"][0]
    G = local_ms * 1e-3 / (68 * N)
    g = stage_ms * 1e-3 / (4 * N)
    lg = int(math.log2(p)) if p & (p - 1) == 0 else math.log2(p)
    other = "oet" if name == "btn" else "btn"
    other_stages = p if other == "oet" else int(lg * (lg + 1) / 2)
    pred_other_ms = local_ms + other_stages * stage_ms
    # the other network, measured
    algo = rs.RS_ALGO_OET if other == "oet" else rs.RS_ALGO_BTN
    if other == "btn" and p & (p - 1):
        other_ms = None
    else:
        out = torch.empty_like(keys)
        ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_BLOCKS, n, 4, 0, 0, algo, p), dtype=torch.uint8,
                         device="cuda")
        other_ms, _ = timed_steps(lambda: rs.rs_sort_blocks_u32(keys, out, algo=algo, p=p, ws=ws), 2, 1, rs, torch)
        del ws, out
    # the serial sort: one workgroup sorts all n keys (one segment, never
    # the device-wide rounds: algo LSD)
    off = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    out = torch.empty_like(keys)
    ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SEGMENTED, n, 4, 0, 0, rs.RS_ALGO_LSD, 1), dtype=torch.uint8,
                     device="cuda")
    serial_ms, _ = timed_steps(lambda: rs.rs_sort_segmented(keys, off, out, algo=rs.RS_ALGO_LSD, ws=ws), 1, 1,
                               rs, torch)
    del ws, out
    btn_ms = ms if name == "btn" else other_ms
    oet_ms = ms if name == "oet" else other_ms
    btn_stages = int(lg * (lg + 1) / 2)
    return {
        "G_ps": G * 1e12, "g_ps": g * 1e12, "g_over_G": g / G,
        "local_sort_ms": local_ms, "stage_ms": stage_ms,
        "predicted_%s_ms" % other: pred_other_ms, "measured_%s_ms" % other: other_ms,
        "oet_over_btn_measured": (oet_ms / btn_ms) if (oet_ms and btn_ms) else None,
        "oet_over_btn_model": (68 + 4 * p * g / G) / (68 + 4 * btn_stages * g / G),
        "serial_one_workgroup_ms": serial_ms, "serial_predicted_ms": 68 * n * G * 1e3,
        "serial_over_btn_measured": (serial_ms / btn_ms) if btn_ms else None,
        "serial_over_btn_model": 68 * p / (68 + 4 * btn_stages * g / G),
    }


def mbsp_radix_check(args, torch, rs, keys, n, bits, ms):
    """The MBSP model of the parallel radix sort (Section 3, Eqs. TsG, Tp,
    Tp4, Tp2) and Observation 7 on this GPU, with a processor read as a
    workgroup slot: p = the workgroups the onesweep round holds at once (2 per
    compute unit).  G is calibrated on the serial sort, T_s = 68 n G (one
    workgroup's radix-2^8 sort of the whole array), and the paper's g = 5G is
    kept, as Eqs. Tp4 and Tp2 do; the model then predicts the device-wide
    sort at radix 2^8 (PR4) and 2^16 (PR2), and Observation 7's bound on the
    speed-up of PR4 over the serial sort, about 68 p / 88 = 0.77 p."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    p = 2 * cus
    off = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    out = torch.empty_like(keys)
    ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SEGMENTED, n, 4, 0, 0, rs.RS_ALGO_LSD, 1), dtype=torch.uint8,
                     device="cuda")
    serial_ms, _ = timed_steps(lambda: rs.rs_sort_segmented(keys, off, out, algo=rs.RS_ALGO_LSD, ws=ws), 1, 1,
                               rs, torch)
    del ws
    G = serial_ms * 1e-3 / (68 * n)
    res = {"p": p, "G_ps": G * 1e12, "serial_one_workgroup_ms": serial_ms}
    for name, b, coef, cnt in (("pr4", 8, 88, 40 * 256), ("pr2", 16, 44, 20 * 256 * 256)):
        if b == bits:
            meas = ms
        else:
            ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SORT, n, 4, 0, b, rs.RS_ALGO_LSD), dtype=torch.uint8,
                             device="cuda")
            meas, _ = timed_steps(lambda: rs.rs_sort_u32(keys, out, radix_bits=b, algo=rs.RS_ALGO_LSD, ws=ws),
                                  3, 1, rs, torch)
            del ws
        pred = (coef * n / p + cnt * p) * G * 1e3
        res[name] = {"measured_ms": meas, "predicted_ms": pred, "predicted_count_exchange_ms": cnt * p * G * 1e3,
                     "speedup_over_serial_measured": serial_ms / meas,
                     "speedup_over_serial_model": serial_ms / pred}
    res["obs7_pr4_speedup_bound"] = 68 * p / 88
    del out
    return res


# ---- the small-n crossover: one array at a time, networks against radix ----------

def bench_crossover(args, torch, rs, gen, np):
    """One array of n uint32 keys per call, n = 2^lo .. 2^hi: the block
    networks (one workgroup up to 16,384 keys at the tuned p, device scale
    above at the MBSP model's p) and the one-workgroup LDS radix sort against
    the device-wide LSD sort, each timed alone (launch latency included);
    the crossover is the smallest n from which LSD is faster than both
    networks."""
    rows = []
    cap = rs.rs_small_capacity(4)
    table = {e[0]: e for e in rs.rs_tune_get()}
    for lg in range(args.cross_lo, args.cross_hi + 1):
        n = 1 << lg
        keys = torch.empty(n, dtype=torch.int32, device="cuda")
        gen.uniform_u32_dev(gen.S0 + 3 + lg, keys)
        out = torch.empty_like(keys)
        lws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SORT, n, 4, 0, 8, rs.RS_ALGO_LSD), dtype=torch.uint8,
                          device="cuda")
        row = {"log2n": lg}
        steps = max(5, args.steps)
        row["lsd_us"] = timed_steps(lambda: rs.rs_sort_u32(keys, out, radix_bits=8, algo=rs.RS_ALGO_LSD,
                                                           ws=lws), steps, 2, rs, torch)[0] * 1e3
        for name, algo in (("btn", rs.RS_ALGO_BTN), ("oet", rs.RS_ALGO_OET)):
            if n <= cap:
                p = table[lg][2] if table[lg][1] == algo else 0
                row[name + "_us"] = timed_steps(lambda: rs.rs_sort_batch_u32(keys, n, 1, out, algo=algo, p=p),
                                                steps, 2, rs, torch)[0] * 1e3
                row[name + "_p"] = rs.rs_get_stats().runs_p
            else:
                p = rs.rs_blocks_default_p(n, algo)
                bws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_BLOCKS, n, 4, 0, 0, algo, p), dtype=torch.uint8,
                                  device="cuda")
                row[name + "_us"] = timed_steps(lambda: rs.rs_sort_blocks_u32(keys, out, algo=algo, p=p, ws=bws),
                                                steps, 2, rs, torch)[0] * 1e3
                row[name + "_p"] = p
                del bws
        if n <= cap:
            row["lds_radix_us"] = timed_steps(lambda: rs.rs_sort_batch_u32(keys, n, 1, out,
                                                                           algo=rs.RS_ALGO_LDS_RADIX),
                                              steps, 2, rs, torch)[0] * 1e3
        # the device-wide LSD sort against the best one-array alternative
        # (the networks, and the one-workgroup LDS radix sort where it fits)
        row["lsd_wins"] = row["lsd_us"] < min(row["btn_us"], row["oet_us"], row.get("lds_radix_us", float("inf")))
        print("crossover n=2^%d: lsd %.1f us  btn %.1f us (p=%d)  oet %.1f us (p=%d)%s" % (
            lg, row["lsd_us"], row["btn_us"], row["btn_p"], row["oet_us"], row["oet_p"],
            ("  lds radix %.1f us" % row["lds_radix_us"]) if "lds_radix_us" in row else ""),
            file=sys.stderr, flush=True)
        rows.append(row)
        del keys, out, lws
        torch.cuda.empty_cache()
    wins = [r["log2n"] for r in rows if r["lsd_wins"]]
    first = None
    for r in rows:                       # the smallest n from which LSD wins at every larger n
        if all(q["lsd_wins"] for q in rows if q["log2n"] >= r["log2n"]):
            first = r["log2n"]
            break
    last = rows[-1]
    n = 1 << last["log2n"]
    best_us = min(last["lsd_us"], last["btn_us"], last["oet_us"])
    res = line(args, n / (best_us * 1e-6) / 1e9, best_us * 1e-3, "u32",
               "synthetic: SplitMix64 uniform u32 keys, one array per call, seed S0+3+lg n",
               {"workload": "small-n crossover: one array of n = 2^%d .. 2^%d uint32 keys per call, BTN / OET "
                            "against LSD radix" % (args.cross_lo, args.cross_hi), "n": n},
               None, {}, {"crossover": rows, "lsd_wins_from_log2n": first, "lsd_wins_at": wins})
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(every sort runs on a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1708_09495_amd as rs

    torch.cuda.set_device(torch.device("cuda:0"))
    if args.log2n is None:
        args.log2n = 27 if args.workload == "blocks" else 28
    tuning = None
    if args.tuning_file:
        rs.rs_tune_load(args.tuning_file)
        tuning = {"file": args.tuning_file}
    if args.tune:
        t0 = time.perf_counter()
        rs.rs_tune_run(instances=args.tune)
        tuning = {"instances": args.tune, "seconds": time.perf_counter() - t0}
        if args.save_tuning:
            rs.rs_tune_save(args.save_tuning)
    if tuning is not None:
        tuning["table"] = [e for e in rs.rs_tune_get() if e[0] >= 1]
    fn = {"lsd": bench_lsd, "small": bench_small, "segmented": bench_segmented,
          "learned": bench_learned, "blocks": bench_blocks, "crossover": bench_crossover}[args.workload]
    res = fn(args, torch, rs, gen, np)
    if tuning is not None:
        res["tuning"] = tuning
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
