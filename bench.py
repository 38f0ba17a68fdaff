#!/usr/bin/env python3
"""Benchmark of the plain LSD radix sort hot path on one MI355X.

One step = one complete rs_sort_u32 call (all count-sort rounds: the fill,
the all-round histogram and the four rank-and-scatter rounds) over 2^28
uint32 keys drawn uniform on [0, 2^32) by SplitMix64, radix 2^8, with the
input already resident in HBM.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
                  [--radix-bits B] [--key-bytes 4|8] [--kv]

The roofline object covers the dominant kernel (the onesweep rank-and-scatter
round): its algorithmic bytes per launch (one read and one write of every key
and value) over its mean launch time, timed with HIP events that the library
records on the launch stream during the timed steps.  The cpu_baseline object
times the serial C oracle on a bounded sample of the same input on one host
core (mean of four runs, as the paper reports its timings).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gkeys/s + HBM GB/s, uint32 n=2^28; batched/learned vs plain radix"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--radix-bits", type=int, default=8)
    ap.add_argument("--key-bytes", type=int, default=4, choices=[4, 8])
    ap.add_argument("--kv", action="store_true", help="stable sort with a payload = index")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-log2n", type=int, default=26)
    return ap.parse_args()


def pmc_traffic(kernel, workload, src_hash):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if one
    exists for this kernel, workload and kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.json" % (kernel, workload))
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != src_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("rs_lsd.hip", "rs_dev.h"):
        with open(os.path.join(ROOT, "paper_1708_09495_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cpu_baseline(args, keys_host):
    import numpy as np

    import oracle
    m = 1 << args.cpu_log2n
    sample = np.ascontiguousarray(keys_host[:m])
    vals = np.arange(m, dtype=np.uint32) if args.kv else None
    times = []
    for _ in range(4):
        t0 = time.perf_counter()
        oracle.lsd(sample, args.radix_bits, vals=vals)
        times.append(time.perf_counter() - t0)
    mean = sum(times) / len(times)
    return {
        "value": m / mean / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
        "sample": "first 2^%d keys of the same input, serial C oracle o_lsd radix 2^%d%s, "
                  "mean of 4 runs on one host core" % (args.cpu_log2n, args.radix_bits,
                                                        ", payload = index" if args.kv else ""),
        "seconds_per_run": mean,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(every sort runs on a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1708_09495_amd as rs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = 1 << args.log2n
    kb = args.key_bytes
    bits = args.radix_bits
    seed = gen.S0 + 2
    kdt = torch.int32 if kb == 4 else torch.int64
    keys = torch.empty(n, dtype=kdt, device=dev)
    (gen.uniform_u32_dev if kb == 4 else gen.uniform_u64_dev)(seed, keys)
    out = torch.empty_like(keys)
    vals = vout = None
    vb = 0
    if args.kv:
        vb = 4
        vals = torch.empty(n, dtype=torch.int32, device=dev)
        gen.iota_dev(vals)
        vout = torch.empty_like(vals)
    op = rs.RS_OP_SORT_KV if args.kv else rs.RS_OP_SORT
    ws = torch.empty(rs.rs_workspace_bytes(op, n, kb, vb, bits, rs.RS_ALGO_LSD), dtype=torch.uint8,
                     device=dev)
    torch.cuda.synchronize()

    def step():
        if args.kv:
            rs.rs_sort_kv(keys, vals, out, vout, radix_bits=bits, algo=rs.RS_ALGO_LSD, ws=ws)
        elif kb == 4:
            rs.rs_sort_u32(keys, out, radix_bits=bits, algo=rs.RS_ALGO_LSD, ws=ws)
        else:
            rs.rs_sort_u64(keys, out, radix_bits=bits, algo=rs.RS_ALGO_LSD, ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = rs.rs_get_stats()
    assert st.device_error == 0, "device reported a bounded-wait error"
    passes = st.passes

    rs.rs_profile_read()          # drop anything recorded before the timed region
    rs.rs_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rs.rs_profile_enable(False)
    prof = rs.rs_profile_read()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gkeys = n / (ms_per_step * 1e-3) / 1e9
    # whole-call algorithmic bytes: one histogram read, then one read + write
    # of keys (and values) per round
    # (wide digits: a counting read of the keys in every round instead)
    wide = bits >= 12
    kname = "wide_scatter" if wide else "onesweep"
    call_bytes = (passes if wide else 1) * n * kb + passes * 2 * n * (kb + vb)
    launches, tot_ms = prof.get(kname, (0, 0.0))
    avg_ms = tot_ms / launches if launches else float("nan")
    bytes_per_launch = 2 * n * (kb + vb)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if launches else None
    workload = "lsd_%s%s_n2p%d_b%d" % ("u32" if kb == 4 else "u64", "_kv32" if args.kv else "",
                                        args.log2n, bits)
    traffic = pmc_traffic(kname, workload, source_hash())
    kernels = {k: {"launches": c, "avg_ms": (t / c if c else None)} for k, (c, t) in prof.items()}

    res = {
        "metric": METRIC,
        "value": gkeys,
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if kb == 4 else "u64",
        "data": "synthetic: SplitMix64 uniform keys on the full range, seed S0+2"
                + (", payload = original index (u32)" if args.kv else ""),
        "config": {
            "workload": "plain LSD radix sort, %s keys%s, n=2^%d, radix 2^%d (%d count-sort rounds)"
                        % ("uint32" if kb == 4 else "uint64",
                           " + uint32 payload (stable)" if args.kv else " only", args.log2n, bits,
                           passes),
            "n": n, "key_bytes": kb, "val_bytes": vb, "radix_bits": bits, "passes": passes,
            "tile_keys": st.tile_keys,
        },
        "hbm_gbs": call_bytes / (ms_per_step * 1e-3) / 1e9,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "kernel": kname, "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms,
        },
        "kernels": kernels,
    }
    if not args.no_cpu:
        kh = keys[: 1 << args.cpu_log2n].cpu().numpy().view(np.uint32 if kb == 4 else np.uint64)
        res["cpu_baseline"] = cpu_baseline(args, kh)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
