"""GPU tests of the learned-CDF bucket path (an extension; not in the
paper): the network's forward pass and gradient against the fp64 oracle, and
the sort itself bit for bit against the oracle's stable LSD sort, including
the fallback paths forced from the host."""
import numpy as np
import pytest

from gpu_util import first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

H = 32
I_V1, I_B1, I_V2, I_B2, I_V3, I_B3 = 0, H, 2 * H, 2 * H + H * H, 3 * H + H * H, 4 * H + H * H


@pytest.fixture(scope="module")
def rs():
    import paper_1708_09495_amd as rs
    rs.lib()
    return rs


def _params(seed):
    rng = np.random.default_rng(seed)
    q = rng.normal(0.0, 0.5, 1153)
    for lo, hi in ((I_V1, I_B1), (I_V2, I_B2), (I_V3, I_B3)):
        q[lo:hi] -= 2.0
    return q


def _f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_forward_matches_fp64_oracle(rs, orc):
    for seed in (1, 2, 3):
        q = _params(seed)
        x = np.linspace(0, 1, 4097)
        y = rs.rs_mlp_forward(_f32(q), _f32(x)).cpu().numpy().astype(np.float64)
        ref = np.array([orc.mlp_forward_f64(q.astype(np.float32).astype(np.float64), xi)
                        for xi in x.astype(np.float32)])
        assert np.max(np.abs(y - ref) / np.maximum(np.abs(ref), 1e-3)) < 1e-4
        assert np.all(np.diff(y) >= -1e-7)          # monotone up to float rounding


def test_gradient_matches_fp64_oracle(rs, orc):
    """Every one of the 1,153 gradient entries against the fp64 oracle:
    |g - g_ref| <= 1e-4 max(|g_ref|, s), where s is the mean over the
    samples of |per-sample gradient| of that entry (the scale at which an
    fp32 sum of those terms rounds; an entry whose terms cancel is held to
    that scale, not to its near-zero total)."""
    rng = np.random.default_rng(4)
    worst = 0.0
    for seed, m in ((5, 1000), (6, 4096), (7, 777)):
        q = _params(seed).astype(np.float32).astype(np.float64)
        xs = rng.random(m).astype(np.float32).astype(np.float64)
        ts = rng.random(m).astype(np.float32).astype(np.float64)
        g = rs.rs_mlp_loss_grad(_f32(q), _f32(xs), _f32(ts)).cpu().numpy().astype(np.float64)
        loss_ref, g_ref = orc.mlp_loss_grad_f64(q, xs, ts)
        scale = np.zeros(1153)
        for i in range(m):
            scale += np.abs(orc.mlp_loss_grad_f64(q, xs[i:i + 1], ts[i:i + 1])[1])
        scale /= m
        err = np.abs(g[:1153] - g_ref)
        bound = 1e-4 * np.maximum(np.abs(g_ref), scale)
        ratio = err / np.maximum(bound, 1e-300)
        worst = max(worst, float(ratio.max()))
        bad = np.nonzero(err > bound)[0]
        assert bad.size == 0, "m=%d entry %d: %g vs %g (bound %g)" % (
            m, bad[0], g[bad[0]], g_ref[bad[0]], bound[bad[0]])
        assert abs(g[1153] / m - loss_ref) / loss_ref < 1e-5
    print("largest error / bound: %.3g" % worst)


def test_adam_step_matches_fp64_oracle(rs, orc):
    """The update training applies after each gradient (rs_mlp_adam_step,
    the kernel the learned path runs) against the oracle's fp64 Adam step on
    the same float32 inputs, entry by entry: moments to a few float32 ulps,
    parameters to 2 ulps of the parameter plus 1e-5 of the step taken."""
    import torch
    rng = np.random.default_rng(8)
    n = 1153
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    f = lambda v: float(np.float32(v))
    for step in (0, 1, 9, 99):
        p = rng.normal(0, 1, n).astype(np.float32)
        m1 = (rng.normal(0, 1e-2, n) if step else np.zeros(n)).astype(np.float32)
        m2 = (rng.random(n) * 1e-4 if step else np.zeros(n)).astype(np.float32)
        g = (rng.normal(0, 1, n) * 10.0 ** rng.integers(-9, 1, n)).astype(np.float32)
        g[:5] = 0.0
        dp, d1, d2, dg = _f32(p), _f32(m1), _f32(m2), _f32(g)
        rs.rs_mlp_adam_step(dp, d1, d2, dg, step, lr, b1, b2, eps)
        torch.cuda.synchronize()
        rp, r1, r2 = p.astype(np.float64), m1.astype(np.float64), m2.astype(np.float64)
        orc.adam_step_f64(rp, g.astype(np.float64), r1, r2, step + 1, lr=f(lr), beta1=f(b1), beta2=f(b2),
                          eps=f(eps))
        gp, g1, g2 = (t.cpu().numpy().astype(np.float64) for t in (dp, d1, d2))

        def ulps(*terms):
            # float32 spacing at the largest of the terms a result is summed from
            big = np.max(np.abs(np.stack(terms)), axis=0).astype(np.float32)
            return np.spacing(big).astype(np.float64)

        g64 = g.astype(np.float64)
        e1 = np.abs(g1 - r1)
        e2 = np.abs(g2 - r2)
        assert np.all(e1 <= 4 * ulps(b1 * m1, (1 - b1) * g64, r1)), step
        assert np.all(e2 <= 4 * ulps(b2 * m2, (1 - b2) * g64 * g64, r2)), step
        # the step lr (m1/c1) / (sqrt(m2/c2) + eps) carries the moments'
        # relative errors, plus a few float32 roundings of its own
        step_ref = np.abs(rp - p.astype(np.float64))
        rel = 1e-5 + e1 / np.maximum(np.abs(r1), 1e-300) + 0.5 * e2 / np.maximum(r2, 1e-300)
        bound = 2 * ulps(p, rp) + step_ref * rel
        bad = np.nonzero(np.abs(gp - rp) > bound)[0]
        assert bad.size == 0, "step %d entry %d: %r vs %r" % (step, bad[0], gp[bad[0]], rp[bad[0]])
        assert np.array_equal(dg.cpu().numpy(), g)      # the gradient is only read


def _dist(name, n, seed):
    import gen
    return {"zipf": lambda: gen.zipf_u64(seed, n),
            "lognormal": lambda: gen.lognormal_u64(seed, n),
            "mixture": lambda: gen.gauss_mix_u64(seed, n),
            "uniform": lambda: gen.uniform_u64(seed, n)}[name]()


def _learned(rs, keys, vals=None):
    kt = to_dev(keys)
    if vals is None:
        out = rs.rs_sort_u64(kt, algo=rs.RS_ALGO_LEARNED)
        return to_host(out, np.uint64), None, rs.rs_get_stats()
    ko, vo = rs.rs_sort_kv(kt, to_dev(vals), algo=rs.RS_ALGO_LEARNED)
    return to_host(ko, np.uint64), to_host(vo, np.uint64), rs.rs_get_stats()


@pytest.mark.parametrize("dist", ["zipf", "lognormal", "mixture", "uniform"])
def test_learned_kv_parity(rs, orc, dist):
    import gen
    for n in (1 << 20, (1 << 22) + 977):
        print("case learned kv %s n=%d" % (dist, n), flush=True)
        keys = _dist(dist, n, gen.S0 + 5)
        vals = np.arange(n, dtype=np.uint64)
        ko, vo, st = _learned(rs, keys, vals)
        rk, rv = orc.lsd(keys, 8, vals=vals)
        assert first_mismatch(ko, rk) is None
        assert first_mismatch(vo, rv) is None
        assert st.algo == rs.RS_ALGO_LEARNED and st.device_error == 0
        print("  loss %.3g overflowed buckets %d keys %d fallback %d" %
              (st.train_loss, st.buckets_overflowed, st.keys_overflowed, st.fallback))


def test_learned_keys_only(rs, orc):
    import gen
    keys = gen.lognormal_u64(gen.S0 + 6, 1 << 20)
    ko, _, st = _learned(rs, keys)
    assert first_mismatch(ko, orc.lsd(keys, 8)) is None


@pytest.mark.parametrize("opts", [dict(bucket_cap=2), dict(bucket_cap=16),
                                  dict(use_network=0), dict(feature_mode=0), dict(feature_mode=1),
                                  dict(train_steps=0)])
def test_learned_forced_paths_stay_exact(rs, orc, opts):
    import gen
    old = rs.rs_learned_set_opts(**opts)
    try:
        keys = gen.gauss_mix_u64(gen.S0 + 7, 300_001)
        vals = np.arange(keys.size, dtype=np.uint64)
        ko, vo, st = _learned(rs, keys, vals)
        rk, rv = orc.lsd(keys, 8, vals=vals)
        assert first_mismatch(ko, rk) is None and first_mismatch(vo, rv) is None
        if "bucket_cap" in opts:
            # buckets over the capacity go through the one-workgroup rounds
            assert st.buckets_overflowed > 0 and st.fallback == 0
    finally:
        rs.rs_learned_set_opts(**old)


@pytest.mark.parametrize("whole", [False, True])
def test_learned_giant_bucket_fallbacks(rs, orc, whole):
    """2.5M distinct keys within 2^40 of 2^63 next to 300K small keys,
    bucketed by a linear feature without the network: the dense cluster is
    one float value of the feature, hence one bucket, far more keys than one
    workgroup sorts.  It is sorted by the device-wide LSD rounds
    (whole=False), or the whole array is (whole=True); exact either way."""
    old = rs.rs_learned_set_opts(use_network=0, feature_mode=0,
                                 fallback_frac=(0.0 if whole else 1.0))
    try:
        rng = np.random.default_rng(12)
        small = rng.permutation(300_000).astype(np.uint64)
        high = (np.uint64(1) << np.uint64(63)) + rng.integers(0, 1 << 40, 2_500_000).astype(np.uint64)
        keys = rng.permutation(np.concatenate([small, high]))
        vals = np.arange(keys.size, dtype=np.uint64)
        ko, vo, st = _learned(rs, keys, vals)
        rk, rv = orc.lsd(keys, 8, vals=vals)
        assert first_mismatch(ko, rk) is None and first_mismatch(vo, rv) is None
        assert st.fallback == (1 if whole else 0)
        assert st.keys_overflowed >= 2_500_000
    finally:
        rs.rs_learned_set_opts(**old)


def test_small_and_in_place_take_lsd(rs, orc):
    import gen
    keys = gen.zipf_u64(gen.S0 + 8, 1000)
    ko, _, st = _learned(rs, keys)
    assert st.fallback == 1 and first_mismatch(ko, np.sort(keys)) is None
    big = gen.zipf_u64(gen.S0 + 8, 1 << 17)
    t = to_dev(big)
    rs.rs_sort_u64(t, t, algo=rs.RS_ALGO_LEARNED)
    assert first_mismatch(to_host(t, np.uint64), np.sort(big)) is None


def test_network_gain_over_feature_only(rs):
    """What the trained network buys over the method without it: how evenly
    keys spread over the 65,536 buckets, measured as the share of keys in
    buckets holding more than twice the mean (bucket capacity set to
    2 n / 65,536), with the network and with the feature alone (same
    calibration knots).  On the key's log-scaled global position (feature
    mode 1) the network is the CDF model, and it halves that share on
    lognormal and uniform keys.  On the default feature (mode 2: the key's
    place among 4,096 sample key quantiles) the feature already carries the
    sample CDF; there the network must not make things worse."""
    import gen
    n = 1 << 22
    cap = 2 * n // 65536
    res = {}
    for mode, dists in ((1, ("lognormal", "uniform")), (2, ("mixture", "lognormal", "zipf"))):
        for dist in dists:
            keys = _dist(dist, n, gen.S0 + 9)
            vals = np.arange(n, dtype=np.uint64)
            # mode 1: 32 Adam steps (the network has the whole CDF to learn);
            # mode 2: the default training
            steps = 32 if mode == 1 else rs.rs_learned_get_opts()["train_steps"]
            old = rs.rs_learned_set_opts(fallback_frac=1.0, max_fallback_buckets=1 << 30, bucket_cap=cap,
                                         feature_mode=mode, train_steps=steps)
            try:
                _, _, st_net = _learned(rs, keys, vals)
                rs.rs_learned_set_opts(use_network=0)
                _, _, st_feat = _learned(rs, keys, vals)
            finally:
                rs.rs_learned_set_opts(**old)
            res[(mode, dist)] = (st_net.keys_overflowed / n, st_feat.keys_overflowed / n, st_net.train_loss)
            print("mode %d %-9s keys in buckets over 2x the mean: network %.4f  feature only %.4f  (loss %.2e)"
                  % ((mode, dist) + res[(mode, dist)]), flush=True)
    for dist in ("lognormal", "uniform"):
        net, feat, _ = res[(1, dist)]
        assert net < 0.75 * feat, dist
    for dist in ("mixture", "lognormal", "zipf"):
        net, feat, loss = res[(2, dist)]
        assert net <= 1.5 * feat + 2e-4 and loss < 1e-4, dist


def _quantile_splitters(keys):
    """65,535 splitters at the keys' own quantiles (non-decreasing)."""
    srt = np.sort(keys)
    j = np.arange(1, 65536, dtype=np.uint64)
    return srt[(j * np.uint64(keys.size)) // np.uint64(65536)]


def test_injected_weights_are_used_and_output_exact(rs, orc):
    """rs_mlp_set_weights: the learned path takes the caller's parameters
    instead of training.  A flat network (output weights softplus(-30),
    about 1e-13) gives every key the same output, so every key falls in one
    bucket, far beyond what one workgroup sorts: all n keys are reported
    overflowed and the output is still the stable sort.  Random weights give
    some other spread; the output is exact again.  Clearing the hook brings
    training back."""
    import gen
    n = (1 << 20) + 4097
    keys = gen.lognormal_u64(gen.S0 + 13, n)
    vals = np.arange(n, dtype=np.uint64)
    rk, rv = orc.lsd(keys, 8, vals=vals)
    flat = _params(21).astype(np.float32)
    flat[I_V3:I_B3] = -30.0
    try:
        for w, all_over in ((flat, True), (_params(22).astype(np.float32), False)):
            rs.rs_mlp_set_weights(w)
            ko, vo, st = _learned(rs, keys, vals)
            assert first_mismatch(ko, rk) is None and first_mismatch(vo, rv) is None
            assert st.device_error == 0 and st.train_loss == 0.0
            if all_over:
                assert st.keys_overflowed == n and st.buckets_overflowed == 1
    finally:
        rs.rs_mlp_set_weights(None)
    ko, vo, st = _learned(rs, keys, vals)
    assert st.train_loss > 0.0 and first_mismatch(vo, rv) is None


def test_out_of_order_splitters_stay_exact(rs, orc):
    """Splitters injected out of order (a block of them reversed) in place of
    the derived ones: the bucket search is a fixed binary decision tree, so
    the key-to-bucket map stays monotone whatever the splitters' order, and
    a bucket whose bounds are out of order ranks on its keys' own range.
    The output is the stable sort and no fallback fires (the overflow
    thresholds are disabled); the same with the splitters sorted."""
    import gen
    n = (1 << 20) + 333
    keys = gen.gauss_mix_u64(gen.S0 + 14, n)
    vals = np.arange(n, dtype=np.uint64)
    rk, rv = orc.lsd(keys, 8, vals=vals)
    good = _quantile_splitters(keys)
    bad = good.copy()
    bad[20000:30000] = bad[20000:30000][::-1].copy()
    old = rs.rs_learned_set_opts(fallback_frac=1.0, max_fallback_buckets=1 << 30)
    try:
        for spl in (good, bad):
            rs.rs_learned_debug_fault(rs.RS_LEARNED_FAULT_SPLITTERS, spl)
            ko, vo, st = _learned(rs, keys, vals)
            assert first_mismatch(ko, rk) is None and first_mismatch(vo, rv) is None
            assert st.fallback == 0 and st.device_error == 0
    finally:
        rs.rs_learned_debug_fault(rs.RS_LEARNED_FAULT_NONE)
        rs.rs_learned_set_opts(**old)


@pytest.mark.parametrize("kv", [True, False])
def test_planted_bucket_error_takes_the_check_fallback(rs, orc, kv):
    """A bucket-sort error planted after the buckets are sorted (the first
    and last output pairs swapped): the final sortedness check catches it
    and the whole array is sorted again by the LSD rounds from the untouched
    input.  No other fallback can fire (overflow thresholds disabled), so
    the fallback flag shows the check at work; the output is exact."""
    import gen
    n = (1 << 20) + 777
    keys = gen.lognormal_u64(gen.S0 + 15, n)
    vals = np.arange(n, dtype=np.uint64) if kv else None
    ref = orc.lsd(keys, 8, vals=vals)
    old = rs.rs_learned_set_opts(fallback_frac=1.0, max_fallback_buckets=1 << 30)
    try:
        for fault, expect_fb in ((rs.RS_LEARNED_FAULT_NONE, 0), (rs.RS_LEARNED_FAULT_SWAP, 1)):
            print("case planted fault %d kv %d" % (fault, kv), flush=True)
            rs.rs_learned_debug_fault(fault)
            ko, vo, st = _learned(rs, keys, vals)
            if kv:
                assert first_mismatch(ko, ref[0]) is None and first_mismatch(vo, ref[1]) is None
            else:
                assert first_mismatch(ko, ref) is None
            assert st.fallback == expect_fb and st.device_error == 0
    finally:
        rs.rs_learned_debug_fault(rs.RS_LEARNED_FAULT_NONE)
        rs.rs_learned_set_opts(**old)


@pytest.mark.parametrize("dist,opts", [("lognormal", {}), ("zipf", {}), ("mixture", {}), ("uniform", {}),
                                       ("mixture", dict(use_network=0)), ("lognormal", dict(feature_mode=1)),
                                       ("mixture", dict(feature_mode=0))])
def test_splitters_match_direct_bucket_map(rs, dist, opts):
    """The splitter form of inference against its definition: for every
    key, the bucket the splitter search assigns equals the bucket from
    evaluating the feature, the network and the calibration on the key
    itself (splitter j is the smallest key reaching bucket j, found by
    inverting the map in feature space, then in key space).  Along the
    sorted keys the direct map is non-decreasing (monotone network)."""
    import gen
    import torch
    old = rs.rs_learned_set_opts(**opts) if opts else None
    try:
        n = (1 << 20) + 17
        print("case splitters %s %s" % (dist, opts), flush=True)
        keys = _dist(dist, n, gen.S0 + 9)
        direct = torch.full((n,), -1, dtype=torch.int16, device="cuda")
        assigned = torch.full((n,), -1, dtype=torch.int16, device="cuda")
        rs.rs_learned_debug_ids(direct, assigned)
        try:
            ko, _, st = _learned(rs, keys)
        finally:
            rs.rs_learned_debug_ids()
        assert st.fallback == 0 and st.device_error == 0
        d = to_host(direct, np.uint16).astype(np.int64)
        a = to_host(assigned, np.uint16).astype(np.int64)
        bad = np.nonzero(d != a)[0]
        assert bad.size == 0, "%d keys differ, first key %d: direct %d, splitters %d" % (
            bad.size, keys[bad[0]], d[bad[0]], a[bad[0]])
        order = np.argsort(keys, kind="stable")
        assert np.all(np.diff(d[order]) >= 0)
        assert first_mismatch(ko, np.sort(keys)) is None
    finally:
        if old is not None:
            rs.rs_learned_set_opts(**old)
