"""Pins for the oracle's monotone MLP, Adam step and mid-rank targets (the
learned-CDF extension; not in the paper).

What pins them:
  * the backward pass against central finite differences of the forward loss;
  * forward special cases with closed forms: near-zero weights give
    sigmoid(b3); a network whose second layer has a single live weight
    (o, i) reduces to a short expression that also tells W2 from its
    transpose;
  * monotonicity in x for random parameters (non-negative weights, monotone
    activations);
  * the first two Adam steps from zero moments in closed form;
  * mid-rank targets by brute-force counting.
"""
import math

import numpy as np
import pytest

H = 32
I_V1, I_B1, I_V2, I_B2, I_V3, I_B3 = 0, H, 2 * H, 2 * H + H * H, 3 * H + H * H, 4 * H + H * H


def inv_softplus(w):
    return math.log(math.expm1(w))


def rand_params(seed, scale=0.5):
    """Raw weights near -2 (softplus ~ 0.13) keep every layer out of
    saturation, so no gradient is vanishingly small."""
    rng = np.random.default_rng(seed)
    q = rng.normal(0.0, scale, 4 * H + H * H + 1)
    for lo, hi in ((I_V1, I_B1), (I_V2, I_B2), (I_V3, I_B3)):
        q[lo:hi] -= 2.0
    return q


def test_param_count(orc):
    assert orc.NPARAM == 1153 == I_B3 + 1


def test_backward_matches_central_differences(orc):
    rng = np.random.default_rng(0)
    q = rand_params(1)
    xs = rng.random(17)
    ts = rng.random(17)
    loss, g = orc.mlp_loss_grad_f64(q, xs, ts)
    h = 1e-4   # truncation O(h^2) ~ 1e-8 relative; smaller h is roundoff-bound
    worst = 0.0
    for j in range(q.size):
        qp = q.copy(); qp[j] += h
        qm = q.copy(); qm[j] -= h
        fd = (orc.mlp_loss_grad_f64(qp, xs, ts)[0] - orc.mlp_loss_grad_f64(qm, xs, ts)[0]) / (2 * h)
        err = abs(fd - g[j]) / max(1e-7, abs(fd) + abs(g[j]))
        worst = max(worst, err)
    assert worst < 1e-6, worst


def test_loss_is_mean_squared_error(orc):
    q = rand_params(2)
    xs = np.array([0.0, 0.25, 1.0])
    ts = np.array([0.1, 0.5, 0.9])
    loss, _ = orc.mlp_loss_grad_f64(q, xs, ts)
    ys = [orc.mlp_forward_f64(q, x) for x in xs]
    assert loss == pytest.approx(sum((y - t) ** 2 for y, t in zip(ys, ts)) / 3, rel=1e-14)


def test_forward_near_zero_weights_is_sigmoid_of_output_bias(orc):
    q = np.full(1153, -60.0)   # softplus(-60) ~ 1e-26
    q[I_B1:I_B1 + H] = 0.3
    q[I_B2:I_B2 + H] = -0.2
    q[I_B3] = 0.7
    for x in (0.0, 0.5, 1.0):
        assert orc.mlp_forward_f64(q, x) == pytest.approx(1 / (1 + math.exp(-0.7)), abs=1e-15)


def test_forward_single_live_weight_closed_form(orc):
    q = np.full(1153, -60.0)
    a1, b1 = 2.0, -0.5        # w1[5], b1[5]
    a2, b2o = 1.5, 0.25       # w2[3][5], b2[3]
    a3, b3 = 3.0, -1.0        # w3[3], b3
    q[I_B1:I_B1 + H] = 0.0
    q[I_B2:I_B2 + H] = 0.0
    q[I_V1 + 5] = inv_softplus(a1); q[I_B1 + 5] = b1
    q[I_V2 + 3 * H + 5] = inv_softplus(a2); q[I_B2 + 3] = b2o
    q[I_V3 + 3] = inv_softplus(a3); q[I_B3] = b3
    for x in (0.0, 0.3, 0.9):
        h15 = math.tanh(a1 * x + b1)
        h23 = math.tanh(a2 * h15 + b2o)
        y = 1 / (1 + math.exp(-(a3 * h23 + b3)))
        assert orc.mlp_forward_f64(q, x) == pytest.approx(y, rel=1e-12)
    # the transposed layer (w2[5][3]) must give a different value
    qt = q.copy()
    qt[I_V2 + 3 * H + 5] = -60.0
    qt[I_V2 + 5 * H + 3] = inv_softplus(a2)
    assert abs(orc.mlp_forward_f64(qt, 0.9) - orc.mlp_forward_f64(q, 0.9)) > 1e-3


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_forward_is_monotone(orc, seed):
    q = rand_params(seed, 1.5)
    xs = np.linspace(0, 1, 2001)
    ys = np.array([orc.mlp_forward_f64(q, x) for x in xs])
    assert np.all(np.diff(ys) >= 0)
    y32 = np.array([orc.mlp_forward_f32(q.astype(np.float32), np.float32(x)) for x in xs])
    assert np.max(np.abs(y32 - ys)) < 1e-5


def test_adam_first_two_steps_closed_form(orc):
    rng = np.random.default_rng(7)
    n = 50
    p = rng.normal(size=n)
    g1 = rng.normal(size=n)
    g2 = rng.normal(size=n)
    m1 = np.zeros(n); m2 = np.zeros(n)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    p0 = p.copy()
    orc.adam_step_f64(p, g1, m1, m2, 1, lr, b1, b2, eps)
    # step 1: bias-corrected moments are g and g^2, so the step is lr g/(|g| + eps)
    np.testing.assert_allclose(p, p0 - lr * g1 / (np.abs(g1) + eps), rtol=1e-13, atol=1e-15)
    p1 = p.copy()
    orc.adam_step_f64(p, g2, m1, m2, 2, lr, b1, b2, eps)
    mh = ((1 - b1) * b1 * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = ((1 - b2) * b2 * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    np.testing.assert_allclose(p, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=1e-12, atol=1e-15)


def test_midrank_targets_brute_force(orc):
    rng = np.random.default_rng(8)
    for trial in range(200):
        m = int(rng.integers(1, 40))
        s = np.sort(rng.integers(0, 8, m)).astype(np.uint64)
        t = orc.midrank_targets(s)
        for i in range(m):
            lt = sum(1 for x in s if x < s[i])
            le = sum(1 for x in s if x <= s[i])
            assert t[i] == pytest.approx((lt + le) / (2 * m), abs=0)
