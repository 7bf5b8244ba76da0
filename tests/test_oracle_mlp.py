"""Pins of the oracle's network: modified softplus (Sec. 5, Eq. 22), forward special
cases, finite-difference gradients of the log-radiance loss, and Adam's closed form."""
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")
OFF = dict(W1=0, B1=1280, W2=1344, B2=5440, W3=5504, B3=9600, W4=9664, B4=9728)


def test_softplus_mod_closed_forms(O):
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))["softplus_mod"]
    assert O.softplus_mod(0.0) == pytest.approx(g["value_at_0"], rel=1e-15)
    assert O.softplus_mod_grad(0.0) == g["slope_at_0"]
    assert O.softplus_mod_grad(-1e-12) == pytest.approx(0.5, rel=1e-9)   # C1 at zero
    for z in (-30.0, -3.0, -0.5):
        assert O.softplus_mod(z) == pytest.approx(math.log(1 + math.exp(z)), rel=1e-14)
        assert O.softplus_mod_grad(z) == pytest.approx(1 / (1 + math.exp(-z)), rel=1e-14)
    for z in (0.25, 3.0, 100.0):
        assert O.softplus_mod(z) == pytest.approx(0.5 * z + math.log(2), rel=1e-15)
        assert O.softplus_mod_grad(z) == 0.5


def test_param_count():
    assert 20 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 9729


def test_forward_bias_only(O):
    P = np.zeros(9729)
    P[OFF["B4"]] = -1.3
    y, z = O.mlp_forward(P, np.random.default_rng(0).normal(size=(5, 20)))
    assert np.all(z == -1.3) and np.allclose(y, math.log1p(math.exp(-1.3)), rtol=1e-15)


def test_forward_single_path_network(O):
    # one active unit per layer: z = w4 * relu(w3 * relu(w2 * relu(w1 * x_k + b1) + b2) + b3) + b4
    P = np.zeros(9729)
    k = 7
    P[OFF["W1"] + 20 * 5 + k] = 2.0   # unit 5 of layer 1 reads input k
    P[OFF["B1"] + 5] = -0.5
    P[OFF["W2"] + 64 * 9 + 5] = 1.5   # unit 9 of layer 2 reads unit 5
    P[OFF["W3"] + 64 * 63 + 9] = -0.75
    P[OFF["B3"] + 63] = 2.0
    P[OFF["W4"] + 63] = 0.5
    P[OFF["B4"]] = 0.1
    x = np.zeros((4, 20))
    x[:, k] = [-1.0, 0.2, 1.0, 3.0]
    relu = lambda v: np.maximum(v, 0)
    expect = 0.5 * relu(-0.75 * relu(1.5 * relu(2.0 * x[:, k] - 0.5)) + 2.0) + 0.1
    y, z = O.mlp_forward(P, x)
    assert np.allclose(z, expect, rtol=1e-15)
    assert np.allclose(y, [O.softplus_mod(v) for v in expect], rtol=1e-15)


def test_gradient_finite_differences(O):
    rng = np.random.default_rng(1)
    P = rng.normal(0, 0.4, size=9729)
    x = rng.normal(size=(6, 20))
    tgt = rng.uniform(0.0, 3.0, size=6)
    loss, g = O.mlp_loss_grad(P, x, tgt, 0.01)
    assert loss > 0
    # relative check on a random subset of coordinates, central differences in FP64
    idx = np.concatenate([rng.choice(9729, 150, replace=False), [9728, 9664, 1280, 0]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        num = (O.mlp_loss_grad(Pp, x, tgt, 0.01)[0] - O.mlp_loss_grad(Pm, x, tgt, 0.01)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, i


def test_relative_l2_gradient_is_the_frozen_denominator_derivative(O):
    # with sg(y) in the denominator the gradient equals the derivative of
    # sum (y(theta) - L)^2 / (y0^2 + eps) / n with y0 frozen at the current parameters
    rng = np.random.default_rng(11)
    P = rng.normal(0, 0.4, size=9729)
    x = rng.normal(size=(5, 20))
    tgt = rng.uniform(0.0, 3.0, size=5)
    loss, g = O.mlp_loss_grad(P, x, tgt, 0.01, O.LOSS_REL_L2)
    y0, _ = O.mlp_forward(P, x)
    assert loss == pytest.approx(np.mean((y0 - tgt) ** 2 / (y0 ** 2 + 0.01)), rel=1e-14)
    def surrogate(Q):
        y, _ = O.mlp_forward(Q, x)
        return np.mean((y - tgt) ** 2 / (y0 ** 2 + 0.01))
    h = 1e-6
    for i in np.concatenate([rng.choice(9729, 80, replace=False), [9728, 9700, 1300, 3]]):
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        num = (surrogate(Pp) - surrogate(Pm)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, i


def test_relative_l2_minimiser_is_the_mean(O):
    # Bias-only network (y = softplus_mod(b4) on every row): the root of the oracle's own
    # gradient in b4 (found by bisection) is the stationary point of each loss.  On noisy
    # targets (5 % at 20, else 0; mean 1) the relative L2 settles at the mean, the log loss
    # far below it (at the geometric mean of L + eps, minus eps).
    tgt = np.zeros(400)
    tgt[::20] = 20.0
    x = np.zeros((tgt.size, 20))
    expect_log = math.exp(np.mean(np.log(tgt + 0.01))) - 0.01
    for kind, want, rel in ((O.LOSS_REL_L2, None, None), (O.LOSS_LOG_MSE, expect_log, 1e-6)):
        lo, hi = -20.0, 20.0
        for _ in range(60):
            P = np.zeros(9729)
            P[OFF["B4"]] = 0.5 * (lo + hi)
            _, g = O.mlp_loss_grad(P, x, tgt, 0.01, kind)
            if g[OFF["B4"]] > 0:
                hi = P[OFF["B4"]]
            else:
                lo = P[OFF["B4"]]
        y = O.softplus_mod(0.5 * (lo + hi))
        if kind == O.LOSS_REL_L2:
            # stationary point of sum (y - L)/(y^2 + eps) = 0 is the sample mean
            assert y == pytest.approx(tgt.mean(), rel=1e-6)
        else:
            assert y == pytest.approx(want, rel=rel) and y < 0.1 * tgt.mean()


def test_loss_value_definition(O):
    P = np.zeros(9729)
    P[OFF["B4"]] = 0.0  # y = ln 2 for every row
    tgt = np.array([0.0, 1.0, 5.0])
    loss, _ = O.mlp_loss_grad(P, np.zeros((3, 20)), tgt, 0.01)
    expect = np.mean((math.log(math.log(2) + 0.01) - np.log(tgt + 0.01)) ** 2)
    assert loss == pytest.approx(expect, rel=1e-14)


def test_adam_closed_form(O):
    # constant gradient: m_hat = g, v_hat = g^2 at every step -> w moves by lr * g / (|g| + eps)
    rng = np.random.default_rng(2)
    g = rng.normal(size=50)
    w = rng.normal(size=50)
    w0 = w.copy()
    m, v = np.zeros(50), np.zeros(50)
    lr, eps = 5e-3, 1e-8
    for step in range(1, 11):
        O.adam(w, m, v, g, step, lr, 0.9, 0.999, eps)
        expect = w0 - step * lr * g / (np.abs(g) + eps)
        assert np.allclose(w, expect, rtol=1e-12, atol=1e-15)


def test_bfloat16_rounding_special_values(O):
    # bfloat16 keeps 8 significant bits: the spacing above 1 is 2^-7
    assert O.round_bf16(1.0) == 1.0
    assert O.round_bf16(1.0 + 2 ** -8) == 1.0                   # tie -> even mantissa
    assert O.round_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6     # tie -> even (up)
    assert O.round_bf16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
    assert O.round_bf16(-3.0) == -3.0
    assert O.round_bf16(0.1) == pytest.approx(0.1, rel=2 ** -8)


def test_e4m3_rounding_special_values(O):
    # OCP E4M3: 3 mantissa bits, exponent bias 7, largest normal 448, subnormal step 2^-9
    assert O.round_e4m3(448.0) == 448.0
    assert O.round_e4m3(500.0) == 448.0 and O.round_e4m3(-1e6) == -448.0   # saturate
    assert O.round_e4m3(1.0625) == 1.0                          # tie between 1 and 1.125 -> even
    assert O.round_e4m3(1.1875) == 1.25                         # tie between 1.125 and 1.25 -> even
    assert O.round_e4m3(17.0) == 16.0 and O.round_e4m3(19.0) == 20.0
    assert O.round_e4m3(2 ** -9) == 2 ** -9                     # smallest subnormal
    assert O.round_e4m3(2 ** -10) == 0.0                        # tie -> even (zero)
    assert O.round_e4m3(3 * 2 ** -10) == 2 ** -8                # tie -> even (2 steps)
    assert O.round_e4m3(2 ** -6) == 2 ** -6                     # smallest normal
    assert O.round_e4m3(0.0) == 0.0


def test_quantized_forward_reduces_to_exact_for_representable_weights(O):
    # weights and inputs already on the BF16 / E4M3 grids (small integers x powers of two,
    # activations staying representable) give the exact network output
    rng = np.random.default_rng(21)
    P = np.zeros(9729)
    P[:1280] = rng.integers(-2, 3, size=1280) * 0.25
    P[1344:5440] = rng.integers(-2, 3, size=4096) * 2.0 ** -5
    P[5504:9600] = rng.integers(-2, 3, size=4096) * 2.0 ** -5
    P[9664:9728] = rng.normal(size=64)
    x = rng.integers(-2, 3, size=(50, 20)).astype(np.float64)
    y, z = O.mlp_forward(P, x)
    yb, zb = O.mlp_forward_quant(P, x, 1)
    assert np.allclose(zb, z, rtol=1e-2, atol=1e-2)
    y8, z8 = O.mlp_forward_quant(P, x, 2)
    assert np.allclose(z8, z, rtol=0.1, atol=0.1)
    # and quantization moves a generic network by a bounded amount
    Pg = rng.normal(0, 0.2, size=9729)
    xg = rng.normal(size=(200, 20))
    yg, _ = O.mlp_forward(Pg, xg)
    ybg, _ = O.mlp_forward_quant(Pg, xg, 1)
    y8g, _ = O.mlp_forward_quant(Pg, xg, 2)
    assert np.median(np.abs(ybg / yg - 1)) < 1e-2
    assert np.median(np.abs(y8g / yg - 1)) < 6e-2


# ------------------------------------------------------------- near-tie flags of the quantized forward
# A row is flagged when one of its rounding decisions (an activation's BF16 / E4M3 rounding, or
# the power-of-two scale of a vertex's FP8 activations) lies within the accumulation error of
# the matrix core from changing.  These rows are built so that one layer-1 (or layer-2)
# activation sits exactly on, just off, or far from such a decision; every other activation is 0.
def _one_unit_net(w1=0.0, b1=0.0, w2=0.0, b2=0.0):
    P = np.zeros(9729)
    P[0] = w1           # W1[0][0]
    P[1280] = b1        # b1[0]
    P[1344] = w2        # W2[0][0]
    P[5440] = b2        # b2[0]
    P[9664] = 1.0       # W4[0]: y depends on unit 0 of layer 3
    P[5504] = 1.0       # W3[0][0]
    return P


def _flag(O, P, x0, prec):
    x = np.zeros((1, 20))
    x[0, 0] = x0
    _, _, near = O.mlp_forward_quant(P, x, prec, with_fragile=True)
    return bool(near[0])


def test_bf16_flag_on_off_and_far_from_a_midpoint(O):
    # layer 1: out = 1 * 1 + b; BF16 spacing in [1, 2) is 2^-7, so 1 + 2^-8 is a midpoint
    ulp = 2.0 ** -7
    assert _flag(O, _one_unit_net(w1=1.0, b1=0.5 * ulp), 1.0, 1)                 # on the midpoint
    assert _flag(O, _one_unit_net(w1=1.0, b1=0.5 * ulp + 1e-4 * ulp), 1.0, 1)    # 1e-4 grid steps off
    assert not _flag(O, _one_unit_net(w1=1.0, b1=0.5 * ulp + 1e-3 * ulp), 1.0, 1)  # 1e-3 steps off
    assert not _flag(O, _one_unit_net(w1=1.0, b1=0.25 * ulp), 1.0, 1)           # far
    assert not _flag(O, _one_unit_net(w1=1.0, b1=0.0), 1.0, 1)                  # on the grid
    # layer 2: layer 1 gives exactly 1, layer 2 out = 1 + b2 with the same construction
    assert _flag(O, _one_unit_net(w1=1.0, w2=1.0, b2=0.5 * ulp), 1.0, 1)
    assert not _flag(O, _one_unit_net(w1=1.0, w2=1.0, b2=0.3 * ulp), 1.0, 1)
    # a negative pre-activation is clamped by ReLU to 0: nothing to round
    assert not _flag(O, _one_unit_net(w1=-1.0, b1=0.5 * ulp - 2.0), 1.0, 1)


def test_fp8_flag_on_off_and_far_from_a_midpoint(O):
    # W1[0][0] = 448 * 2^-9 gives the layer scale 2^-9 exactly (code 448); x0 = 1 is code 256 at
    # block scale 2^-8, so layer-1 out = 0.875 + b exactly.  out = 272 * 2^-9 lies in [256, 448]
    # of its block scale 2^-9, on the midpoint of 256 and 288
    w1 = 448.0 * 2.0 ** -9
    unit = 2.0 ** -9
    assert _flag(O, _one_unit_net(w1=w1, b1=272 * unit - w1), 1.0, 2)            # on the midpoint
    assert not _flag(O, _one_unit_net(w1=w1, b1=273 * unit - w1), 1.0, 2)        # 1/32 of a step off
    assert not _flag(O, _one_unit_net(w1=w1, b1=264 * unit - w1), 1.0, 2)        # a quarter step off
    # the scale boundary: out = 448 * 2^-9 makes amax / 448 exactly 2^-9, where the vertex's
    # power-of-two scale switches
    assert _flag(O, _one_unit_net(w1=w1, b1=0.0), 1.0, 2)
    assert not _flag(O, _one_unit_net(w1=w1, b1=3 * unit), 1.0, 2)              # 0.7 % above it
    assert not _flag(O, _one_unit_net(w1=w1, b1=-40 * unit), 1.0, 2)            # 9 % below it


def test_fp8_dot_error_bound_closed_forms(O):
    # products that are multiples of 2^(floor(log2 max|p|) - 13) cost only the FP32 group-sum term
    e32 = 2.0 ** -24
    w = np.array([1.0, 1.0, 2.0])
    x = np.array([256.0, 8.0, 0.5])             # products 256, 8, 1; unit 2^-5
    assert O.fp8_dot_error_bound(w, x) == pytest.approx(16 * e32 * 265.0, rel=1e-15)
    # a product below the unit may vanish whole
    x2 = np.array([256.0, 2.0 ** -6, 0.0])
    assert O.fp8_dot_error_bound(w, x2) == pytest.approx(2.0 ** -6 + 16 * e32 * (256 + 2.0 ** -6), rel=1e-15)
    # a product above the unit that is not a multiple of it loses at most one unit
    x3 = np.array([256.0, 1.0 + 2.0 ** -6, 0.0])
    assert O.fp8_dot_error_bound(w, x3) == pytest.approx(2.0 ** -5 + 16 * e32 * (257 + 2.0 ** -6), rel=1e-15)
    # scale invariance (powers of two) and the empty / all-zero dot product
    assert O.fp8_dot_error_bound(w, 4 * x3) == pytest.approx(4 * O.fp8_dot_error_bound(w, x3), rel=1e-15)
    assert O.fp8_dot_error_bound(w, np.zeros(3)) == 0.0
    # signs do not matter
    assert O.fp8_dot_error_bound(-w, x3) == O.fp8_dot_error_bound(w, x3)


def test_relu_decision_within_the_float32_error_of_zero_is_a_near_tie(O):
    # layer 1: pre = 1 * 1 + b1.  The float32 sum of the product and the bias may land on either
    # side of 0 when the exact value lies within the summation bound (21 terms' gamma of the
    # magnitudes, ~2.5e-6 here); an exact 0 from all-zero terms is no tie
    assert _flag(O, _one_unit_net(w1=1.0, b1=-1.0), 1.0, 1)                 # exactly 0
    assert _flag(O, _one_unit_net(w1=1.0, b1=-1.0 - 1e-7), 1.0, 1)         # just below
    assert _flag(O, _one_unit_net(w1=1.0, b1=-1.0 + 1e-7), 1.0, 1)         # just above
    assert not _flag(O, _one_unit_net(w1=1.0, b1=-1.0 - 1e-4), 1.0, 1)     # clearly negative
    assert not _flag(O, _one_unit_net(w1=1.0, b1=-1.0 + 2.0 ** -10), 1.0, 1)  # clearly positive, on the grid
    # the flag is per activation: the codes call marks unit 0 of layer 1 (index 64 + 0) only
    P = _one_unit_net(w1=1.0, b1=-1.0)
    x = np.zeros((1, 20))
    x[0, 0] = 1.0
    _, _, near, codes, near_act, _ = O.mlp_forward_quant_codes(P, x, 1)
    assert near[0] and near_act[0, 1, 0] and near_act[0, 1, 1:].sum() == 0 and near_act[0, 0].sum() == 0
    # FP8: the same decision against the FP8 dot-product bound (layer-1 out = 0.875 + b1 exactly,
    # as in the midpoint test above)
    w1 = 448.0 * 2.0 ** -9
    assert _flag(O, _one_unit_net(w1=w1, b1=-0.875), 1.0, 2)                # exactly 0
    assert not _flag(O, _one_unit_net(w1=w1, b1=-0.885), 1.0, 2)            # 0.01 below: far


def test_e4m3_code_of_a_negative_value_rounded_to_zero_keeps_the_sign(O):
    # x0 = 1 sets the input block scale 2^-8; x1 = -2^-20 scales to -2^-12, below half the
    # smallest subnormal (2^-10): it rounds to zero and keeps its sign (code 0x80); +0 is 0x00
    P = _one_unit_net(w1=1.0)
    x = np.zeros((1, 20))
    x[0, 0] = 1.0
    x[0, 1] = -(2.0 ** -20)
    _, _, _, codes, _, se = O.mlp_forward_quant_codes(P, x, 2)
    assert se[0, 0] == -8
    assert codes[0, 0, 1] == 0x80 and codes[0, 0, 2] == 0x00
    assert codes[0, 0, 0] == 0x78  # 1 / 2^-8 = 256 = 1.0 x 2^8: exponent 8 + 7 = 15, mantissa 0


def test_bf16_activation_flag_takes_the_float32_summation_bound_where_terms_cancel(O):
    # layer-1 unit 0: 1024 * 1 + (-1016) * 1 + b = 8 + b; the BF16 spacing at 8 is 1/16, so 8 + 1/32
    # is a midpoint.  The float32 sum of products of magnitude ~2040 may be off by up to
    # 21 * 2^-24 * 2040 ~ 2.6e-3 = 0.04 grid steps: 0.01 steps from the midpoint is a near-tie for
    # the exact code-by-code comparison (activation flag) but not for the row flag (2e-4 steps)
    P = np.zeros(9729)
    P[0], P[1] = 1.0, 1.0     # W1[0][0], W1[0][1]
    P[9664], P[5504] = 1.0, 1.0
    x = np.zeros((1, 20))
    x[0, 0], x[0, 1] = 1024.0, -1016.0
    step = 1.0 / 16
    for off, act, row in ((0.01, True, False), (0.1, False, False), (1e-4, True, True)):
        P[1280] = step / 2 + off * step  # b1[0]
        _, _, near, _, near_act, _ = O.mlp_forward_quant_codes(P, x, 1)
        assert bool(near_act[0, 1, 0]) == act, off
        assert bool(near[0]) == row, off
