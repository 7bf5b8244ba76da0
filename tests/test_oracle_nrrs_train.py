"""Pins of the oracle of NRRS training proper (oracle/nrrs_train.c) against what the paper and
the mathematics fix: closed forms of the encodings (Sec. 5 "Input Encoding"), finite
differences of the forward passes for every backward pass, the exact variance of RR and
splitting estimators enumerated outcome by outcome for the gradient transfer (Eqs. 4-7,
17-18), and finite differences of the pixel losses (Eqs. 19-20)."""
import itertools

import numpy as np
import pytest

from oracle import nrrs_train as N

LOG2T = 14  # level 0 (17^3 corners) dense, levels >= 1 hashed


# ---------------------------------------------------------------------- one-blob
def test_oneblob_peaks_at_its_bin_and_falls_by_a_gaussian_of_one_bin_width():
    for bins in (4, 8):
        for i in range(bins):
            e = N.oneblob((i + 0.5) / bins, bins)
            assert e[i] == pytest.approx(1.0)
            for j in range(bins):
                # one bin apart = one sigma: exp(-1/2); two bins: exp(-2)
                assert e[j] == pytest.approx(np.exp(-0.5 * (i - j) ** 2), rel=1e-12)
    # clamped outside [0, 1]
    assert np.array_equal(N.oneblob(-3.0, 4), N.oneblob(0.0, 4))
    assert np.array_equal(N.oneblob(7.0, 8), N.oneblob(1.0, 8))


# --------------------------------------------------------------------- hash grid
def _table(rng):
    return rng.normal(0, 1, size=N.HG_LEVELS * (1 << LOG2T) * N.HG_FEAT)


def test_hashgrid_weights_are_a_partition_of_unity():
    t = np.full(N.HG_LEVELS * (1 << LOG2T) * N.HG_FEAT, 2.5)
    p = np.random.default_rng(0).uniform(0, 1, size=(50, 3))
    assert np.allclose(N.hashgrid_encode(t, LOG2T, p), 2.5, rtol=0, atol=1e-13)


def test_hashgrid_dense_level_reproduces_a_linear_field_exactly():
    # trilinear interpolation of a linear function of the corner coordinates is that function
    R, side = N.HG_BASE, N.HG_BASE + 1
    t = np.zeros(N.HG_LEVELS * (1 << LOG2T) * N.HG_FEAT)
    for z, y, x in itertools.product(range(side), repeat=3):
        idx = x + side * (y + side * z)
        t[idx * 2 + 0] = 0.3 * x - 1.1 * y + 0.7 * z + 0.25
        t[idx * 2 + 1] = -0.2 * x + 0.05 * z
    p = np.random.default_rng(1).uniform(0, 1, size=(200, 3))
    p[0] = [1.0, 1.0, 1.0]  # upper boundary: the last cell, fraction 1
    p[1] = [0.0, 0.5, 1.0]
    enc = N.hashgrid_encode(t, LOG2T, p)
    u = p * R
    assert np.allclose(enc[:, 0], 0.3 * u[:, 0] - 1.1 * u[:, 1] + 0.7 * u[:, 2] + 0.25, atol=1e-12)
    assert np.allclose(enc[:, 1], -0.2 * u[:, 0] + 0.05 * u[:, 2], atol=1e-12)


def test_hashgrid_level_is_dense_exactly_when_its_corners_fit_the_table():
    # with T = 2^16, level 1 (R = 32: 33^3 = 35,937 corners) is stored densely; with T = 2^15
    # it is hashed, so the same dense linear field no longer interpolates to itself
    R, side = N.HG_BASE * 2, N.HG_BASE * 2 + 1
    p = np.random.default_rng(13).uniform(0, 1, size=(100, 3))
    for log2T, dense in ((16, True), (15, False)):
        T = 1 << log2T
        t = np.zeros(N.HG_LEVELS * T * N.HG_FEAT)
        for z, y, x in itertools.product(range(side), repeat=3):
            idx = x + side * (y + side * z)
            if idx < T:
                t[(T + idx) * 2] = 0.5 * x + 0.25 * y - 0.125 * z
        enc = N.hashgrid_encode(t, log2T, p)
        u = p * R
        match = np.allclose(enc[:, 2], 0.5 * u[:, 0] + 0.25 * u[:, 1] - 0.125 * u[:, 2], atol=1e-12)
        assert match == dense


def _tent(u, c):
    return np.maximum(0.0, 1.0 - np.abs(u - c))


def test_hashgrid_hashed_level_reads_the_spatial_hash_slot_with_the_tent_weight():
    # one corner of level 2 (R = 64) holds a feature 1: the encoding is that corner's trilinear
    # (tent) weight, read at the slot (x ^ y * 2654435761 ^ z * 805459861) mod 2^LOG2T
    l, R = 2, N.HG_BASE << 2
    c = (17, 40, 3)
    slot = (c[0] ^ ((c[1] * 2654435761) & 0xFFFFFFFF) ^ ((c[2] * 805459861) & 0xFFFFFFFF)) % (1 << LOG2T)
    t = np.zeros(N.HG_LEVELS * (1 << LOG2T) * N.HG_FEAT)
    t[(l * (1 << LOG2T) + slot) * 2 + 1] = 1.0
    rng = np.random.default_rng(2)
    p = (np.array(c)[None, :] + rng.uniform(-1, 1, size=(100, 3))) / R
    enc = N.hashgrid_encode(t, LOG2T, p)
    u = p * R
    w = _tent(u[:, 0], c[0]) * _tent(u[:, 1], c[1]) * _tent(u[:, 2], c[2])
    assert np.allclose(enc[:, 2 * l + 1], w, atol=1e-12)
    assert np.all(enc[:, 2 * l] == 0.0)


def test_hashgrid_backward_is_the_derivative_of_the_encoding():
    rng = np.random.default_rng(3)
    t = _table(rng)
    p = rng.uniform(0, 1, size=(3, 3))
    dout = rng.normal(0, 1, size=(3, 16))
    dt = N.hashgrid_backward(LOG2T, p, dout)
    # the encoding is linear in the table: its derivative along any direction d is enc(d)
    for _ in range(3):
        d = rng.normal(0, 1, size=t.shape)
        assert np.sum(dt * d) == pytest.approx(np.sum(N.hashgrid_encode(d, LOG2T, p) * dout), rel=1e-10)


# ------------------------------------------------------------------ 32-wide MLP
def test_mlp32_parameter_count_and_closed_form_with_identity_layers():
    assert N.mlp32_nparams(32, 2) == 32 * 32 + 32 + 2 * (32 * 32 + 32) + 2 * 32 + 2
    assert N.mlp32_nparams(7, 1) == 7 * 32 + 32 + 2 * (32 * 32 + 32) + 32 + 1
    # hidden layers = identity, zero biases: positive inputs pass through, negative ones are
    # scaled by the leaky slope 0.01 once per hidden layer
    P = np.zeros(N.mlp32_nparams(32, 2))
    o = 0
    for _ in range(3):
        P[o:o + 1024] = np.eye(32).ravel()
        o += 1024 + 32
    W4 = np.random.default_rng(4).normal(0, 1, size=(2, 32))
    P[o:o + 64] = W4.ravel()
    P[o + 64:o + 66] = [0.5, -0.25]
    x = np.random.default_rng(5).normal(0, 1, size=32)
    h = np.where(x > 0, x, 1e-6 * x)
    assert np.allclose(N.mlp32_forward(P, 32, 2, x)[0], W4 @ h + [0.5, -0.25], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("n_in,n_out", [(32, 2), (7, 1)])
def test_mlp32_backward_matches_finite_differences(n_in, n_out):
    rng = np.random.default_rng(6 + n_in)
    P = rng.normal(0, 0.3, size=N.mlp32_nparams(n_in, n_out))
    x = rng.normal(0, 1, size=(3, n_in))
    dy = rng.normal(0, 1, size=(3, n_out))
    dP, dx = N.mlp32_backward(P, n_in, n_out, x, dy)
    f = lambda PP, xx: float(np.sum(N.mlp32_forward(PP, n_in, n_out, xx) * dy))
    h = 1e-6
    for k in rng.choice(P.size, 40, replace=False):
        e = np.zeros_like(P)
        e[k] = h
        assert dP[k] == pytest.approx((f(P + e, x) - f(P - e, x)) / (2 * h), rel=1e-5, abs=1e-8)
    for r, i in [(0, 0), (1, n_in - 1), (2, n_in // 2)]:
        e = np.zeros_like(x)
        e[r, i] = h
        assert dx[r, i] == pytest.approx((f(P, x + e) - f(P, x - e)) / (2 * h), rel=1e-5, abs=1e-8)


# ------------------------------------------------------------------------ StatNet
def _raw(rng, n):
    w = rng.normal(0, 1, size=(n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    return np.concatenate([rng.uniform(0, 1, size=(n, 3)), w, rng.uniform(0, 1, size=(n, 1))], 1)


def test_statnet_encoding_layout():
    rng = np.random.default_rng(7)
    t = _table(rng)
    raw = _raw(rng, 5)
    enc = N.statnet_encode(t, LOG2T, raw)
    assert np.allclose(enc[:, :16], N.hashgrid_encode(t, LOG2T, raw[:, :3]))
    for r in range(5):
        theta = np.arccos(raw[r, 5])
        phi = np.arctan2(raw[r, 4], raw[r, 3])
        assert np.allclose(enc[r, 16:20], N.oneblob(theta / np.pi, 4))
        assert np.allclose(enc[r, 20:24], N.oneblob(phi / (2 * np.pi) + 0.5, 4))
        assert np.allclose(enc[r, 24:32], N.oneblob(raw[r, 6], 8))
    # +z is theta = 0: the first polar bin is the largest
    up = np.array([[0.3, 0.3, 0.3, 0.0, 0.0, 1.0, 0.5]])
    e = N.statnet_encode(t, LOG2T, up)[0]
    assert np.argmax(e[16:20]) == 0


def test_statnet_gradient_is_the_derivative_with_stop_gradients():
    # Eq. (15) with sg(): the gradient equals the finite difference of the loss whose
    # denominators and variance target are frozen at the current prediction
    rng = np.random.default_rng(8)
    t = _table(rng) * 0.1
    Ps = rng.normal(0, 0.3, size=N.mlp32_nparams(32, 2))
    raw = _raw(rng, 6)
    L = rng.lognormal(-1, 1, size=6)
    eps = 0.01
    loss, dP, dT = N.statnet_loss_grad(Ps, t, LOG2T, raw, L, eps)
    mv0 = N.statnet_forward(Ps, t, LOG2T, raw)
    v1 = (L - mv0[:, 0]) ** 2

    def frozen(PP, tt):
        mv = N.statnet_forward(PP, tt, LOG2T, raw)
        return float(np.mean((mv[:, 0] - L) ** 2 / (L ** 2 + eps) + (mv[:, 1] - v1) ** 2 / (v1 ** 2 + eps)))

    assert loss == pytest.approx(frozen(Ps, t), rel=1e-12)
    h = 1e-6
    for k in rng.choice(Ps.size, 25, replace=False):
        e = np.zeros_like(Ps)
        e[k] = h
        assert dP[k] == pytest.approx((frozen(Ps + e, t) - frozen(Ps - e, t)) / (2 * h), rel=1e-5, abs=1e-9)
    for k in np.flatnonzero(dT)[:: max(1, np.count_nonzero(dT) // 20)]:
        e = np.zeros_like(t)
        e[k] = h
        assert dT[k] == pytest.approx((frozen(Ps, t + e) - frozen(Ps, t - e)) / (2 * h), rel=1e-5, abs=1e-9)


# ---------------------------------------------------------------- RRSNet inputs
def test_rrs_inputs_box_cox_and_second_moment():
    x = N.rrs_inputs([[0.25, 0.5]], [[1.0, 4.0, 0.0]], 9.0, 0.3)[0]
    # Box-Cox lambda = 1/2: 2 (sqrt(x) - 1); E[L^2] = v + m^2
    assert np.allclose(x, [2 * (0.5 - 1), 2 * (np.sqrt(0.5625) - 1), 0.0, 2.0, -2.0, 4.0, 0.3])
    # negative StatNet outputs count as zero
    x = N.rrs_inputs([[-1.0, -2.0]], [[1.0, 1.0, 1.0]], 1.0, 0.0)[0]
    assert x[0] == -2.0 and x[1] == -2.0


# ------------------------------------------------------------- gradient transfer
H_VALS = np.array([0.0, 0.5, 2.0, 5.0])
H_PROB = np.array([0.4, 0.3, 0.2, 0.1])


def _exact_var_rr(g, q):
    # Y = g B H / q, B ~ Bernoulli(q): enumerate (B, H)
    vals, probs = [], []
    for b, pb in ((1, q), (0, 1 - q)):
        for h, ph in zip(H_VALS, H_PROB):
            vals.append(g * b * h / q)
            probs.append(pb * ph)
    vals, probs = np.array(vals), np.array(probs)
    mean = np.sum(vals * probs)
    return np.sum(probs * (vals - mean) ** 2)


def _exact_var_split(g, n):
    # Y = g (1/n) sum of n independent H: enumerate every tuple
    vals, probs = [], []
    for tup in itertools.product(range(len(H_VALS)), repeat=n):
        vals.append(g * np.mean(H_VALS[list(tup)]))
        probs.append(np.prod(H_PROB[list(tup)]))
    vals, probs = np.array(vals), np.array(probs)
    mean = np.sum(vals * probs)
    return np.sum(probs * (vals - mean) ** 2)


def test_gradient_transfer_rr_is_the_derivative_of_the_exact_rr_variance():
    mu, m2 = np.sum(H_PROB * H_VALS), np.sum(H_PROB * H_VALS ** 2)
    var = m2 - mu ** 2
    g = 0.7
    for q in (0.2, 0.5, 0.9):
        h = 1e-5
        fd = (_exact_var_rr(g, q + h) - _exact_var_rr(g, q - h)) / (2 * h)
        d = N.nrrs_dloss_dq(1.0, 1, g, [mu, var], q, 1.0, q, 0.0)
        assert d == pytest.approx(fd, rel=1e-6)


def test_gradient_transfer_splitting_is_the_derivative_of_the_exact_split_variance():
    mu, m2 = np.sum(H_PROB * H_VALS), np.sum(H_PROB * H_VALS ** 2)
    var = m2 - mu ** 2
    g = 1.3
    # the enumerated variance at integer n is g^2 Var[H] / n (Eq. 4) ...
    for n in (1, 2, 3):
        assert _exact_var_split(g, n) == pytest.approx(g * g * var / n, rel=1e-12)
    # ... whose derivative in n is the transfer's splitting estimate
    for n in (1.0, 2.0, 3.5):
        h = 1e-5
        fd = (g * g * var / (n + h) - g * g * var / (n - h)) / (2 * h)
        assert N.nrrs_dloss_dq(1.0, 1, g, [mu, var], n, 1.0, n, 0.0) == pytest.approx(fd, rel=1e-8)


def test_gradient_transfer_scales_by_F_shares_by_k_and_adds_the_bound_loss():
    mv = [0.8, 0.3]
    base = N.nrrs_dloss_dq(1.0, 1, 0.5, mv, 0.6, 1.0, 0.6, 0.0)
    # q_norm = F q_nrrs: the chain rule multiplies by F; the pixel loss is shared by k samples
    assert N.nrrs_dloss_dq(2.0, 4, 0.5, mv, 0.6, 1.7, 0.6 / 1.7, 0.0) == pytest.approx(base * 2.0 / 4 * 1.7)
    # L_rrs = g3 (q_nrrs - sg(q_norm))^2 adds its derivative in q_nrrs
    g3, qn, qr = 0.01, 0.6, 0.45
    h = 1e-6
    fd = (g3 * (qr + h - qn) ** 2 - g3 * (qr - h - qn) ** 2) / (2 * h)
    assert N.nrrs_dloss_dq(0.0, 1, 0.5, mv, qn, 1.0, qr, g3) == pytest.approx(fd, rel=1e-8)
    # no sample of the pixel: no pixel term
    assert N.nrrs_dloss_dq(5.0, 0, 0.5, mv, qn, 1.0, qr, 0.0) == 0.0


# ------------------------------------------------------------------- pixel error
def test_pixel_weights_are_the_derivative_of_the_pixel_losses():
    rng = np.random.default_rng(9)
    w, h = 7, 5
    ref = rng.lognormal(-1, 1, size=w * h)
    cur = ref + rng.normal(0, 0.3, size=w * h)
    g_avg, g_min, eps = 0.01, 0.05, 0.01
    Eavg, E, wpx, acc = N.pixel_weights(cur, np.zeros(w * h), ref, w, h, True, radius=0, var_scale=1.0,
                                        g_avg=g_avg, g_min=g_min, eps=eps)
    var = (cur - ref) ** 2
    assert np.allclose(acc, cur)
    assert np.allclose(E, var / (ref ** 2 + eps))
    assert Eavg == pytest.approx(E.mean())

    def loss(vv):  # Eqs. (19)-(20) as functions of the pixel variances
        Ei = vv / (ref ** 2 + eps)
        return g_avg * np.sum((Ei - Ei.mean()) ** 2) + g_min * np.sum(Ei)

    for i in range(w * h):
        e = np.zeros(w * h)
        e[i] = 1e-3  # the losses are quadratic in the variances: central differences are exact
        fd = (loss(var + e) - loss(var - e)) / (2 * e[i])
        assert wpx[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_pixel_error_temporal_mix_box_filter_and_missing_reference():
    w, h = 6, 4
    ref = np.ones(w * h)
    # temporal mix (Eq. 23): acc = (1 - a) acc + a cur
    _, _, _, acc = N.pixel_weights(np.full(w * h, 3.0), np.full(w * h, 1.0), ref, w, h, False, a_mix=0.25, radius=0)
    assert np.allclose(acc, 0.75 * 1.0 + 0.25 * 3.0)
    # a single error impulse spreads over the clipped (2r + 1)^2 window, averaged over it
    cur = np.ones(w * h)
    cur[0] = 1.0 + np.sqrt(1.01)  # E' = 1 at pixel (0, 0)
    _, E, _, _ = N.pixel_weights(cur, np.zeros(w * h), ref, w, h, True, radius=1, eps=0.01)
    Eimg = E.reshape(h, w)
    assert Eimg[0, 0] == pytest.approx(1 / 4) and Eimg[1, 1] == pytest.approx(1 / 9)
    assert Eimg[0, 1] == pytest.approx(1 / 6) and Eimg[2, 2] == 0.0
    # pixels without a reference (ref < 0) get no error and no weight and leave E_avg alone
    ref2 = ref.copy()
    ref2[5] = -1.0
    Eavg, E, wpx, _ = N.pixel_weights(np.ones(w * h) * 1.5, np.zeros(w * h), ref2, w, h, True, radius=0)
    assert E[5] == 0.0 and wpx[5] == 0.0
    assert Eavg == pytest.approx(0.25 / 1.01)


# ------------------------------------------------------------- RRSNet gradient
def _records(rng, n, npx):
    return dict(raw=_raw(rng, n), t_rgb=rng.uniform(0.05, 1.0, size=(n, 3)), I_px=rng.lognormal(-1, 0.5, size=n),
                lum_t=rng.uniform(0.05, 1.0, size=n), q_norm=rng.uniform(0.2, 2.5, size=n),
                F=rng.uniform(0.5, 1.5, size=n), pix=rng.integers(0, npx, size=n).astype(np.uint32))


def test_rrsnet_step1_gradient_matches_finite_differences():
    rng = np.random.default_rng(10)
    t = _table(rng) * 0.1
    Ps = rng.normal(0, 0.3, size=N.mlp32_nparams(32, 2))
    Pr = rng.normal(0, 0.3, size=N.mlp32_nparams(7, 1))
    R = _records(rng, 5, 4)
    k = np.bincount(R["pix"], minlength=4).astype(np.uint32)
    wpx = np.zeros(4)
    loss, dPr = N.rrsnet_nrrs_grad(Pr, Ps, t, LOG2T, step=1, k_pix=k, wpx=wpx, **R)

    def f(PP):
        q, _, _ = N.nrrs_factor(Ps, PP, t, LOG2T, R["raw"], R["t_rgb"], R["I_px"])
        return float(np.mean((q - 1.0) ** 2 / 1.01))

    assert loss == pytest.approx(f(Pr), rel=1e-12)
    h = 1e-6
    for j in rng.choice(Pr.size, 30, replace=False):
        e = np.zeros_like(Pr)
        e[j] = h
        assert dPr[j] == pytest.approx((f(Pr + e) - f(Pr - e)) / (2 * h), rel=1e-5, abs=1e-9)


def test_rrsnet_step2_gradient_is_the_transferred_pixel_gradient_plus_the_bound_loss():
    rng = np.random.default_rng(11)
    t = _table(rng) * 0.1
    Ps = rng.normal(0, 0.3, size=N.mlp32_nparams(32, 2))
    Pr = rng.normal(0, 0.3, size=N.mlp32_nparams(7, 1))
    R = _records(rng, 6, 3)
    k = np.bincount(R["pix"], minlength=3).astype(np.uint32)
    wpx = np.array([0.7, -0.2, 1.5])
    g3 = 0.01
    _, dPr = N.rrsnet_nrrs_grad(Pr, Ps, t, LOG2T, step=2, k_pix=k, wpx=wpx, g_rrs=g3, **R)
    mv = N.statnet_forward(Ps, t, LOG2T, R["raw"])
    # the transferred part, held fixed: (w / k) F dVar/dq_norm per sample
    m = np.maximum(mv[:, 0], 0)
    v = np.maximum(mv[:, 1], 0)
    S = np.where(R["q_norm"] < 1, v + m * m, v)
    A = wpx[R["pix"]] / k[R["pix"]] * R["F"] * (-(R["lum_t"] ** 2) * S / R["q_norm"] ** 2)

    def G(PP):
        q, _, _ = N.nrrs_factor(Ps, PP, t, LOG2T, R["raw"], R["t_rgb"], R["I_px"])
        return float(np.sum(A * q + g3 * (q - R["q_norm"]) ** 2))

    h = 1e-6
    for j in rng.choice(Pr.size, 30, replace=False):
        e = np.zeros_like(Pr)
        e[j] = h
        assert dPr[j] == pytest.approx((G(Pr + e) - G(Pr - e)) / (2 * h), rel=1e-5, abs=1e-9)


def test_nrrs_factor_is_statnet_then_rrsnet_with_the_modified_softplus():
    rng = np.random.default_rng(12)
    t = _table(rng) * 0.1
    Ps = rng.normal(0, 0.3, size=N.mlp32_nparams(32, 2))
    Pr = rng.normal(0, 0.3, size=N.mlp32_nparams(7, 1))
    raw = _raw(rng, 4)
    tr = rng.uniform(0.1, 1, size=(4, 3))
    I = rng.uniform(0.1, 1, size=4)
    q, mv, z = N.nrrs_factor(Ps, Pr, t, LOG2T, raw, tr, I)
    assert np.allclose(mv, N.statnet_forward(Ps, t, LOG2T, raw))
    x = N.rrs_inputs(mv, tr, I, raw[:, 6])
    assert np.allclose(z, N.mlp32_forward(Pr, 7, 1, x)[:, 0])
    # Eq. (22): ln(1 + e^z) below 0, z / 2 + ln 2 above; continuous at 0
    assert np.allclose(q, np.where(z < 0, np.log1p(np.exp(np.minimum(z, 0))), 0.5 * z + np.log(2)))


# ------------------------------------------------------------- AID-NRRS RRSNet
def test_aid_encoding_layout():
    rng = np.random.default_rng(14)
    t = _table(rng)
    raw = _raw(rng, 4)
    tr = rng.uniform(0.1, 1, size=(4, 3))
    I = rng.uniform(0.1, 2, size=4)
    enc = N.aid_encode(t, LOG2T, raw, tr, I)
    assert np.allclose(enc[:, :16], N.hashgrid_encode(t, LOG2T, raw[:, :3]))
    for r in range(4):
        assert np.allclose(enc[r, 16:20], N.oneblob(np.arccos(raw[r, 5]) / np.pi, 4))
        assert np.allclose(enc[r, 20:24], N.oneblob(np.arctan2(raw[r, 4], raw[r, 3]) / (2 * np.pi) + 0.5, 4))
        assert np.allclose(enc[r, 24:27], 2 * (np.sqrt(tr[r]) - 1))
        assert enc[r, 27] == pytest.approx(2 * (np.sqrt(I[r]) - 1))
        assert np.allclose(enc[r, 28:32], N.oneblob(raw[r, 6], 4))


@pytest.mark.parametrize("step", [1, 2])
def test_aid_gradient_matches_finite_differences(step):
    # step 1: the derivative of the mean relative L2 to 1; step 2: the transferred pixel gradient
    # held fixed plus the bound loss, through the MLP and RRSNet's own hash grid
    rng = np.random.default_rng(15 + step)
    ts, tr = _table(rng) * 0.1, _table(rng) * 0.3
    Ps = rng.normal(0, 0.3, size=N.mlp32_nparams(32, 2))
    Pa = rng.normal(0, 0.2, size=N.mlp32_nparams(32, 1))
    R = _records(rng, 5, 3)
    k = np.bincount(R["pix"], minlength=3).astype(np.uint32)
    wpx = np.array([0.7, -0.2, 1.5])
    g3 = 0.01
    loss, dPa, dT = N.aid_grad(Pa, tr, Ps, ts, LOG2T, R["raw"], R["t_rgb"], R["I_px"], R["lum_t"], R["q_norm"], R["F"],
                               R["pix"], k, wpx, step, g_rrs=g3)
    mv = N.statnet_forward(Ps, ts, LOG2T, R["raw"])
    m, v = np.maximum(mv[:, 0], 0), np.maximum(mv[:, 1], 0)
    S = np.where(R["q_norm"] < 1, v + m * m, v)
    A = wpx[R["pix"]] / k[R["pix"]] * R["F"] * (-(R["lum_t"] ** 2) * S / R["q_norm"] ** 2)

    def G(PP, TT):
        q, _ = N.aid_factor(PP, TT, LOG2T, R["raw"], R["t_rgb"], R["I_px"])
        if step == 1:
            return float(np.mean((q - 1.0) ** 2 / 1.01))
        return float(np.sum(A * q + g3 * (q - R["q_norm"]) ** 2))

    h = 1e-6
    for j in rng.choice(Pa.size, 25, replace=False):
        e = np.zeros_like(Pa)
        e[j] = h
        assert dPa[j] == pytest.approx((G(Pa + e, tr) - G(Pa - e, tr)) / (2 * h), rel=1e-5, abs=1e-9)
    nz = np.flatnonzero(dT)
    assert nz.size > 0
    for j in nz[:: max(1, nz.size // 15)]:
        e = np.zeros_like(tr)
        e[j] = h
        assert dT[j] == pytest.approx((G(Pa, tr + e) - G(Pa, tr - e)) / (2 * h), rel=1e-5, abs=1e-9)
