"""Pins of the oracle's whole estimator: closed forms, exhaustive enumeration and
statistical unbiasedness of the normalized-RRS wavefront (Sec. 3 Eqs. 1-3 and 8,
Sec. 4.1 Eqs. 9-14)."""
import math

import numpy as np
import pytest


def furnace_value(D, a=float(np.float32(0.7)), le=1.0):
    """Depth-D truncated furnace: every vertex emits le and reflects a -> le (1 - a^D) / (1 - a)."""
    return le * (1.0 - a ** D) / (1.0 - a)


@pytest.mark.parametrize("D", [1, 2, 8, 64])
def test_white_furnace_closed_form(O, scenes, D):
    sc = O.OracleScene(scenes.furnace())
    cfg = O.make_cfg(16, 16, 2, D, mode=O.MODE_HEUR, n_passes=2)
    r = O.render(sc, cfg)
    img = r["image"].reshape(-1, 3) / 4.0
    assert np.all(r["n"][1:] == 16 * 16 * 2 * 2)     # no path escaped the closed box
    assert np.allclose(img, furnace_value(D), rtol=1e-12, atol=0)
    # zero variance case: every factor normalises to exactly 1, no split, no kill
    assert np.all(r["S"][1:D] == r["n"][1:D]) and np.all(r["retries"] == 0)


def test_furnace_records_target_closed_form(O, scenes):
    # the record at vertex depth d collects the descendants' emission: a (1 - a^(D-d)) / (1 - a)
    sc = O.OracleScene(scenes.furnace())
    D = 8
    cfg = O.make_cfg(8, 8, 1, D, mode=O.MODE_HEUR, p_train=1.0, rec_cap=4096)
    r = O.render(sc, cfg, records=True)
    rec = r["records"]
    a = float(np.float32(0.7))
    assert r["n_records"] == 64 * 4
    target = rec["acc"] / rec["lum_t"]
    d = rec["depth"].astype(np.float64)
    expect = a * (1 - a ** (D - d)) / (1 - a)
    assert np.allclose(target, expect, rtol=1e-12)
    # closed-form feature entries at a grey Lambertian furnace vertex
    f = rec["feat"]
    t = a ** (d - 1)
    assert np.allclose(f[:, 9], 2 * (np.sqrt(t) - 1), rtol=1e-12)      # Box-Cox lambda 0.5
    assert np.allclose(f[:, 12:15], a)                                # albedo
    assert np.allclose(f[:, 15], 1 - math.exp(-1.0))                  # roughness remap, alpha := 1
    assert np.allclose(f[:, 16], d / D)
    assert np.allclose(np.linalg.norm(f[:, 3:6], axis=1), 1.0)         # unit normal
    assert np.allclose(np.linalg.norm(f[:, 6:9], axis=1), 1.0)         # unit outgoing direction
    assert np.all(np.abs(f[:, 0:3]) <= 1.0 + 1e-12)
    # the normal faces the outgoing direction
    assert np.all(np.einsum("ij,ij->i", f[:, 3:6], f[:, 6:9]) > 0)


def test_exhaustive_enumeration_matches_plain_path_tracing(O, scenes):
    # With every child reusing one continuous sample, the outcome-weighted mean over all
    # roulette outcomes equals the no-RRS estimate on the same samples (E[X/q] = 1, Eq. 8),
    # also through the per-depth normalization (Eqs. 9-10) that couples the paths.
    sc = O.OracleScene(scenes.two_triangle())
    total = 0
    for seed in range(8):
        cfg = O.make_cfg(2, 2, 1, 4, mode=O.MODE_HEUR, cap_factor=2.0, seed=seed)
        ie, io, max_s, branches = O.enumerate_expectation(sc, cfg)
        total += branches
        assert max_s <= 8          # capacity 2 x 4 primary paths
        assert np.abs(io).sum() > 0
        assert np.allclose(ie, io, rtol=1e-12, atol=1e-14)
    assert total > 1000


def _poisson_binomial(r):
    # pmf of a sum of independent Bernoulli(r_i) by convolution, one variable at a time
    pmf = np.array([1.0])
    for ri in r:
        pmf = np.concatenate([pmf * (1.0 - ri), [0.0]]) + np.concatenate([[0.0], pmf * ri])
    return pmf


def test_enumerated_children_count_is_poisson_binomial(O, scenes):
    # Sec. 4.1.3: given the normalized factors, the children count S = sum_i X_i is the integer
    # part sum_i floor(q_i) plus a Poisson-binomial count over the fractional parts, with mean
    # sum_i q_i = B (Eq. 10) at every depth.  The enumerator's outcome probabilities must give
    # exactly that law at depth 1 (one branch) and the mean B on every branch deeper down.
    sc = O.OracleScene(scenes.two_triangle())
    for seed in range(6):
        cfg = O.make_cfg(2, 2, 1, 4, mode=O.MODE_HEUR, cap_factor=2.0, seed=seed)
        _, _, max_s, _, pmf, live, qn1 = O.enumerate_expectation(sc, cfg, with_pmf=True)
        N = 4
        cap = 8
        assert max_s <= cap and np.all(pmf[:, cap + 1] == 0.0)
        assert live[1] == 1.0
        q = qn1.astype(np.float64)
        k = np.floor(q)
        r = q - k
        expect = np.zeros(cap + 2)
        pb = _poisson_binomial(r)
        base = int(k.sum())
        expect[base:base + pb.size] = pb
        assert np.allclose(pmf[1], expect, rtol=0, atol=1e-13)
        assert abs(q.sum() - N) < 1e-5                               # sum of q_norm = B = N
        var = float((r * (1 - r)).sum())
        mean1 = float((np.arange(cap + 2) * pmf[1]).sum())
        assert abs(float(((np.arange(cap + 2) - mean1) ** 2 * pmf[1]).sum()) - var) < 1e-12
        assert var <= N / 4 + 1e-12                                      # Var(S | q) <= |I| / 4
        for d in range(1, cfg.max_depth):
            mass = pmf[d].sum()
            assert abs(mass - live[d]) < 1e-12
            if live[d] > 0:
                mean = float((np.arange(cap + 2) * pmf[d]).sum()) / live[d]
                assert abs(mean - N) < 1e-5, (d, mean)


def _chunk_means(O, sc, mode, chunks, per_chunk, seed, D=8, W=8, H=8, params=None, guide=None):
    means = []
    for c in range(chunks):
        cfg = O.make_cfg(W, H, 1, D, mode=mode, pass_begin=c * per_chunk, n_passes=per_chunk, seed=seed, tau=0.0)
        r = O.render(sc, cfg, params=params, guide=guide)
        img = r["image"].reshape(-1, 3)
        means.append(float((img @ np.array([0.2126, 0.7152, 0.0722])).mean()) / per_chunk)
    return np.array(means)


def test_normalized_rrs_is_unbiased_cornell(O, scenes):
    # Mean image luminance of an 8x8 Cornell render: normalized heuristic RRS vs plain PT
    sc = O.OracleScene(scenes.cornell(), bvh=False)
    h = _chunk_means(O, sc, O.MODE_HEUR, 60, 100, seed=1)
    p = _chunk_means(O, sc, O.MODE_OFF, 60, 100, seed=2)
    se = math.sqrt(h.var(ddof=1) / h.size + p.var(ddof=1) / p.size)
    assert abs(h.mean() - p.mean()) < 3.5 * se
    assert se < 0.02 * p.mean()


def test_normalized_rrs_is_unbiased_cornell_200k_realizations(O, scenes):
    # 204,800 realizations of the 8x8, 1-spp Cornell image per mode (passes of 1024 images each,
    # normalized together), in 20 independent chunks: heuristic normalized RRS and plain path
    # tracing have the same mean image luminance within 3 standard errors
    sc = O.OracleScene(scenes.cornell())
    lum = np.array([0.2126, 0.7152, 0.0722])
    means = {}
    for mode, seed in ((O.MODE_HEUR, 3), (O.MODE_OFF, 4)):
        m = []
        for c in range(20):
            cfg = O.make_cfg(8, 8, 1024, 8, mode=mode, pass_begin=10 * c, n_passes=10, seed=seed, tau=0.0)
            img = O.render(sc, cfg)["image"].reshape(-1, 3)
            m.append(float((img @ lum).mean()) / (10 * 1024))
        means[mode] = np.array(m)
    h, p = means[O.MODE_HEUR], means[O.MODE_OFF]
    se = math.sqrt(h.var(ddof=1) / h.size + p.var(ddof=1) / p.size)
    assert abs(h.mean() - p.mean()) < 3.0 * se, (h.mean(), p.mean(), se)
    assert se < 0.005 * p.mean()


def test_net_mode_furnace_unbiased(O, scenes):
    # Network factors make q vary per vertex (splitting + roulette happen), the estimate
    # stays unbiased: the mean matches the furnace closed form.
    sc = O.OracleScene(scenes.furnace())
    rng = np.random.default_rng(0)
    params = rng.normal(0, 0.3, size=O.NPARAM)
    guide = np.full(64, 1.0)
    D = 6
    vals = []
    for c in range(40):
        cfg = O.make_cfg(8, 8, 1, D, mode=O.MODE_NET, pass_begin=c * 10, n_passes=10, tau=0.0)
        r = O.render(sc, cfg, params=params, guide=guide)
        vals.append(r["image"].reshape(-1, 3)[:, 0].mean() / 10)
        assert np.any(r["S"][1:D] != r["n"][1:D]) or c > 0
    vals = np.array(vals)
    se = vals.std(ddof=1) / math.sqrt(vals.size)
    assert se > 0
    assert abs(vals.mean() - furnace_value(D)) < 4 * se


def test_cornell_camera_orientation(O, scenes):
    # the ceiling light appears in the top rows, centred (y = 0 is the top image row)
    sc = O.OracleScene(scenes.cornell())
    cfg = O.make_cfg(32, 32, 1, 1, mode=O.MODE_OFF, n_passes=4)
    img = O.render(sc, cfg)["image"].reshape(32, 32, 3)[..., 0]
    ys, xs = np.nonzero(img > 5.0)
    assert ys.size > 0
    assert ys.max() < 8 and abs(xs.mean() - 15.5) < 2.0


def test_queue_statistics(O, scenes):
    sc = O.OracleScene(scenes.cornell())
    D = 8
    r = O.render(sc, O.make_cfg(32, 32, 2, D, mode=O.MODE_HEUR, n_passes=2))
    nprim = 32 * 32 * 2
    assert np.all(r["S"][1:D] <= 2 * (2 * nprim))     # never exceeds the capacity, in each of 2 passes
    assert abs(r["S"][1:D].mean() / 2 - nprim) < 0.05 * nprim  # E[S] = budget per pass
    off = O.render(sc, O.make_cfg(32, 32, 2, D, mode=O.MODE_OFF, n_passes=2))
    assert np.all(np.diff(off["n"][1:D + 1]) <= 0)    # plain PT only loses paths
    down = O.render(sc, O.make_cfg(32, 32, 2, D, mode=O.MODE_HEUR, norm_mode=O.NORM_DOWNSCALE))
    assert np.all(down["F"][1:D] <= 1.0)


def test_forced_overflow_reduces_alpha(O, scenes):
    sc = O.OracleScene(scenes.cornell())
    cfg = O.make_cfg(16, 16, 1, 6, mode=O.MODE_HEUR, cap_factor=0.9, n_passes=3)
    r = O.render(sc, cfg)
    assert r["status"] == 0
    assert r["retries"].sum() > 0 and r["alpha"] < 1.0
    assert np.all(r["S"][1:6] <= 3 * int(0.9 * 256))
