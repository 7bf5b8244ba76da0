"""GPU parity of NRRS proper (StatNet, NRRS RRSNet, gradient transfer, pixel error; Sec. 4.2,
Sec. 5) against the FP64 oracle, through the C ABI.

Inputs are seeded and synthetic: vertex positions uniform in the scene box, unit outgoing
directions, remapped roughness in [0, 1], throughputs in [0.05, 1], pixel values and radiance
targets log-normal, normalized factors in [0.2, 2.5] (both sides of the RR / splitting switch),
random pixels with several records each.  Tolerances: the GPU computes in float32 (hash-grid
cells and fractions are exact for float32 positions, since the resolutions are powers of two);
the oracle in double."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LOG2T = 14


@pytest.fixture(scope="module")
def nrrs_mod():
    from paper_2510_07868_amd import nrrs
    nrrs.load()
    return nrrs


@pytest.fixture(scope="module")
def N():
    import oracle
    from oracle import nrrs_train
    if not __import__("os").path.exists(oracle.LIB_PATH):
        oracle.build()
    return nrrs_train


def make(nrrs_mod, scenes, W=64, H=48, records_cap=8192, **kw):
    sc = scenes.cornell()
    r = nrrs_mod.Renderer(W, H, s_batch=kw.pop("s_batch", 1), max_tris=max(sc.n_tris, 64),
                          max_materials=max(len(sc.mat_type), 4), records_cap=records_cap, hash_log2=LOG2T, **kw)
    r.upload_scene(sc)
    return r


def params(seed, nrrs_mod):
    rng = np.random.default_rng(seed)
    Ps = rng.normal(0, 0.3, size=nrrs_mod.STAT_NPARAM).astype(np.float32)
    Pr = rng.normal(0, 0.3, size=nrrs_mod.RRS_NPARAM).astype(np.float32)
    T = (rng.normal(0, 0.5, size=8 * 2 * (1 << LOG2T))).astype(np.float32)
    return Ps, Pr, T


def raw_rows(rng, n):
    w = rng.normal(0, 1, size=(n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    raw = np.concatenate([rng.uniform(0, 1, size=(n, 3)), w, rng.uniform(0, 1, size=(n, 1))], 1).astype(np.float32)
    raw[:5, :3] = [[0, 0, 0], [1, 1, 1], [0.5, 0.25, 0.125], [1.0, 0.0, 0.999], [0.0625, 0.5, 1.0]]  # cell edges
    return raw


def test_nrrs_forward_matches_oracle(N, nrrs_mod, scenes):
    r = make(nrrs_mod, scenes)
    Ps, Pr, T = params(1, nrrs_mod)
    r.set_nrrs_params(Ps, Pr, T)
    rng = np.random.default_rng(2)
    n = 2000 + 37  # several blocks and a ragged tail
    raw = raw_rows(rng, n)
    t = rng.uniform(0.05, 1.0, size=(n, 3)).astype(np.float32)
    I = rng.lognormal(-1, 0.7, size=n).astype(np.float32)
    mv, q, enc = r.debug_nrrs_forward(raw, t, I, with_enc=True)
    oenc = N.statnet_encode(T.astype(np.float64), LOG2T, raw.astype(np.float64))
    oq, omv, _ = N.nrrs_factor(Ps.astype(np.float64), Pr.astype(np.float64), T.astype(np.float64), LOG2T,
                               raw.astype(np.float64), t.astype(np.float64), I.astype(np.float64))
    assert np.allclose(enc, oenc, rtol=1e-5, atol=2e-6), np.abs(enc - oenc).max()
    scale = np.abs(omv).max(0)
    assert np.all(np.abs(mv - omv) <= 2e-5 * scale + 1e-5 * np.abs(omv)), np.abs(mv - omv).max(0)
    assert np.allclose(q, oq, rtol=1e-4, atol=1e-6), np.abs(q / oq - 1).max()
    r.close()


@pytest.mark.parametrize("step", [1, 2])
def test_nrrs_gradients_match_oracle(N, nrrs_mod, scenes, step):
    r = make(nrrs_mod, scenes)
    Ps, Pr, T = params(3, nrrs_mod)
    Ps[-2:] = [0.4, 0.2]   # StatNet output biases: means and variances of the targets' scale
    T *= 0.2
    r.set_nrrs_params(Ps, Pr, T)
    rng = np.random.default_rng(4 + step)
    n, npx = 1000 + 29, 97
    raw = raw_rows(rng, n)
    I = rng.lognormal(-1, 0.5, size=n).astype(np.float32)
    L = rng.lognormal(-1, 1.0, size=n).astype(np.float32)
    lum_t = rng.uniform(0.05, 1.0, size=n).astype(np.float32)
    t = rng.uniform(0.05, 1.0, size=(n, 3)).astype(np.float32)
    qn = rng.uniform(0.2, 2.5, size=n).astype(np.float32)
    qn[:7] = 0.0  # no children: skipped by the transfer
    F = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    pix = rng.integers(0, npx, size=n).astype(np.uint32)
    k = np.bincount(pix, minlength=npx).astype(np.uint32)
    wpx = rng.normal(0.5, 1.0, size=npx).astype(np.float32)
    g = r.debug_nrrs_grads(raw, I, L, lum_t, t, qn, F, pix, wpx, k, step, g_rrs=0.01)
    d = lambda a: np.asarray(a, np.float64)
    ols, odPs, odT = N.statnet_loss_grad(d(Ps), d(T), LOG2T, d(raw), d(L), 0.01)
    olr, odPr = N.rrsnet_nrrs_grad(d(Pr), d(Ps), d(T), LOG2T, d(raw), d(t), d(I), d(lum_t), d(qn), d(F), pix, k,
                                   d(wpx), step, g_rrs=0.01, eps=0.01)

    def close(a, b, tol):
        s = np.abs(b).max()
        err = np.abs(a - b).max() / s
        assert err <= tol, err

    assert g["loss_stat"] == pytest.approx(ols, rel=1e-4)
    assert g["loss_rrs"] == pytest.approx(olr, rel=1e-4, abs=1e-7)
    close(g["g_stat"], odPs, 2e-5)
    close(g["g_table"], odT, 2e-5)
    close(g["g_rrs"], odPr, 2e-5)
    r.close()


@pytest.mark.parametrize("first", [True, False])
def test_pixel_error_matches_oracle(N, nrrs_mod, scenes, first):
    r = make(nrrs_mod, scenes, W=64, H=48)
    rng = np.random.default_rng(10 + first)
    w, h = 37, 23  # a ragged block count
    ref = rng.lognormal(-1, 1, size=w * h).astype(np.float32)
    ref[rng.choice(w * h, 40, replace=False)] = -1.0  # pixels without a previous frame
    cur = np.abs(ref + rng.normal(0, 0.2, size=w * h)).astype(np.float32)
    acc = rng.lognormal(-1, 1, size=w * h).astype(np.float32)
    for radius in (0, 2):
        e, E, wpx, acc_g = r.debug_pixel_error(cur, acc, ref, w, h, first, a_mix=0.5, radius=radius, var_scale=48.0)
        oe, oE, owpx, oacc = N.pixel_weights(cur, acc, ref, w, h, first, a_mix=0.5, radius=radius, var_scale=48.0,
                                             g_avg=0.01, g_min=0.05, eps=0.01)
        assert np.allclose(acc_g, oacc, rtol=1e-6, atol=1e-7)
        assert np.allclose(E, oE, rtol=2e-5, atol=1e-7 * oE.max())
        assert e == pytest.approx(oe, rel=2e-5)
        assert np.allclose(wpx, owpx, rtol=2e-5, atol=1e-6 * np.abs(owpx).max())
    r.close()


def test_nrrs_render_is_unbiased_in_the_furnace(nrrs_mod, scenes):
    # any positive factor leaves the estimator unbiased: in the closed grey furnace (albedo a,
    # emission 1) every pixel's expectation is sum_{d < D} a^d, and the pixel mean of an NRRS
    # render stays there within the noise that the varying factors bring
    sc = scenes.furnace()
    D = 8
    a = float(np.float32(0.7))
    expect = (1.0 - a ** D) / (1.0 - a)
    r = nrrs_mod.Renderer(32, 32, s_batch=2, max_tris=max(sc.n_tris, 64), max_materials=4, hash_log2=LOG2T)
    r.upload_scene(sc)
    Ps, Pr, T = params(7, nrrs_mod)
    r.set_nrrs_params(Ps, Pr * 0.3, T * 0.3)
    r.set_guide(np.full(32 * 32, 0.5, np.float32))
    st = r.render(64, D, nrrs_mod.MODE_NRRS)
    img, spp = r.read_image()
    lum = img.reshape(-1, 3) @ np.array([0.2126, 0.7152, 0.0722])
    assert spp == 64 and st["status"] == 0
    se = lum.std() / np.sqrt(lum.size)
    assert abs(lum.mean() - expect) < 5 * se + 1e-6, (lum.mean(), expect, se)
    # the NRRS factors vary from vertex to vertex: unlike the heuristic furnace, pixels differ
    assert lum.std() > 1e-4
    r.close()


def test_nrrs_training_loop_runs_and_lowers_the_statnet_loss(nrrs_mod, scenes):
    r = make(nrrs_mod, scenes, W=64, H=48, s_batch=4, records_cap=1 << 15, p_train=0.25)
    losses, steps2 = [], []
    for f in range(12):
        st = r.render(4, 6, nrrs_mod.MODE_NRRS)
        n = min(st["records"], 1 << 15)
        assert n > 1000
        out = r.train_step_nrrs(n, 1 if f < 6 else 2)
        losses.append(out["loss_stat"])
        if f >= 6:
            steps2.append(out)
        assert np.isfinite(out["loss_stat"]) and np.isfinite(out["loss_rrs"]) and np.isfinite(out["e_avg"])
    assert all(o["rrs_trained"] for o in steps2)
    assert np.mean(losses[-3:]) < np.mean(losses[:3])
    Ps, Pr, T = r.get_nrrs_params()
    assert np.all(np.isfinite(Ps)) and np.all(np.isfinite(Pr)) and np.all(np.isfinite(T))
    img, _ = r.read_image()
    assert np.all(np.isfinite(img))
    r.close()


def _he(rng, n_in, n_out):
    # He-uniform hidden layers, output layer x 0.1, small random biases (the library's init shape)
    p = []
    for L, (fi, fo) in enumerate(((n_in, 32), (32, 32), (32, 32), (32, n_out))):
        lim = np.sqrt(6.0 / fi) * (0.1 if L == 3 else 1.0)
        p.append(rng.uniform(-lim, lim, size=fi * fo))
        p.append(rng.uniform(-0.1, 0.1, size=fo))
    return np.concatenate(p).astype(np.float32)


# (19: the benchmark's table size; history 0.5: half the pixels, at random, have no history and
# keep the heuristic factor, so the kernel's groups gather live entries from ragged runs)
@pytest.mark.parametrize("log2t,history", [(LOG2T, 1.0), (19, 1.0), (LOG2T, 0.5)])
def test_nrrs_cornell_paths_match_oracle(O, nrrs_mod, scenes, log2t, history):
    # every primary path of a 64x64, 4-spp Cornell pass in NRRS mode (StatNet + RRSNet factors at
    # depths 1-4) against the oracle on the same random numbers, at 1e-4 relative, up to the depth
    # of its first near-tie decision (the oracle widens the roulette's near-tie margin by the
    # factor's change over its inputs' float32 error bounds)
    from test_gpu_parity import _compare_paths, _report_paths
    W = H = 64
    D = 8
    sc = scenes.cornell()
    r = nrrs_mod.Renderer(W, H, s_batch=4, max_tris=max(sc.n_tris, 64), max_materials=max(len(sc.mat_type), 4),
                          trace_depth=D, hash_log2=log2t)
    r.upload_scene(sc)
    rng = np.random.default_rng(21)
    Ps, Pr = _he(rng, 32, 2), _he(rng, 7, 1)
    Pr[-1] = 2.0 * (1.0 - np.log(2.0))  # factors around 1
    T = rng.uniform(-0.3, 0.3, size=8 * 2 * (1 << log2t)).astype(np.float32)
    guide = rng.uniform(0.02, 2.0, size=W * H).astype(np.float32)
    guide[rng.random(W * H) >= history] = -1.0  # no history: the heuristic factor stays
    r.set_nrrs_params(Ps, Pr, T)
    r.set_guide(guide)
    r.set_trace(True)
    st = r.render(4, D, nrrs_mod.MODE_NRRS)
    gp = r.read_trace()
    img, _ = r.read_image()
    params = np.concatenate([Ps, Pr, T]).astype(np.float64)
    o = O.render(O.OracleScene(sc), O.make_cfg(W, H, 4, D, n_passes=1, mode=O.MODE_NRRS, tau=1e-4, hash_log2=log2t),
                 paths=True, params=params, guide=guide.astype(np.float64))
    bad, some, full, covered = _compare_paths(gp, o, D)
    _report_paths("cornell NRRS", gp, o, D, bad, some, full, covered)
    assert bad.sum() == 0
    assert some > 0.99 and covered > 0.9
    assert np.allclose(gp.reshape(W * H, 4, D, 3).sum((1, 2)), img.reshape(-1, 3) * 4, rtol=1e-9, atol=1e-12)
    # the NRRS factors differ from the heuristic ones: the per-depth factor sums differ
    oh = O.render(O.OracleScene(sc), O.make_cfg(W, H, 4, D, n_passes=1, mode=O.MODE_HEUR, tau=1e-4))
    assert not np.allclose(o["sumq"][1:5], oh["sumq"][1:5], rtol=1e-3)
    assert st["overflow"] == 0
    r.close()


# ------------------------------------------------------------------ AID-NRRS
def test_aid_forward_matches_oracle(N, nrrs_mod, scenes):
    r = make(nrrs_mod, scenes)
    rng = np.random.default_rng(31)
    Pa = _he(rng, 32, 1)
    Tr = rng.normal(0, 0.5, size=8 * 2 * (1 << LOG2T)).astype(np.float32)
    r.set_aid_params(Pa, Tr)
    n = 2000 + 37
    raw = raw_rows(rng, n)
    t = rng.uniform(0.05, 1.0, size=(n, 3)).astype(np.float32)
    I = rng.lognormal(-1, 0.7, size=n).astype(np.float32)
    q, enc = r.debug_aid_forward(raw, t, I, with_enc=True)
    d = lambda a: np.asarray(a, np.float64)
    oenc = N.aid_encode(d(Tr), LOG2T, d(raw), d(t), d(I))
    oq, _ = N.aid_factor(d(Pa), d(Tr), LOG2T, d(raw), d(t), d(I))
    assert np.allclose(enc, oenc, rtol=1e-5, atol=2e-6), np.abs(enc - oenc).max()
    assert np.allclose(q, oq, rtol=1e-4, atol=1e-6), np.abs(q / oq - 1).max()
    r.close()


@pytest.mark.parametrize("step", [1, 2])
def test_aid_gradients_match_oracle(N, nrrs_mod, scenes, step):
    r = make(nrrs_mod, scenes)
    Ps, _, T = params(33, nrrs_mod)
    Ps[-2:] = [0.4, 0.2]
    T *= 0.2
    rng = np.random.default_rng(34 + step)
    Pa = _he(rng, 32, 1)
    Tr = (rng.normal(0, 0.3, size=8 * 2 * (1 << LOG2T))).astype(np.float32)
    r.set_nrrs_params(Ps, None, T)
    r.set_aid_params(Pa, Tr)
    n, npx = 1000 + 29, 97
    raw = raw_rows(rng, n)
    I = rng.lognormal(-1, 0.5, size=n).astype(np.float32)
    lum_t = rng.uniform(0.05, 1.0, size=n).astype(np.float32)
    t = rng.uniform(0.05, 1.0, size=(n, 3)).astype(np.float32)
    qn = rng.uniform(0.2, 2.5, size=n).astype(np.float32)
    qn[:7] = 0.0
    F = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    pix = rng.integers(0, npx, size=n).astype(np.uint32)
    k = np.bincount(pix, minlength=npx).astype(np.uint32)
    wpx = rng.normal(0.5, 1.0, size=npx).astype(np.float32)
    g = r.debug_aid_grads(raw, I, lum_t, t, qn, F, pix, wpx, k, step, g_rrs=0.01)
    d = lambda a: np.asarray(a, np.float64)
    ol, odPa, odT = N.aid_grad(d(Pa), d(Tr), d(Ps), d(T), LOG2T, d(raw), d(t), d(I), d(lum_t), d(qn), d(F), pix, k,
                               d(wpx), step, g_rrs=0.01, eps=0.01)

    def close(a, b, tol):
        err = np.abs(a - b).max() / np.abs(b).max()
        assert err <= tol, err

    assert g["loss"] == pytest.approx(ol, rel=1e-4, abs=1e-7)
    close(g["g_aid"], odPa, 2e-5)
    close(g["g_table_r"], odT, 2e-5)
    r.close()


@pytest.mark.parametrize("log2t,history", [(LOG2T, 1.0), (19, 1.0), (LOG2T, 0.5)])
def test_aid_cornell_paths_match_oracle(O, nrrs_mod, scenes, log2t, history):
    # the AID-NRRS factor in a 64x64, 4-spp Cornell pass, path by path against the oracle
    from test_gpu_parity import _compare_paths, _report_paths
    W = H = 64
    D = 8
    sc = scenes.cornell()
    r = nrrs_mod.Renderer(W, H, s_batch=4, max_tris=max(sc.n_tris, 64), max_materials=max(len(sc.mat_type), 4),
                          trace_depth=D, hash_log2=log2t)
    r.upload_scene(sc)
    rng = np.random.default_rng(41)
    Pa = _he(rng, 32, 1)
    Pa[-1] = 2.0 * (1.0 - np.log(2.0))
    Tr = rng.uniform(-0.3, 0.3, size=8 * 2 * (1 << log2t)).astype(np.float32)
    guide = rng.uniform(0.02, 2.0, size=W * H).astype(np.float32)
    guide[rng.random(W * H) >= history] = -1.0
    r.set_aid_params(Pa, Tr)
    r.set_guide(guide)
    r.set_trace(True)
    st = r.render(4, D, nrrs_mod.MODE_AID)
    gp = r.read_trace()
    params = np.concatenate([Pa, Tr]).astype(np.float64)
    o = O.render(O.OracleScene(sc), O.make_cfg(W, H, 4, D, n_passes=1, mode=O.MODE_AID, tau=1e-4, hash_log2=log2t),
                 paths=True, params=params, guide=guide.astype(np.float64))
    bad, some, full, covered = _compare_paths(gp, o, D)
    _report_paths("cornell AID-NRRS", gp, o, D, bad, some, full, covered)
    assert bad.sum() == 0
    assert some > 0.99 and covered > 0.9
    assert st["overflow"] == 0
    r.close()


def test_aid_training_loop_runs(nrrs_mod, scenes):
    r = make(nrrs_mod, scenes, W=64, H=48, s_batch=4, records_cap=1 << 15, p_train=0.25)
    for f in range(8):
        st = r.render(4, 6, nrrs_mod.MODE_AID)
        n = min(st["records"], 1 << 15)
        out = r.train_step_nrrs(n, 1 if f < 4 else 2, variant=1)
        assert np.isfinite(out["loss_stat"]) and np.isfinite(out["loss_rrs"])
        assert out["rrs_trained"]
    pa, tr = r.get_aid_params()
    assert np.all(np.isfinite(pa)) and np.all(np.isfinite(tr))
    pa0 = r.get_nrrs_params()[1]
    assert np.all(np.isfinite(pa0))
    r.close()
