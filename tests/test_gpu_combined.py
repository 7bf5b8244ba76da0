"""GPU parity where the options meet: next-event estimation with the NRRS factor, instanced
scenes in the NRRS and AID-NRRS modes (against the oracle on the flattened scene), and
hipGraph replay of passes with NEE on an instanced scene against direct launches.

Per-path radiance within 1e-4 relative up to each path's first near-tie decision, as in the
single-option tests; graph replay equal to direct launches within FP64 summation order.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LUM = np.array([0.2126, 0.7152, 0.0722])
LOG2T = 14


@pytest.fixture(scope="module")
def nrrs_mod():
    from paper_2510_07868_amd import nrrs
    nrrs.load()
    return nrrs


def make(nrrs_mod, scene, W, H, s_batch=1, **kw):
    ntri = getattr(scene, "workspace_tris", scene.n_tris)
    base = getattr(scene, "base", scene)
    r = nrrs_mod.Renderer(W, H, s_batch=s_batch, max_tris=max(ntri, 64), max_materials=max(len(base.mat_type), 4),
                          **kw)
    r.upload_scene(scene)
    return r


def _he(rng, n_in, n_out):
    # He-uniform hidden layers, output layer x 0.1, small random biases
    p = []
    for L, (fi, fo) in enumerate(((n_in, 32), (32, 32), (32, 32), (32, n_out))):
        lim = np.sqrt(6.0 / fi) * (0.1 if L == 3 else 1.0)
        p.append(rng.uniform(-lim, lim, size=fi * fo))
        p.append(rng.uniform(-0.1, 0.1, size=fo))
    return np.concatenate(p).astype(np.float32)


def _compare_paths(gp, o, D, rtol=1e-4):
    op = o["path_rgb"]
    first = o["path_first"]
    gp = gp[:, :D]
    keep = (np.arange(1, D + 1)[None, :] < first[:, None])[..., None]
    g = (gp * keep).sum(1)
    ref = (op * keep).sum(1)
    err = np.abs(g - ref) <= rtol * np.abs(ref) + 1e-7 * max(1.0, float(np.abs(ref).mean()))
    bad = ~err.all(1)
    lum = op @ LUM
    covered = float((lum * keep[..., 0]).sum() / max(lum.sum(), 1e-300))
    return bad, float((first > 1).mean()), covered


def _run(O, nrrs_mod, scene, oscene, mode, nee, seed, W=64, H=64, D=8):
    r = make(nrrs_mod, scene, W, H, s_batch=4, trace_depth=D, hash_log2=LOG2T, nee=nee)
    rng = np.random.default_rng(seed)
    guide = rng.uniform(0.02, 2.0, size=W * H).astype(np.float32)
    if mode == nrrs_mod.MODE_NRRS:
        Ps, Pr = _he(rng, 32, 2), _he(rng, 7, 1)
        Pr[-1] = 2.0 * (1.0 - np.log(2.0))  # factors around 1
        T = rng.uniform(-0.3, 0.3, size=8 * 2 * (1 << LOG2T)).astype(np.float32)
        r.set_nrrs_params(Ps, Pr, T)
        params = np.concatenate([Ps, Pr, T]).astype(np.float64)
    else:
        Pa = _he(rng, 32, 1)
        Pa[-1] = 2.0 * (1.0 - np.log(2.0))
        Tr = rng.uniform(-0.3, 0.3, size=8 * 2 * (1 << LOG2T)).astype(np.float32)
        r.set_aid_params(Pa, Tr)
        params = np.concatenate([Pa, Tr]).astype(np.float64)
    r.set_guide(guide)
    r.set_trace(True)
    st = r.render(4, D, mode)
    gp = r.read_trace()
    img, _ = r.read_image()
    r.close()
    o = O.render(oscene, O.make_cfg(W, H, 4, D, n_passes=1, mode=mode, tau=1e-4, hash_log2=LOG2T, nee=nee),
                 paths=True, params=params, guide=guide.astype(np.float64))
    bad, some, covered = _compare_paths(gp, o, D)
    for k in np.nonzero(bad)[0][:5]:
        print("  path", k, "first near-tie depth", o["path_first"][k], "gpu", gp[k, :D].sum(0),
              "oracle", o["path_rgb"][k].sum(0), flush=True)
    assert np.allclose(gp.reshape(W * H, 4, D, 3).sum((1, 2)), img.reshape(-1, 3) * 4, rtol=1e-9, atol=1e-12)
    assert st["overflow"] == 0
    return bad, some, covered


@pytest.mark.parametrize("mode_name", ["MODE_NRRS", "MODE_AID"])
def test_nee_with_the_learned_factor_paths_match_oracle(O, nrrs_mod, scenes, mode_name):
    sc = scenes.cornell()
    mode = getattr(nrrs_mod, mode_name)
    print(f"cornell NEE {mode_name}", flush=True)
    bad, some, covered = _run(O, nrrs_mod, sc, O.OracleScene(sc), mode, 1, 31)
    print(f"cornell NEE {mode_name}: paths compared {some:.4f}, radiance compared {covered:.4f}, "
          f"{int(bad.sum())} paths differ", flush=True)
    assert bad.sum() == 0
    assert some > 0.9 and covered > 0.7


@pytest.mark.parametrize("mode_name,nee", [("MODE_NRRS", 0), ("MODE_AID", 0), ("MODE_NRRS", 1)])
def test_instanced_scene_with_the_learned_factor_paths_match_oracle(O, nrrs_mod, scenes, mode_name, nee):
    isc = scenes.instance_field()
    mode = getattr(nrrs_mod, mode_name)
    print(f"instance field {mode_name} nee {nee}", flush=True)
    bad, some, covered = _run(O, nrrs_mod, isc, O.OracleScene(isc.flatten()), mode, nee, 37)
    print(f"instance field {mode_name} nee {nee}: paths compared {some:.4f}, radiance compared {covered:.4f}, "
          f"{int(bad.sum())} paths differ", flush=True)
    assert bad.sum() == 0
    assert some > 0.95 and covered > 0.85


def test_graph_replay_with_nee_on_an_instanced_scene(nrrs_mod, scenes):
    # each render replays the captured pass; between renders the program reads the image back and
    # synchronizes; every replay equals direct launches (records on, heuristic factor)
    isc = scenes.instance_field()
    W = H = 64
    D = 8
    rg = make(nrrs_mod, isc, W, H, s_batch=2, nee=1, records_cap=4096, p_train=0.3)
    rd = make(nrrs_mod, isc, W, H, s_batch=2, nee=1, records_cap=4096, p_train=0.3)
    rd.set_launch_mode(False)
    for k in range(4):
        sg = rg.render(4, D, nrrs_mod.MODE_HEURISTIC)
        sd = rd.render(4, D, nrrs_mod.MODE_HEURISTIC)
        ig, ng = rg.read_image()
        idr, nd = rd.read_image()
        assert ng == nd == 4 * (k + 1)
        assert np.allclose(ig, idr, rtol=1e-12, atol=1e-15)
        for key in ("n", "S", "retries"):
            assert np.array_equal(sg[key], sd[key]), key
        assert sg["records"] == sd["records"]
    rg.close()
    rd.close()
