"""GPU parity of two-level (instanced) scenes against the FP64 oracle on the flattened scene.

The renderer keeps one copy of each object-space mesh, a tree per mesh and a tree over the
instances' world boxes, and moves rays into an instance's object space during traversal; the
oracle traces the flattened world-space triangles.  Closest hits: same triangle (in the
flattened numbering) and t within 1e-5 (plus the effect of the flattened corners' float32
rounding) outside the oracle's near-ties, for every traversal
variant available to such scenes; per-path radiance within 1e-4 relative up to each path's
first near-tie decision, with and without next-event estimation, also for a scene made of
instances only (its lights too).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LUM = np.array([0.2126, 0.7152, 0.0722])


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


def _assert_t_close(flat, rays32, op, ot, gt, hit):
    # distances within 1e-5 relative, plus the rounding of the flattened triangle's corners to
    # float32 (the renderer intersects the exactly placed object-space triangle): a corner moved
    # by half a unit in the last place of its coordinates moves the hit by that over |cos| of
    # the ray against the triangle (and the float32 move of the ray into object space, by up to
    # a few units in the last place of the scene's coordinates times the map's condition)
    k = np.nonzero(hit)[0]
    v = flat.verts.astype(np.float64)[flat.tris[op[k]].astype(np.int64)]
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    d = rays32[k, 3:].astype(np.float64)
    cos = np.abs(np.einsum("ij,ij->i", nrm, d)) / np.linalg.norm(d, axis=1)
    scale = np.maximum(np.abs(v).max((1, 2)), np.abs(rays32[k, :3]).max(1))
    tol = 1e-5 * ot[k] + 1e-6 + 32.0 * 2.0 ** -24 * scale / np.maximum(cos, 1e-4)
    err = np.abs(gt[k] - ot[k])
    worst = int(np.argmax(err / tol))
    assert np.all(err <= tol), (int((err > tol).sum()), float(err[worst]), float(tol[worst]), float(cos[worst]))


def _rays(sc, n, seed):
    rng = np.random.default_rng(seed)
    lo = sc.verts.min(0).astype(np.float64)
    hi = sc.verts.max(0).astype(np.float64)
    o = lo + (hi - lo) * rng.uniform(-0.05, 1.05, size=(n, 3))
    o[:, 1] = np.maximum(o[:, 1], lo[1] + 0.05 * (hi[1] - lo[1]))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.concatenate([o, d], 1).astype(np.float32)


@pytest.mark.parametrize("name", ["cornell_instanced", "instance_field", "instances_only"])
def test_instanced_closest_hits_match_the_flattened_oracle(O, nrrs_mod, scenes, name):
    isc = getattr(scenes, name)()
    flat = isc.flatten()
    print(f"closest hits {name}", flush=True)
    r = make(nrrs_mod, isc, 256, 256)
    osc = O.OracleScene(flat)
    n = 50000
    rays32 = _rays(flat, n, 11)
    op, ot, _, _, frag = O.trace(osc, rays32.astype(np.float64), None, tau=1e-4, with_fragile=True)
    ok = ~frag
    hit = ok & (op != O.MISS)
    assert ok.mean() > 0.95 and hit.sum() > n // 10
    # rays that hit an instance, not only the base mesh
    assert (op[hit] >= isc.base.n_tris).sum() > n // 50
    occ = r.get_tuning()["extend_max_blocks_per_cu"]
    assert occ[2] == 0 and occ[4] == 0  # variants 2 and 4 are not offered for instanced scenes
    for variant, bpc, refill, batch, chunk in ((3, occ[3], 16, 12, 64), (3, 1, 1, 1, 0), (1, occ[1], 16, 32, 64),
                                               (1, 1, 8, 1, 0), (0, occ[0], 16, 32, 0), (0, 1, 1, 1, 1)):
        r.set_tuning(variant, bpc, refill, batch, chunk)
        gp, gt, _, _ = r.debug_trace(rays32)
        bad = ok & (gp != op)
        assert bad.sum() == 0, (variant, bpc, np.nonzero(bad)[0][:8], gp[bad][:8], op[bad][:8])
        _assert_t_close(flat, rays32, op, ot, gt, hit)
    for variant in (2, 4):
        with pytest.raises(RuntimeError):
            r.set_tuning(variant, 1, 16, 16, 64)


def test_instanced_closest_hits_with_excluded_triangles(O, nrrs_mod, scenes):
    # rays leaving points 1e-4 above random triangles (base and instances) with that triangle
    # excluded, as continuation rays are: the exclusion names a placed triangle, not its mesh's
    isc = scenes.instance_field(2, 64)
    flat = isc.flatten()
    r = make(nrrs_mod, isc, 256, 256)
    osc = O.OracleScene(flat)
    rng = np.random.default_rng(5)
    n = 40000
    tri = rng.integers(0, flat.n_tris, size=n)
    v = flat.verts.astype(np.float64)[flat.tris[tri].astype(np.int64)]
    a, b = rng.uniform(size=(2, n))
    swap = a + b > 1.0
    a[swap], b[swap] = 1.0 - a[swap], 1.0 - b[swap]
    p = v[:, 0] + a[:, None] * (v[:, 1] - v[:, 0]) + b[:, None] * (v[:, 2] - v[:, 0])
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True) + 1e-300
    d = rng.normal(size=(n, 3))
    d *= np.sign(np.einsum("ij,ij->i", d, nrm))[:, None]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = p + 1e-4 * nrm
    rays32 = np.concatenate([o, d], 1).astype(np.float32)
    op, ot, _, _, frag = O.trace(osc, rays32.astype(np.float64), tri.astype(np.uint32), tau=1e-4, with_fragile=True)
    gp, gt, _, _ = r.debug_trace(rays32, tri.astype(np.uint32))
    ok = ~frag
    hit = ok & (op != O.MISS)
    assert ok.mean() > 0.9 and hit.sum() > n // 20
    bad = ok & (gp != op)
    assert bad.sum() == 0, (np.nonzero(bad)[0][:10], bad.sum())
    _assert_t_close(flat, rays32, op, ot, gt, hit)


def _compare_paths(gp, o, D, rtol=1e-4):
    op = o["path_rgb"]
    first = o["path_first"]
    assert gp.shape[0] == op.shape[0] and gp.shape[1] >= D
    gp = gp[:, :D]
    keep = (np.arange(1, D + 1)[None, :] < first[:, None])[..., None]
    g = (gp * keep).sum(1)
    ref = (op * keep).sum(1)
    err = np.abs(g - ref) <= rtol * np.abs(ref) + 1e-7 * max(1.0, float(np.abs(ref).mean()))
    bad = ~err.all(1)
    lum = op @ LUM
    covered = float((lum * keep[..., 0]).sum() / max(lum.sum(), 1e-300))
    return bad, float((first > 1).mean()), covered


@pytest.mark.parametrize("name,mode,nee", [("cornell_instanced", 0, 0), ("cornell_instanced", 1, 0),
                                           ("cornell_instanced", 1, 1), ("instance_field", 1, 0),
                                           ("instance_field", 1, 1), ("instances_only", 1, 0),
                                           ("instances_only", 1, 1)])
def test_instanced_paths_match_the_flattened_oracle(O, nrrs_mod, scenes, name, mode, nee):
    # every primary path of a 64x64, 4-spp pass against the oracle on the flattened scene at
    # 1e-4 relative up to its first near-tie decision
    W = H = 64
    D = 8
    isc = getattr(scenes, name)()
    print(f"paths {name} mode {mode} nee {nee}", flush=True)
    r = make(nrrs_mod, isc, W, H, s_batch=4, trace_depth=D, nee=nee)
    r.set_trace(True)
    st = r.render(4, D, mode)
    gp = r.read_trace()
    img, _ = r.read_image()
    o = O.render(O.OracleScene(isc.flatten()), O.make_cfg(W, H, 4, D, n_passes=1, mode=mode, tau=1e-4, nee=nee),
                 paths=True)
    bad, some, covered = _compare_paths(gp, o, D)
    print(f"{name} mode {mode} nee {nee}: paths compared {some:.4f}, radiance compared {covered:.4f}, "
          f"{int(bad.sum())} paths differ", flush=True)
    for k in np.nonzero(bad)[0][:5]:
        print("  path", k, "first near-tie depth", o["path_first"][k], "gpu", gp[k, :D].sum(0),
              "oracle", o["path_rgb"][k].sum(0), flush=True)
    assert bad.sum() == 0
    assert some > (0.9 if nee else 0.97) and covered > (0.7 if nee else 0.9)
    assert np.allclose(gp.reshape(W * H, 4, D, 3).sum((1, 2)), img.reshape(-1, 3) * 4, rtol=1e-9, atol=1e-12)
    assert st["overflow"] == 0


def test_terrain5m_instanced_full_size_paths(O, nrrs_mod, scenes):
    # the batched configuration's scene with its 2000 boxes as instances of one unit box, at full
    # size (1920x1080, 1 spp, depth 32, heuristic normalized RRS, as the benchmark's instanced
    # leg): sampled closest hits against the oracle's BVH over the flattened 5.0 M triangles, the
    # depth-1 factor sum of the free-running pass, and with the oracle's normalization factors
    # (one near-tie path moves every path's factor) every primary path up to its first near-tie
    isc = scenes.terrain5m_instanced(0)
    flat = isc.flatten()
    W, H, D = 1920, 1080, 32
    print("terrain5m instanced: upload", flush=True)
    r = make(nrrs_mod, isc, W, H, s_batch=1, trace_depth=D)
    osc = O.OracleScene(flat)
    n = 4000
    rays32 = _rays(flat, n, 21)
    op, ot, _, _, frag = O.trace(osc, rays32.astype(np.float64), None, tau=1e-4, with_fragile=True)
    gp, gt, _, _ = r.debug_trace(rays32)
    ok = ~frag
    hit = ok & (op != O.MISS)
    assert ok.mean() > 0.95 and hit.sum() > n // 10
    assert np.array_equal(gp[ok], op[ok])
    _assert_t_close(flat, rays32, op, ot, gt, hit)
    print("terrain5m instanced: oracle pass", flush=True)
    o = O.render(osc, O.make_cfg(W, H, 1, D, n_passes=1, mode=O.MODE_HEUR, tau=1e-4), paths=True)
    print("terrain5m instanced: GPU pass", flush=True)
    st = r.render(1, D, nrrs_mod.MODE_HEURISTIC)
    assert st["overflow"] == 0
    assert st["sumq"][1] == pytest.approx(o["sumq"][1], rel=2e-5)
    r.set_pass_index(0)
    r.reset_image()
    r.debug_set_norm_factors(o["F"][1:D])
    r.set_trace(True)
    print("terrain5m instanced: GPU pass with the oracle's factors", flush=True)
    st2 = r.render(1, D, nrrs_mod.MODE_HEURISTIC)
    tr = r.read_trace()
    assert st2["overflow"] == 0
    bad, some, covered = _compare_paths(tr, o, D)
    print(f"terrain5m instanced: paths compared {some:.4f}, radiance compared {covered:.4f}, "
          f"{int(bad.sum())} paths differ", flush=True)
    for k in np.nonzero(bad)[0][:5]:
        f = int(o["path_first"][k])
        print("  path", k, "first near-tie depth", f, "gpu", tr[k, :min(f, D)].sum(0).tolist(),
              "oracle", o["path_rgb"][k, :min(f, D)].sum(0).tolist(), flush=True)
    assert bad.sum() == 0 and some > 0.97 and covered > 0.88
