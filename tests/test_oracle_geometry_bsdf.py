"""Pins of the oracle's closest-hit query and BSDF sampling.

The rendering equation and its one-sample estimator (Sec. 3, Eqs. 1-2) weight a
sampled direction by f cos / pdf; these tests pin that weight against direct
quadrature of f cos, and the closest-hit query against brute force.
"""
import math

import numpy as np
import pytest


def _soup(rng, n):
    from paper_2510_07868_amd.scenes import Scene
    v = rng.uniform(-1, 1, size=(n * 3, 3)).astype(np.float32)
    # a few large triangles and many small ones
    v[: 3 * (n // 2)] *= 0.2
    v[: 3 * (n // 2)] += rng.uniform(-1, 1, size=(n // 2, 1, 3)).repeat(3, 1).reshape(-1, 3).astype(np.float32)
    return Scene("soup", v, np.arange(3 * n, dtype=np.uint32).reshape(n, 3), np.zeros(n, np.uint32),
                 np.zeros(1, np.uint32), np.array([[0.5, 0.5, 0.5, 1, 0, 0, 0]], np.float32),
                 np.array([0, 0, -3, 0, 0, 0, 0, 1, 0, 60], np.float32), np.zeros(3, np.float32))


def test_bvh_matches_brute_force(O, scenes):
    rng = np.random.default_rng(0)
    for sc in (_soup(rng, 600), scenes.cornell(), scenes.furnace()):
        a = O.OracleScene(sc, bvh=True)
        n = 4000
        o = rng.uniform(-1.2, 1.2, size=(n, 3)) + (0.5 if sc.name != "soup" else 0.0)
        d = rng.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        # aim a quarter of the rays exactly at triangle vertices and edge midpoints
        tv = sc.verts[sc.tris].astype(np.float64)
        k = rng.integers(0, sc.n_tris, size=n // 4)
        tgt = np.where(rng.uniform(size=(n // 4, 1)) < 0.5, tv[k, 0], 0.5 * (tv[k, 0] + tv[k, 1]))
        dd = tgt - o[: n // 4]
        d[: n // 4] = dd / np.linalg.norm(dd, axis=1, keepdims=True)
        rays = np.concatenate([o, d], axis=1)
        ex = rng.integers(0, sc.n_tris, size=n).astype(np.uint32)
        p1, t1, _, _ = O.trace(a, rays, ex, bvh=True)
        p2, t2, _, _ = O.trace(a, rays, ex, bvh=False)
        assert np.array_equal(p1, p2)
        hit = p1 != O.MISS
        assert np.array_equal(t1[hit], t2[hit])
        assert hit.mean() > 0.2


def test_hit_point_is_the_barycentric_point(O, scenes):
    sc = scenes.cornell()
    a = O.OracleScene(sc)
    rng = np.random.default_rng(2)
    tv = sc.verts[sc.tris].astype(np.float64)
    for p in range(sc.n_tris):
        b1, b2 = 0.25, 0.35
        x = (1 - b1 - b2) * tv[p, 0] + b1 * tv[p, 1] + b2 * tv[p, 2]
        n = np.cross(tv[p, 1] - tv[p, 0], tv[p, 2] - tv[p, 0])
        n /= np.linalg.norm(n)
        o = x + 0.05 * n + 0.01 * rng.normal(size=3)
        d = (x - o) / np.linalg.norm(x - o)
        prim, t, bb1, bb2 = O.trace(a, np.concatenate([o, d])[None], None, bvh=False)
        if prim[0] != p:
            continue  # occluded by a nearer triangle (box interiors); the BVH test covers closest-hit
        assert np.allclose(o + t[0] * d, x, atol=1e-12)
        assert bb1[0] == pytest.approx(b1, abs=1e-12) and bb2[0] == pytest.approx(b2, abs=1e-12)


def test_parent_exclusion_and_miss(O, scenes):
    a = O.OracleScene(scenes.two_triangle())
    # from inside triangle R straight towards -z: with R excluded it sees the env
    rays = np.array([[0.0, -1.0, 2.0, 0.0, 0.0, -1.0]])
    p, _, _, _ = O.trace(a, rays, np.array([0], np.uint32))
    assert p[0] == O.MISS


def _hemi_quadrature(fn, nth=400, nph=400):
    """Midpoint rule over the hemisphere in (cos theta, phi): integral of fn(w) dw."""
    ct = (np.arange(nth) + 0.5) / nth
    ph = (np.arange(nph) + 0.5) / nph * 2 * math.pi
    total = 0.0
    for c in ct:
        s = math.sqrt(1 - c * c)
        for p in ph[:: max(1, nph // 100)]:
            total += fn(np.array([s * math.cos(p), s * math.sin(p), c]))
    return total * (1.0 / nth) * (2 * math.pi / len(ph[:: max(1, nph // 100)]))


@pytest.mark.parametrize("alpha", [0.05, 0.2, 0.5])
def test_ggx_ndf_is_normalised(O, alpha):
    # integral of D(h) cos(theta_h) over the hemisphere = 1
    ct = (np.arange(20000) + 0.5) / 20000
    vals = np.array([O.ggx_D(alpha, [math.sqrt(1 - c * c), 0.0, c]) for c in ct])
    assert (vals * ct).sum() / 20000 * 2 * math.pi == pytest.approx(1.0, rel=2e-3 if alpha < 0.1 else 1e-4)


@pytest.mark.parametrize("alpha,theta", [(0.2, 0.3), (0.5, 1.1)])
def test_ggx_visible_normal_identity(O, alpha, theta):
    # integral G1(wo) max(0, wo.h) D(h) dh = cos(theta_o): the visible normals normalise
    wo = np.array([math.sin(theta), 0.0, math.cos(theta)])
    g1 = O.ggx_G1(alpha, wo)
    val = _hemi_quadrature(lambda h: g1 * max(0.0, float(wo @ h)) * O.ggx_D(alpha, h), 600, 200)
    assert val == pytest.approx(wo[2], rel=5e-3)


@pytest.mark.parametrize("alpha,theta,f0", [(0.1, 0.4, 0.9), (0.3, 1.0, 0.5), (0.5, 0.2, 0.1)])
def test_ggx_sample_weight_matches_albedo_quadrature(O, alpha, theta, f0):
    # E[w] over visible-normal samples = integral of f cos over the hemisphere
    wo = np.array([math.sin(theta), 0.0, math.cos(theta)])
    n = 256
    g = (np.arange(n) + 0.5) / n
    ws = []
    for u1 in g:
        for u2 in g[::4]:
            ok, wi, w, pdf = O.ggx_sample(alpha, f0, wo, u1, u2)
            ws.append(w if ok else 0.0)
            if ok:
                # returned weight = f cos / pdf
                assert w == pytest.approx(O.ggx_eval_cos(alpha, f0, wo, wi) / pdf, rel=1e-9)
    mc = float(np.mean(ws))
    quad = _hemi_quadrature(lambda wi: O.ggx_eval_cos(alpha, f0, wo, wi), 800, 400)
    assert mc == pytest.approx(quad, rel=0.02 if alpha < 0.2 else 0.01)


def test_ggx_reciprocity_and_fresnel_limit(O):
    rng = np.random.default_rng(4)
    for _ in range(50):
        a = rng.normal(size=3); a[2] = abs(a[2]); a /= np.linalg.norm(a)
        b = rng.normal(size=3); b[2] = abs(b[2]); b /= np.linalg.norm(b)
        fa = O.ggx_eval_cos(0.3, 0.4, a, b) / b[2]
        fb = O.ggx_eval_cos(0.3, 0.4, b, a) / a[2]
        assert fa == pytest.approx(fb, rel=1e-12)
    # normal incidence mirror configuration: Schlick F = F0
    wo = np.array([0.0, 0.0, 1.0])
    ok, wi, w, _ = O.ggx_sample(0.05, 0.37, wo, 0.0, 0.0)
    assert ok and w == pytest.approx(0.37 * O.ggx_G2(0.05, wo, wi) / O.ggx_G1(0.05, wo), rel=1e-9)


def test_lambert_cosine_sampling_moments(O):
    n = 200
    g = (np.arange(n) + 0.5) / n
    cs = []
    for u1 in g:
        for u2 in g[::10]:
            wi, pdf = O.lambert_sample(u1, u2)
            assert abs(np.linalg.norm(wi) - 1) < 1e-12 and wi[2] > 0
            assert pdf == pytest.approx(wi[2] / math.pi, rel=1e-12)
            cs.append(wi[2])
    cs = np.array(cs)
    # cosine-weighted hemisphere: E[cos] = 2/3, E[cos^2] = 1/2
    assert cs.mean() == pytest.approx(2 / 3, rel=1e-3)
    assert (cs ** 2).mean() == pytest.approx(0.5, rel=1e-3)
