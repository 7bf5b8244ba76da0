"""Pins of the oracle's next-event estimation (one light sample per vertex, shadow ray,
power-heuristic MIS with the BSDF-sampled light hits; the paper's experiments enable NEE, Sec. 6
setup): the MIS pdf of GGX sampling against the sampler itself and its normalisation, and the
unbiasedness of NEE renders against plain path tracing and the furnace's closed form."""
import numpy as np
import pytest

LUMW = np.array([0.2126, 0.7152, 0.0722])


def test_ggx_pdf_is_the_samplers_pdf_and_integrates_with_the_lost_mass_to_one(O):
    rng = np.random.default_rng(0)
    for alpha in (0.05, 0.3, 0.8):
        th = 0.7
        wo = np.array([np.sin(th), 0.0, np.cos(th)])
        lost = 0
        n = 20000
        for _ in range(n):
            ok, wi, w, pdf = O.ggx_sample(alpha, 0.5, wo, rng.random(), rng.random())
            if not ok:
                lost += 1
                continue
            assert O.ggx_pdf(alpha, wo, wi) == pytest.approx(pdf, rel=1e-9)
        # the pdf over the upper hemisphere plus the sampled mass below the horizon is 1
        nt, npph = 400, 400
        ths = (np.arange(nt) + 0.5) / nt * (np.pi / 2)
        phs = (np.arange(npph) + 0.5) / npph * 2 * np.pi
        total = 0.0
        for t in ths:
            for ph in phs[::1]:
                wi = np.array([np.sin(t) * np.cos(ph), np.sin(t) * np.sin(ph), np.cos(t)])
                total += O.ggx_pdf(alpha, wo, wi) * np.sin(t)
        total *= (np.pi / 2 / nt) * (2 * np.pi / npph)
        assert total + lost / n == pytest.approx(1.0, abs=0.02 if alpha < 0.1 else 0.01)


def _mean_lum(O, S, W, H, D, passes, nee, mode, seed):
    vals = []
    for p in range(passes):
        o = O.render(S, O.make_cfg(W, H, 4, D, pass_begin=p, n_passes=1, mode=mode, tau=0.0, nee=nee, seed=seed))
        vals.append((o["image"].reshape(-1, 3) @ LUMW).mean() / 4)
    vals = np.array(vals)
    return vals.mean(), vals.std() / np.sqrt(len(vals))


@pytest.mark.parametrize("mode", [0, 1])
def test_nee_is_unbiased_against_plain_path_tracing_and_lowers_the_variance(O, scenes, mode):
    S = O.OracleScene(scenes.cornell())
    m0, s0 = _mean_lum(O, S, 16, 16, 6, 300, 0, mode, 7)
    m1, s1 = _mean_lum(O, S, 16, 16, 6, 300, 1, mode, 1007)
    assert abs(m1 - m0) < 4 * np.hypot(s0, s1), (m0, m1, s0, s1)
    assert s1 < s0


def test_nee_furnace_mean_is_the_closed_form(O, scenes):
    # every surface emits 1 and reflects 0.7: the expectation of a pixel is sum_{d < D} 0.7^d;
    # NEE and the MIS-weighted hits split that sum between them without changing it
    S = O.OracleScene(scenes.furnace())
    D = 5
    a = float(np.float32(0.7))
    expect = (1 - a ** D) / (1 - a)
    m, se = _mean_lum(O, S, 8, 8, D, 150, 1, 1, 3)
    assert abs(m - expect) < 4 * se + 1e-9, (m, expect, se)
    assert se > 0  # the light samples vary (without NEE the heuristic furnace is exact)
