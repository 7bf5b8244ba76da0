"""Mix-Depth (Sec. 4.3): the table searches (host logic) and the oracle's per-depth method gate.

Search pins: the table counts the section states (3^6 = 729, 3^10 = 59,049, and 3^6 + 3^4 = 810
for the segmented search with T_d = 6 over 10 bounces), the brute force returning the maximum
found by scoring every table independently, and the segmented search holding the bounces after
the current segment at the fallback method.

Oracle pins: a NET-mode render whose table selects no depth is the heuristic render; the
default table is depths 1..net_max_depth; bit d-1 gates exactly depth d (the factors, hence the
FP64 sums, at depths before the first network depth are the heuristic ones, and at the first
network depth they are the network's).
"""
import itertools

import numpy as np
import pytest

from paper_2510_07868_amd import mixdepth as M

THREE = ("nrrs", "adrrs", "fixed")


def _counting(score):
    calls = []

    def f(table):
        calls.append(table)
        return score(table)
    return f, calls


@pytest.mark.parametrize("B,count", [(6, 729), (10, 59049)])
def test_brute_force_counts(B, count):
    f, calls = _counting(lambda t: 0.0)
    _, _, n = M.brute_force(B, THREE, f)
    assert n == count == len(calls) == len(set(calls))


def test_heuristic_search_count_depth_10_segment_6():
    f, calls = _counting(lambda t: 0.0)
    table, _, n = M.heuristic_search(10, 6, THREE, f, fallback="fixed")
    assert n == 810 == len(calls)
    assert len(table) == 10
    # first segment: bounces 7..10 held at the fallback while 1..6 are searched
    assert all(t[6:] == ("fixed",) * 4 for t in calls[:729])
    assert len({t[:6] for t in calls[:729]}) == 729
    # second segment: bounces 1..6 fixed to one combination, 7..10 searched
    assert len({t[:6] for t in calls[729:]}) == 1
    assert len({t[6:] for t in calls[729:]}) == 81


def test_brute_force_finds_the_maximum_of_an_arbitrary_score():
    rng = np.random.default_rng(5)
    vals = {t: rng.normal() for t in itertools.product(THREE, repeat=5)}
    best, s, _ = M.brute_force(5, THREE, vals.__getitem__)
    assert s == max(vals.values()) and vals[best] == s


def test_heuristic_search_is_exact_on_a_separable_score():
    # a score that is a sum of per-bounce terms is maximized segment by segment
    rng = np.random.default_rng(6)
    w = {(d, m): rng.normal() for d in range(10) for m in THREE}
    score = lambda t: sum(w[(d, m)] for d, m in enumerate(t))
    best, s, _ = M.heuristic_search(10, 4, THREE, score, fallback="fixed")
    expect = tuple(max(THREE, key=lambda m: w[(d, m)]) for d in range(10))
    assert best == expect and s == pytest.approx(score(expect))


def test_segment_longer_than_the_depth_is_the_brute_force():
    rng = np.random.default_rng(7)
    vals = {t: rng.normal() for t in itertools.product(THREE, repeat=4)}
    a = M.heuristic_search(4, 6, THREE, vals.__getitem__, fallback="fixed")
    b = M.brute_force(4, THREE, vals.__getitem__)
    assert a == b


def test_table_to_mask():
    assert M.table_to_mask((M.NET,) * 4 + (M.HEUR,) * 3) == 0b1111
    assert M.table_to_mask((M.HEUR, M.NET, M.HEUR, M.NET)) == 0b1010
    assert M.table_to_mask((M.FIXED, M.NET, M.FIXED), M.FIXED) == 0b101
    assert M.table_to_mask(()) == 0


def _net_render(O, sc, net_depths, mode=None, seed=0, fixed_depths=0):
    W = H = 16
    rng = np.random.default_rng(11)
    params = rng.normal(0, 0.3, size=O.NPARAM)
    guide = rng.uniform(0.05, 2.0, size=W * H)
    cfg = O.make_cfg(W, H, 2, 6, n_passes=1, mode=O.MODE_NET if mode is None else mode, tau=0.0, seed=seed,
                     net_depths=net_depths, fixed_depths=fixed_depths)
    return O.render(sc, cfg, params=params, guide=guide)


def test_oracle_table_without_network_depths_is_the_heuristic_render(O, scenes):
    sc = O.OracleScene(scenes.cornell())
    a = _net_render(O, sc, 0)
    b = _net_render(O, sc, 0, mode=O.MODE_HEUR)
    assert np.array_equal(a["image"], b["image"])
    assert np.array_equal(a["S"], b["S"]) and np.array_equal(a["sumq"], b["sumq"])


def test_oracle_default_table_is_depths_up_to_net_max_depth(O):
    assert O.make_cfg(4, 4, net_max_depth=4).net_depths == 0b1111
    assert O.make_cfg(4, 4, net_max_depth=2).net_depths == 0b11
    assert O.make_cfg(4, 4, net_max_depth=0).net_depths == 0


def test_oracle_table_bit_gates_its_own_depth(O, scenes):
    sc = O.OracleScene(scenes.cornell())
    heur = _net_render(O, sc, 0)
    full = _net_render(O, sc, 0b1111)
    only2 = _net_render(O, sc, 0b10)
    only1 = _net_render(O, sc, 0b1)
    # depth 1 keeps the heuristic factors when only bit 1 (depth 2) is set
    assert only2["sumq"][1] == heur["sumq"][1] and only2["S"][1] == heur["S"][1]
    assert only2["sumq"][2] != heur["sumq"][2]
    # bit 0 alone gives depth 1 the network factors of the full table
    assert only1["sumq"][1] == full["sumq"][1] and only1["S"][1] == full["S"][1]
    assert full["sumq"][1] != heur["sumq"][1]
    # depth 2 of the depth-1-only table is the heuristic factor on the network's children
    assert only1["sumq"][2] != full["sumq"][2]


class _FakeRenderer:
    """Host stand-in with the renderer's calls: the image of a pass depends only on its pass
    index and the table, the way the random numbers and factors of a real pass do."""

    def __init__(self):
        self.width, self.height, self.s_batch = 4, 2, 2
        self.pass_index, self.mask, self.guide, self.log = 9, 0b1111, np.full(8, 0.5, np.float32), []

    def get_guide(self):
        return self.guide.copy()

    def set_guide(self, g):
        self.guide = np.asarray(g, np.float32).copy()

    def set_timing(self, on):
        pass

    def get_pass_index(self):
        return self.pass_index

    def set_pass_index(self, p):
        self.pass_index = p

    def set_mix_depth(self, m):
        self.mask = m

    def set_mix_depth_fixed(self, m):
        self.fixed = m

    def reset_image(self):
        self.img = None

    def render(self, spp, D, mode):
        self.log.append((self.pass_index, self.mask, spp, float(self.guide[0]), self.fixed))
        rng = np.random.default_rng(self.pass_index)
        self.img = 0.5 + rng.normal(0, 0.1, size=(8, 3)) * (1.0 + 0.1 * bin(self.mask).count("1"))
        self.guide[:] = 123.0          # a real pass refreshes the guide
        self.pass_index += spp // self.s_batch
        return {"stage_ms": {"extend": 2.0, "network": 0.5 * bin(self.mask).count("1")}}

    def read_image(self):
        return self.img.reshape(-1), 2


def test_scorer_renders_every_table_on_the_same_pass_and_cache_state():
    r = _FakeRenderer()
    score = M.render_efficiency_scorer(r, 4, np.full(8, 0.5), mode_net=2)
    tables = list(itertools.product(M.METHODS, repeat=3))
    s = {t: score(t) for t in tables}
    assert [e[0] for e in r.log] == [9] * 27          # common random numbers: pass 9 every time
    assert [e[3] for e in r.log] == [0.5] * 27        # the guide restored before each pass
    assert [e[1] for e in r.log] == [M.table_to_mask(t, M.NET) for t in tables]
    assert [e[4] for e in r.log] == [M.table_to_mask(t, M.FIXED) for t in tables]
    assert all(e[2] == r.s_batch for e in r.log)
    # fewer network depths: lower error and less time in this stand-in, so a higher score
    # (ties between heuristic and fixed keep the first table found)
    assert max(s, key=s.get) == (M.HEUR,) * 3
    assert r.get_pass_index() == 10


def test_oracle_fixed_rate_gives_every_continuing_vertex_one_factor(O, scenes):
    # furnace: every vertex continues; at a fixed-rate depth the raw factors sum to the number of
    # entries (each is 1), and with the budget equal to that count every path has one child
    sc = O.OracleScene(scenes.furnace())
    D = 6
    cfg = O.make_cfg(8, 8, 1, D, mode=O.MODE_HEUR, tau=0.0, fixed_depths=0b11111)
    r = O.render(sc, cfg)
    assert np.all(r["sumq"][1:D] == r["n"][1:D])
    assert np.all(r["S"][1:D] == r["n"][1:D]) and np.all(r["F"][1:D] == 1.0)


def test_oracle_fixed_rate_wins_over_the_network_and_only_at_its_depth(O, scenes):
    sc = O.OracleScene(scenes.cornell())
    both = _net_render(O, sc, 0b1111, fixed_depths=0b10)
    heur_fixed = _net_render(O, sc, 0, mode=O.MODE_HEUR, fixed_depths=0b10)
    net = _net_render(O, sc, 0b1111)
    # depth 1 keeps the network, depth 2 is the fixed rate: a sum of ones, an integer
    assert both["sumq"][1] == net["sumq"][1]
    assert both["sumq"][2] == float(int(both["sumq"][2])) and both["sumq"][2] > 0
    assert heur_fixed["sumq"][2] == float(int(heur_fixed["sumq"][2]))
    assert net["sumq"][2] != float(int(net["sumq"][2]))
