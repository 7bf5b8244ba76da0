"""Pins of the oracle's random numbers and of its normalization / roulette / scan step.

Normalization: Sec. 4.1.2, Eqs. (9)-(11).  Stochastic rounding: Sec. 3, Eq. (8).
Boundedness statement and proof: Sec. 4.1.3.  Rate control, Bernstein bound and
adaptive alpha: Sec. 4.1.4, Eqs. (12)-(14).  Downscale-only variant: Sec. 5 "Compromise".
"""
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(O):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(O.philox(ctr, key)) == out


def test_uniform_mapping_range(O):
    # u = (x >> 8) * 2^-24 lies in [0, 1) and is exactly representable in float32
    xs = np.array([0, 255, 256, 0xFFFFFFFF], np.uint64)
    u = (xs >> 8).astype(np.float64) * 2.0 ** -24
    assert u[0] == 0.0 and u[1] == 0.0 and u[2] == 2.0 ** -24 and u[3] == 1.0 - 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def _draw_u(rng, n):
    return (rng.integers(0, 2 ** 24, size=n)).astype(np.float64) * 2.0 ** -24


def test_integer_factors_are_deterministic(O):
    # q_norm integral => X = q_norm exactly, whatever u (Eq. 8 with zero residual)
    q = np.array([1.0, 2.0, 3.0, 0.0, 2.0])  # sum 8, budget 8 -> F = 1
    for s in range(5):
        r = O.rrs_expand(q, _draw_u(np.random.default_rng(s), 5), budget_base=8, cap=100)
        assert list(r["X"]) == [1, 2, 3, 0, 2]
        assert r["S"] == 8
        assert list(r["offset"]) == [0, 1, 3, 6, 6]
        assert list(r["parent"]) == [0, 1, 1, 2, 2, 2, 4, 4]


def test_all_zero_factors_end_the_pass(O):
    r = O.rrs_expand(np.zeros(7), np.zeros(7), budget_base=7)
    assert r["S"] == 0 and np.all(r["X"] == 0)


def test_empty_input(O):
    r = O.rrs_expand(np.zeros(0), np.zeros(0), budget_base=4)
    assert r["S"] == 0 and r["X"].size == 0


def test_normalized_factors_sum_to_budget(O):
    # Eq. (11): sum q_norm = N_px (up to the float32 rounding of each factor)
    rng = np.random.default_rng(1)
    q = rng.lognormal(0.0, 2.0, size=5000)
    r = O.rrs_expand(q, _draw_u(rng, q.size), budget_base=5000)
    qn = r["q_norm"].astype(np.float64)
    assert abs(qn.sum() - 5000.0) < 5000 * 2e-7 * 4
    assert r["F"] == pytest.approx(5000.0 / q.sum(), rel=1e-15)
    # floor/ceil bounds and the scan / parent map
    X = r["X"].astype(np.int64)
    assert np.all(X >= np.floor(qn)) and np.all(X <= np.ceil(qn))
    assert np.array_equal(r["offset"], np.concatenate([[0], np.cumsum(X)[:-1]]).astype(np.uint64))
    assert np.array_equal(r["parent"], np.repeat(np.arange(q.size), X).astype(np.uint32))


def test_residual_rule_is_strict_less(O):
    # X = floor(q) + [u < frac(q)]: u equal to the residual does not add a child
    q = np.array([0.5, 0.5, 1.25, 1.25])
    u = np.array([0.5, 0.5 - 2 ** -24, 0.25, 0.25 - 2 ** -24])
    r = O.rrs_expand(q, u, budget_base=3.5, cap=10)
    assert list(r["X"]) == [0, 1, 1, 2]


def test_expectation_and_variance_of_S(O):
    # Sec. 4.1.3: E[S] = N_px and Var(S | q) = sum r_i (1 - r_i) <= rho <= N_px, <= |I|/4
    rng = np.random.default_rng(7)
    n, budget = 400, 300.0
    q = rng.uniform(0.0, 3.0, size=n)
    trials = 20000
    S = np.empty(trials)
    for k in range(trials):
        S[k] = O.rrs_expand(q, _draw_u(rng, n), budget_base=budget, cap=10 ** 6)["S"]
    qn = O.rrs_expand(q, np.zeros(n), budget_base=budget, cap=10 ** 6)["q_norm"].astype(np.float64)
    r = qn - np.floor(qn)
    var_theory = float(np.sum(r * (1 - r)))
    mean_theory = float(qn.sum())
    assert abs(S.mean() - mean_theory) < 4 * math.sqrt(var_theory / trials)
    assert abs(mean_theory - budget) < 1e-3
    # sample variance within 4 standard errors (SE of a variance ~ var*sqrt(2/(n-1)))
    assert abs(S.var(ddof=1) - var_theory) < 4 * var_theory * math.sqrt(2.0 / (trials - 1))
    assert var_theory <= r.sum() <= budget + 1e-9
    assert var_theory <= n / 4.0


def test_each_count_is_unbiased(O):
    # E[X_i] = q_norm_i for every parent (Eq. 8), checked per entry
    rng = np.random.default_rng(3)
    q = np.array([0.1, 0.9, 1.5, 2.25, 0.0, 4.75])
    acc = np.zeros(q.size)
    trials = 40000
    for _ in range(trials):
        acc += O.rrs_expand(q, _draw_u(rng, q.size), budget_base=q.sum(), cap=100)["X"]
    qn = O.rrs_expand(q, np.zeros(q.size), budget_base=q.sum(), cap=100)["q_norm"].astype(np.float64)
    r = qn - np.floor(qn)
    se = np.sqrt(np.maximum(r * (1 - r), 1e-12) / trials)
    assert np.all(np.abs(acc / trials - qn) < 5 * se + 1e-12)


def test_bernstein_exponent_example():
    # The paper prints exponent ~ -0.0125 N_px for f_rate = 0.85 (Eq. 13)
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))["bernstein_f_rate_example"]
    f = g["f_rate"]
    expo = -((1 - f) ** 2) / (2 * f + (2.0 / 3.0) * (1 - f))
    assert expo == pytest.approx(g["exponent_per_Npx"], rel=1e-12)


def test_rate_controlled_overflow_frequency_below_bernstein_bound(O):
    # P(S' >= N_px) <= exp(-(1-f)^2 N / (2f + 2/3 (1-f))) for q' = f_rate * q_norm (Eqs. 12-13)
    rng = np.random.default_rng(11)
    N, f = 64, 0.85
    q = rng.uniform(0.0, 2.0, size=N)
    bound = math.exp(-((1 - f) ** 2) * N / (2 * f + (2.0 / 3.0) * (1 - f)))
    trials, over = 20000, 0
    for _ in range(trials):
        r = O.rrs_expand(q, _draw_u(rng, N), budget_base=N, f_rate=f, cap=10 ** 6)
        over += r["S"] >= N
        assert abs(float(r["q_norm"].astype(np.float64).sum()) - f * N) < 1e-3
    assert over / trials <= bound
    assert over > 0  # the bound is not vacuous here: overflow does happen sometimes


def test_overflow_guard_shrinks_alpha(O):
    # Eq. (14): alpha <- alpha (1 - 0.01) until the realised count fits the capacity
    rng = np.random.default_rng(5)
    n = 1000
    q = rng.uniform(0.0, 1.0, size=n)
    u = _draw_u(rng, n)
    r = O.rrs_expand(q, u, budget_base=n, cap=int(0.9 * n))
    assert r["status"] == 0 and r["S"] <= int(0.9 * n)
    assert r["retries"] >= 1
    assert r["alpha"] == pytest.approx(0.99 ** r["retries"], rel=1e-12)
    # one retry fewer would not fit: the guard stops at the first alpha that fits
    prev = O.rrs_expand(q, u, budget_base=n, alpha=0.99 ** (r["retries"] - 1), cap=10 ** 9)
    assert prev["S"] > int(0.9 * n)
    # same uniforms: counts only shrink as alpha shrinks (X is monotone in q)
    assert np.all(r["X"] <= prev["X"])


def test_overflow_guard_gives_up_below_min_alpha(O):
    q = np.ones(10)
    r = O.rrs_expand(q, np.zeros(10), budget_base=10, cap=0)
    assert r["status"] == -5


def test_downscale_only_mode(O):
    # Sec. 5 "Compromise": normalise only when F_norm < 1
    q = np.full(10, 0.1)  # sum 1 < budget 10 -> F would be 10, downscale keeps 1
    r = O.rrs_expand(q, np.zeros(10), budget_base=10, norm_mode=O.NORM_DOWNSCALE)
    assert r["F"] == 1.0
    r2 = O.rrs_expand(np.full(10, 5.0), np.zeros(10), budget_base=10, norm_mode=O.NORM_DOWNSCALE)
    assert r2["F"] == pytest.approx(0.2, rel=1e-15)


def test_one_parent_owns_the_whole_budget(O):
    q = np.zeros(257)
    q[100] = 3.0
    r = O.rrs_expand(q, np.full(257, 0.5), budget_base=512, cap=1024)
    assert r["X"][100] == 512 and r["S"] == 512
    assert np.all(r["parent"] == 100)
