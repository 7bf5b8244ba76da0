"""Mix-Depth (Sec. 4.3): choose the RRS method per bounce by searching over method tables.

A table assigns one method to each bounce 1..B.  `brute_force` scores every table (k^B for
k methods); `heuristic_search` splits the bounces into segments of T_d, fills every bounce
with the fallback method, then brute-forces the segments from the shallowest one, fixing
each segment to its best combination before moving on (k^T_d + k^(B - T_d) + ... tables).
Both are host-side post-processing over a caller-supplied score (higher = better); they do
not touch training.

`render_efficiency_scorer` is the score this renderer uses: one wavefront pass rendered with
the table on common random numbers, efficiency = 1 / (RelMSE against a reference image x GPU
time of the pass).  The methods available per bounce here are the network factor (NET), the
heuristic factor lum(throughput x albedo) (HEUR) and the fixed rate (FIXED: the same raw factor
for every vertex that continues), all normalized per depth (Sec. 4.1 Eqs. 9-10).
"""
import itertools

import numpy as np

NET, HEUR, FIXED = "net", "heur", "fixed"
METHODS = (NET, HEUR, FIXED)
LUM = np.array([0.2126, 0.7152, 0.0722])


def brute_force(n_bounces, methods, score, prefix=(), suffix=()):
    """Score prefix + c + suffix for every c in methods^n_bounces; return (best table, best
    score, number of tables scored).  Ties keep the first table in the order `methods` enumerates."""
    best, best_s, n = None, -np.inf, 0
    for combo in itertools.product(methods, repeat=n_bounces):
        table = tuple(prefix) + combo + tuple(suffix)
        s = score(table)
        n += 1
        if s > best_s:
            best, best_s = table, s
    return best, best_s, n


def heuristic_search(n_bounces, t_d, methods, score, fallback):
    """Segmented search: bounces [1, t_d], (t_d, 2 t_d], ... are searched in turn by brute force,
    earlier segments fixed to their selected combination, later ones held at `fallback`.
    Returns (table, score of the table, number of tables scored)."""
    if t_d < 1:
        raise ValueError("segment length must be >= 1")
    chosen, total, best_s = (), 0, -np.inf
    for lo in range(0, n_bounces, t_d):
        width = min(t_d, n_bounces - lo)
        rest = (fallback,) * (n_bounces - lo - width)
        table, best_s, n = brute_force(width, methods, score, prefix=chosen, suffix=rest)
        chosen = table[:lo + width]
        total += n
    return chosen, best_s, total


def table_to_mask(table, method=NET):
    """Depth mask of one method in a table: bit d-1 set where bounce d uses `method`."""
    return sum(1 << d for d, m in enumerate(table) if m == method)


def relmse(img, ref):
    return float(np.mean((img - ref) ** 2 / (ref ** 2 + 0.01)))


def render_efficiency_scorer(renderer, max_depth, reference, mode_net, passes=1):
    """Score of a table: render `passes` passes (s_batch samples per pixel each) in NET mode with
    the table's network and fixed-rate depth masks; efficiency = 1 / (RelMSE of the luminance image against
    `reference` (RGB or luminance per pixel, e.g. the guide image: the running mean of the
    frames rendered so far) x GPU milliseconds of the render).

    Every table is rendered on the same random numbers (common random numbers: the pass index
    is set back to its value at the first call before each render), so two tables differ by what
    the table changes, not by independent sampling noise.  The accumulated image is reset and
    the guide image restored before each render, so every table starts from the same cache
    state; the caller's accumulated image is therefore lost (the search runs between training
    and the final render).  Afterwards the pass index is past the scored passes."""
    ref = np.asarray(reference, dtype=np.float64)
    if ref.size == 3 * renderer.width * renderer.height:
        ref = ref.reshape(-1, 3) @ LUM
    guide = renderer.get_guide()
    renderer.set_timing(True)
    first_pass = renderer.get_pass_index()

    def score(table):
        renderer.set_mix_depth(table_to_mask(table, NET))
        renderer.set_mix_depth_fixed(table_to_mask(table, FIXED))
        renderer.reset_image()
        renderer.set_guide(guide)
        renderer.set_pass_index(first_pass)
        st = renderer.render(renderer.s_batch * passes, max_depth, mode_net)
        img, _ = renderer.read_image()   # mean radiance of the render
        lum = img.reshape(-1, 3) @ LUM
        ms = sum(st["stage_ms"].values())
        return 1.0 / (max(relmse(lum, ref), 1e-30) * ms)

    return score
