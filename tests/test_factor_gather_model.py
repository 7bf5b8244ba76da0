"""CPU model of how the NRRS factor kernel hands queue entries to its 64-vertex groups.

Each wave walks its strided share of the queue in chunks of 64 entries, appends the entries
that take the learned factor (q > 0 and a pixel with history) to a 128-slot list in LDS,
computes the first 64 listed entries as one group once 64 are listed (or its share is used up),
and moves the rest to the front of the list.  The model replays that arithmetic step for step
and checks, over random live masks, queue sizes and grid shapes (empty, ragged, one live entry,
all live), that every list slot written or read is below 128, that every live entry is computed
exactly once and no other entry at all, and that every group but a wave's last is full.
"""
import numpy as np
import pytest

LIST = 128


def _wave(take, n, first_group, waves):
    """Entries computed by one wave, group by group, following the kernel's loop."""
    groups = (n + 63) // 64
    buf = [None] * LIST
    cnt, gi, out = 0, first_group, []
    while True:
        while cnt < 64 and gi < groups:
            live = [j for j in range(gi * 64, gi * 64 + 64) if j < n and take[j]]
            for r, j in enumerate(live):  # lane's rank among the live lanes of the chunk
                slot = cnt + r
                assert slot < LIST, (cnt, r)
                buf[slot] = j
            cnt += len(live)
            gi += waves
        if cnt == 0:
            return out
        assert cnt < LIST
        group = [buf[lane] for lane in range(64) if lane < cnt]
        rest = [buf[lane + 64] for lane in range(64) if lane + 64 < cnt]
        for lane, v in enumerate(rest):
            buf[lane] = v
        cnt = cnt - 64 if cnt > 64 else 0
        out.append(group)


@pytest.mark.parametrize("n,p_live,waves", [(0, 0.5, 4), (1, 1.0, 4), (63, 0.3, 1), (64, 1.0, 2), (65, 0.5, 8),
                                            (1000, 0.0, 8), (4099, 0.43, 8), (20000, 0.7, 20), (20000, 1.0, 7),
                                            (20000, 0.02, 3), (777, 0.97, 1000)])
def test_every_live_entry_is_computed_once(n, p_live, waves):
    rng = np.random.default_rng(n * 31 + waves)
    take = rng.random(n) < p_live
    if n > 200:  # dead runs as long as whole chunks, as the sky rows give at the first bounce
        take[64:200] = False
    seen = np.zeros(n, np.int64)
    for w in range(waves):
        groups = _wave(take, n, w, waves)
        for k, g in enumerate(groups):
            assert 1 <= len(g) <= 64
            if k + 1 < len(groups):
                assert len(g) == 64  # a wave computes partial groups only at the end of its share
            for j in g:
                seen[j] += 1
    assert np.array_equal(seen, take.astype(np.int64))
