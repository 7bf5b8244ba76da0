"""The allocation-free variant of the roulette / scan / parent-map step against the entry point
it varies (nrrs_debug_rrs_expand, workspace scratch): same kernels, same inputs, so every output
is bit-exact.  Two calls in a row, the second on a smaller input, then one that overflows."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_rrs_expand_noalloc_matches_the_workspace_entry_point(scenes):
    import torch
    from paper_2510_07868_amd import nrrs
    nrrs.load()
    sc = scenes.cornell()
    r = nrrs.Renderer(256, 256, s_batch=2, max_tris=64, max_materials=4)
    r.upload_scene(sc)
    dev = r.device
    rng = np.random.default_rng(3)
    for n, cap_frac, alpha, depth in ((100000, 2.0, 1.0, 3), (4099, 2.0, 0.7, 5), (777, 0.5, 1.0, 2), (500, 0.0, 1.0, 4)):
        print(f"noalloc n={n} cap={cap_frac} alpha={alpha}", flush=True)
        q = rng.lognormal(0.0, 1.0, size=n).astype(np.float32)
        lo = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
        hi = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
        budget = float(n)
        cap = int(cap_frac * budget)
        ref = r.debug_rrs_expand(q, lo, hi, depth, budget, alpha=alpha, cap=cap)
        q_t = torch.from_numpy(q).to(dev)
        lin_t = torch.from_numpy(np.stack([lo, hi], 1).view(np.int32).copy()).to(dev)
        off_t = torch.full((n,), -1, dtype=torch.int32, device=dev)
        par_t = torch.full((cap,), -1, dtype=torch.int32, device=dev)
        res_t = torch.zeros(32, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        r.rrs_expand_noalloc(q_t, lin_t, off_t, res_t, depth, budget, alpha=alpha, cap=cap, parent=par_t)
        r.stream.synchronize()
        res = nrrs.Renderer.decode_expand_result(res_t.cpu().numpy())
        assert res["retries"] == ref["retries"] and res["alpha"] == ref["alpha"]
        if ref["status"] != 0:
            assert res["overflow"] == 1 and res["S"] == 0
            continue
        assert res["overflow"] == 0 and res["S"] == ref["S"] and res["F"] == ref["F"]
        off = off_t.cpu().numpy().view(np.uint32)
        assert np.array_equal(off, ref["offset"])
        X = np.diff(np.append(off.astype(np.int64), res["S"]))
        assert np.array_equal(X, ref["X"].astype(np.int64))
        assert np.array_equal(par_t.cpu().numpy()[: res["S"]].view(np.uint32), ref["parent"])
    r.close()
