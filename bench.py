"""Benchmark of the normalized-RRS wavefront path tracer on one MI355X.

A step is one NRRS frame over the 512x512 heightfield workload (about 1.05 M triangles,
16 spp traced as one 4.19 M-path wavefront, max depth 16): the full bounce loop
(camera, extend, shade, RRS network at depth <= 4, FP64 normalization, roulette/split
expansion, FP64 pixel accumulation, training-record capture) followed by one train_step
on 2^18 records.  `value` is rays extended per second (Mpaths/s) over the timed steps.

The network is first trained online for --train-frames frames (120 by default, whatever
--warmup is); the timed steps replay one captured hipGraph per pass (the library's default
launch path).  Also reported, outside the timed region: a per-stage breakdown from steps
with HIP events recorded on the render stream after every stage (direct launches), the
roofline of the dominant kernel from those events, the render efficiency 1/(relMSE * t) of
the trained network (NRRS), of NRRS with a searched Mix-Depth table (NRRS+) and of plain
heuristic normalized RRS at equal spp against a high-spp reference, the online-training
configuration (1024^2 room, 32 frames of 4 spp: trained vs untrained network vs heuristic),
the batched 1920x1080 configuration (5 M triangles, FP8 / BF16 / FP32 network), and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "render efficiency 1/(relMSE·s) + Mpaths/s, NRRS vs plain norm. RRS, 1 GPU"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK = 157.3   # TFLOP/s, MI355X published FP32 vector peak (packed FP32)
FP32_UNPACKED_PEAK = 78.6  # TFLOP/s without packed FP32 (256 CUs x 128 FLOP/clk x 2.4 GHz)
OPS_PER_NODE = 52          # two slab tests: 12 FMA (24 FLOP) + 28 min/max/compare/scale
OPS_PER_TRI = 56           # division-free Moller-Trumbore pre-test
LUM = np.array([0.2126, 0.7152, 0.0722])


def counted_traffic():
    """Bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, per kernel,
    kept only while the kernel's source file is the one the counters were taken on."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_extend_heightfield512_hbm_traffic.md")
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if not line.startswith("traffic: "):
            continue
        _, kernel, nbytes, src, digest = line.split()
        try:
            now = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()[:16]
        except OSError:
            continue
        if now == digest:
            out[kernel] = int(nbytes)
    return out


def counted_sq():
    """Vector-instruction counters per dispatch from the committed rocprofv3 SQ summary, per
    kernel, kept only while the kernel's source file is the one the counters were taken on."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_extend_heightfield512_sq_counters.md")
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if not line.startswith("sq: "):
            continue
        _, kernel, insts, active, thread_cycles, src, digest = line.split()
        try:
            now = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()[:16]
        except OSError:
            continue
        if now == digest:
            out[kernel] = (float(insts), float(active), float(thread_cycles))
    return out


def counted_mfma():
    """Matrix-core busy cycles, active cycles and vector instructions per dispatch from the
    committed rocprofv3 summary of the network kernel, kept only while its source file is the one
    the counters were taken on."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_rrsnet_mfma_heightfield512_mfma_counters.md")
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if not line.startswith("mfma: "):
            continue
        _, kernel, busy, gui, valu, src, digest = line.split()
        try:
            now = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()[:16]
        except OSError:
            continue
        if now == digest:
            out[kernel] = (float(busy), float(gui), float(valu))
    return out


def relmse(img, ref):
    return float(np.mean((img - ref) ** 2 / (ref ** 2 + 0.01)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--train-frames", type=int, default=120,
                    help="online-training frames (render + train_step) run before warmup, whatever --warmup is")
    ap.add_argument("--stage-steps", type=int, default=4,
                    help="extra steps with per-stage HIP events (direct launches) for the stage breakdown")
    ap.add_argument("--width", type=int, default=512)
    ap.add_argument("--spp", type=int, default=16)
    ap.add_argument("--depth", type=int, default=16)
    ap.add_argument("--ref-spp", type=int, default=2048)
    ap.add_argument("--eval-renders", type=int, default=8)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-eff", action="store_true")
    ap.add_argument("--no-room", action="store_true", help="skip the 1024^2 room online-training study")
    ap.add_argument("--no-batched", action="store_true", help="skip the 1920x1080 5 M-triangle batched render")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-nrrs", action="store_true", help="skip the NRRS-proper (StatNet + RRSNet) study")
    ap.add_argument("--nrrs-frames", type=int, default=120,
                    help="online-training frames of the NRRS-proper study (the first third in step 1)")
    ap.add_argument("--tuning", default=None,
                    help="traversal launch 'variant,blocks_per_cu,refill,leaf_batch,chunk' instead of autotuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the render is not sharded over "
              "several GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        copy_calibration(torch)
        return

    from paper_2510_07868_amd import nrrs, scenes

    prec = {"fp32": nrrs.PREC_FP32, "bf16": nrrs.PREC_BF16, "fp8": nrrs.PREC_FP8}[args.precision]
    W = H = args.width
    spp = args.spp
    D = args.depth
    nprim = W * H * spp
    rec_n = 1 << 18
    minibatch = 1 << 13
    p_train = min(1.0, 0.05 * (4194304 / nprim))
    t_scene = time.time()
    sc = scenes.heightfield(0)
    r = nrrs.Renderer(W, H, s_batch=spp, cap_factor=2.0, seed=0, net_max_depth=4, precision=prec,
                      records_cap=rec_n, p_train=p_train, max_tris=sc.n_tris, max_materials=len(sc.mat_type),
                      loss=nrrs.LOSS_REL_L2, ema_decay=0.99)
    r.upload_scene(sc)
    t_upload = time.time() - t_scene
    t_tune = time.time()
    if args.tuning:
        v, b, rf, lb, ch = (int(t) for t in args.tuning.split(","))
        r.set_tuning(v, b, rf, lb, ch)
        tuning, table = r.get_tuning(), []
    elif args.no_autotune:
        tuning, table = r.get_tuning(), []
    else:
        tuning, table = r.autotune(D, with_table=True)
    for t in table:
        print(f"#   candidate {t}", flush=True)
    print(f"# traversal launch {tuning} ({time.time() - t_tune:.1f}s)", flush=True)
    print(f"# scene {sc.n_tris} tris, setup+BVH {t_upload:.1f}s, workspace {r.workspace_bytes / 2**30:.2f} GiB",
          flush=True)

    def step():
        st = r.render(spp, D, nrrs.MODE_NET)
        n = min(st["records"], rec_n) // minibatch * minibatch
        loss = r.train_step(n, minibatch, 5e-3) if n > 0 else float("nan")
        return st, loss, n

    # online training of the network (one NET frame + one train_step per frame), then warmup
    t_train = time.perf_counter()
    for f in range(args.train_frames):
        st, loss, n = step()
        if f % 20 == 0 or f == args.train_frames - 1:
            print(f"# training frame {f}: rays {st['rays']}, records {st['records']}, loss {loss:.4f}", flush=True)
    t_train = time.perf_counter() - t_train
    for w in range(args.warmup):
        st, loss, n = step()
        print(f"# warmup {w}: rays {st['rays']}, records {st['records']}, loss {loss:.4f}", flush=True)

    # timed region: the product's default launch path (one captured hipGraph replayed per pass)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rays = 0
    for k in range(args.steps):
        st, loss, n = step()
        rays += st["rays"]
        print(f"# step {k}: rays {st['rays']}, loss {loss:.4f}, trained on {n}", flush=True)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    mpaths = rays / secs / 1e6

    # stage breakdown: the same steps with HIP events recorded on the render stream after every
    # stage (direct launches, since event-separated stages are not captured)
    r.set_timing(True)
    stage_ms = {k: 0.0 for k in nrrs.STAGES}
    stage_n = {k: 0 for k in nrrs.STAGES}
    nodes = tris = s_rays = 0
    net_rows = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.stage_steps):
        st, loss, n = step()
        net_rows += int(sum(st["n"][1:5]))
        s_rays += st["rays"]
        nodes += st["nodes_visited"]
        tris += st["tris_tested"]
        for s_ in nrrs.STAGES:
            stage_ms[s_] += st["stage_ms"][s_]
            stage_n[s_] += st["stage_launches"][s_]
    torch.cuda.synchronize()
    direct_secs = time.perf_counter() - t0
    r.set_timing(False)
    n_stage = max(args.stage_steps, 1)

    # roofline of the dominant kernel (traversal).  It is bound by vector-ALU issue (its BVH and
    # triangles stay cache-resident: the counted HBM traffic is a small fraction of the bytes it
    # reads), so it is measured in useful FP32 operations (FMA = 2): 52 per BVH node visited
    # (two ray/box slab tests) and 56 per triangle tested (Moller-Trumbore division-free test).
    dom = max(nrrs.STAGES, key=lambda s_: stage_ms[s_])
    ext_launches = max(stage_n["extend"], 1)
    ext_ms = stage_ms["extend"] / ext_launches
    ext_ops = (OPS_PER_NODE * nodes + OPS_PER_TRI * tris) / ext_launches
    ext_bytes = (64.0 * s_rays + 64.0 * nodes + 48.0 * tris) / ext_launches
    traffic = counted_traffic()
    v = tuning["extend_variant"]
    # the event-timed steps run the traversal variant that also counts nodes and triangles
    ext_kernel = "k_extend_immediate<true>" if v == 0 else f"k_extend<{v},true>"
    tb = traffic.get(ext_kernel)
    achieved = ext_ops / (ext_ms * 1e-3) / 1e12
    roofline = {"kernel": ext_kernel, "bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK, 4), "traffic": tb,
                "avg_launch_ms": round(ext_ms, 4), "algorithmic_ops_per_launch": int(ext_ops),
                "ops_per_node": OPS_PER_NODE, "ops_per_triangle": OPS_PER_TRI,
                "frac_of_unpacked_fp32_peak": round(achieved / FP32_UNPACKED_PEAK, 4),
                "nodes_per_ray": round(nodes / max(s_rays, 1), 2), "tris_per_ray": round(tris / max(s_rays, 1), 2),
                "grays_per_s": round(s_rays / (stage_ms["extend"] * 1e-3) / 1e9, 3),
                "node_and_triangle_bytes_gbs": round(ext_bytes / (ext_ms * 1e-3) / 1e9, 1),
                "hbm_gbs_counted": round(tb / (ext_ms * 1e-3) / 1e9, 1) if tb else None,
                "dominant_stage": dom, "timed_on": f"{args.stage_steps} event-timed steps after the timed region"}
    # vector-ALU issue: wave64 FP32 instructions take 4 cycles on one of 1024 SIMDs (256 CUs x 4)
    # at 2.4 GHz; lane use = active lanes per executed vector instruction (SQ counters)
    sq = counted_sq().get(ext_kernel)
    if sq:
        insts, active, thread_cycles = sq
        roofline["valu_issue_busy"] = round(insts * 4.0 / (1024 * 2.4e9 * ext_ms * 1e-3), 3)
        roofline["valu_lane_use"] = round(thread_cycles / (64.0 * active), 3)
    else:
        roofline["valu_issue_busy"] = roofline["valu_lane_use"] = None

    # the network stage: 19,072 useful FLOP per evaluated vertex (20-64-64-64-1)
    net_ms = stage_ms["network"] / max(stage_n["network"], 1)
    net_flop = 19072.0 * net_rows / max(stage_n["network"], 1)
    peak = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}[args.precision]
    network = {"kernel": "k_rrsnet_f32" if args.precision == "fp32" else f"k_rrsnet_mfma ({args.precision})",
               "bound": "alu" if args.precision == "fp32" else "mfma", "achieved": round(net_flop / (net_ms * 1e-3) / 1e12, 2),
               "peak": peak, "unit": "TFLOP/s", "frac": round(net_flop / (net_ms * 1e-3) / 1e12 / peak, 4),
               "avg_launch_ms": round(net_ms, 4), "rows_per_launch": int(net_rows / max(stage_n["network"], 1))}
    # matrix-core busy share and vector-issue share of the kernel's cycles (committed counters:
    # busy cycles summed over the 1024 SIMDs, active cycles summed over the 8 XCDs)
    mc = counted_mfma().get({"bf16": "k_rrsnet_mfma<1>", "fp8": "k_rrsnet_mfma<2>"}.get(args.precision, ""))
    if mc:
        busy, gui, valu = mc
        network["mfma_busy_share"] = round(busy / (gui / 8.0 * 1024.0), 3)
        network["valu_issue_share"] = round(valu * 4.0 / (gui / 8.0 * 1024.0), 3)
    else:
        network["mfma_busy_share"] = network["valu_issue_share"] = None

    # queue stages: counted HBM bytes per launch (rocprofv3, committed summary) over the live
    # per-launch stage time
    queue = {}
    for stage, kern in (("camera", "k_camera"), ("shade", "k_shade<false,false>"), ("expand", "k_expand")):
        ms = stage_ms[stage] / max(stage_n[stage], 1)
        b = traffic.get(kern)
        queue[kern] = {"avg_launch_ms": round(ms, 4), "hbm_bytes_per_launch": b,
                       "hbm_gbs": round(b / (ms * 1e-3) / 1e9, 1) if b else None,
                       "frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if b else None}
    for stage, kerns in (("sum_q", ("k_sum_q_partial", "k_sum_q_final")),
                         ("roulette_scan", ("k_roulette_count", "k_roulette_scan", "k_guard_count",
                                            "k_guard_select", "k_offsets"))):
        ms = stage_ms[stage] / max(stage_n[stage], 1)
        b = [traffic.get(k) for k in kerns]
        tot = sum(x for x in b if x) if any(b) else None
        queue["+".join(kerns)] = {"avg_launch_ms": round(ms, 4), "hbm_bytes_per_launch": tot,
                                  "hbm_gbs": round(tot / (ms * 1e-3) / 1e9, 1) if tot else None,
                                  "frac": round(tot / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if tot else None}

    out = {
        "metric": METRIC, "value": round(mpaths, 2), "unit": "Mpaths/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(secs / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == nrrs.PREC_FP32 else f"f32 (network {args.precision})",
        "data": "synthetic",
        "config": {"workload": f"heightfield {sc.n_tris} tris, {W}x{H}, {spp} spp in one {nprim}-path wavefront, "
                               f"max depth {D}, NRRS (network at depth<=4) + train_step(2^18 records)",
                   "width": W, "height": H, "spp": spp, "max_depth": D, "triangles": sc.n_tris,
                   "queue_capacity": 2 * nprim, "parallelism": "single GPU",
                   "launch": "one captured hipGraph per pass, replayed"},
        "training": {"frames": args.train_frames, "seconds": round(t_train, 2), "p_train": p_train,
                     "records_per_frame": rec_n, "minibatch": minibatch, "lr": 5e-3, "loss": "relative L2",
                     "ema_decay": 0.99},
        "direct_launch_ms_per_step": round(direct_secs / n_stage * 1e3, 3),
        "stage_ms_per_step": {s_: round(stage_ms[s_] / n_stage, 3) for s_ in nrrs.STAGES},
        "roofline": roofline,
        "network": network,
        "queue_stages": queue,
        "autotuned": None if (args.no_autotune or args.tuning) else tuning,
    }

    if not args.no_eff:
        def make_reference(ref_spp):
            rr = nrrs.Renderer(W, H, s_batch=spp, cap_factor=2.0, seed=0x5EED5EED, max_tris=sc.n_tris,
                               max_materials=len(sc.mat_type))
            rr.upload_scene(sc)
            rr.render(ref_spp, D, nrrs.MODE_OFF, stats=False)
            img, _ = rr.read_image()
            rr.close()
            return img
        refs = {}

        def reference_once(ref_spp):
            if ref_spp not in refs:
                refs[ref_spp] = make_reference(ref_spp)
            return refs[ref_spp]
        out["efficiency"] = efficiency(r, nrrs, spp, D, args.ref_spp, args.eval_renders, reference_once)
        out["efficiency"]["trained_frames"] = args.train_frames
    r.close()
    del r
    torch.cuda.empty_cache()
    if not args.no_eff:
        out["log_loss_network"] = log_loss_study(nrrs, sc, torch, W, H, spp, D, prec, args.train_frames,
                                                 args.eval_renders, reference_once(args.ref_spp), p_train, tuning,
                                                 out["efficiency"]["heuristic"]["efficiency"])
        torch.cuda.empty_cache()
    if not args.no_eff and not args.no_nrrs:
        out["nrrs_proper"] = nrrs_proper_study(nrrs, sc, torch, W, H, spp, D, args.nrrs_frames, args.eval_renders,
                                               reference_once(args.ref_spp), p_train, tuning)
        out["nrrs_proper"]["over_heuristic_in_the_efficiency_study"] = (
            out["nrrs_proper"]["nrrs"]["efficiency"] / out["efficiency"]["heuristic"]["efficiency"])
        torch.cuda.empty_cache()
    if not args.no_room:
        out["room_online_training"] = room_study(nrrs, scenes, torch)
    if not args.no_batched:
        out["batched_1080p"] = batched_study(nrrs, scenes, torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sc, W, H, D)
    print(json.dumps(out), flush=True)


def efficiency(r, nrrs, spp, D, ref_spp, renders, make_reference):
    """relMSE and 1/(relMSE * t) at equal spp of NRRS, NRRS with a Mix-Depth table found by the
    segmented search (NRRS+, Sec. 4.3) and heuristic normalized RRS."""
    import torch
    from paper_2510_07868_amd import mixdepth

    res = {}
    guide = r.get_guide()
    default = r.get_mix_depth()
    # Mix-Depth search: one timed pass per table, scored against the guide image (the running
    # mean of the training frames); segments of 5 bounces over the D - 1 that take a decision,
    # the bounces after the segment being searched held at the fixed rate
    t0 = time.perf_counter()
    score = mixdepth.render_efficiency_scorer(r, D, guide, nrrs.MODE_NET)
    table, _, n_tables = mixdepth.heuristic_search(D - 1, 5, mixdepth.METHODS, score, fallback=mixdepth.FIXED)
    t_search = time.perf_counter() - t0
    plus = (mixdepth.table_to_mask(table, mixdepth.NET), mixdepth.table_to_mask(table, mixdepth.FIXED))
    for name, mode, (mask, fixed) in (("nrrs", nrrs.MODE_NET, (default, 0)), ("nrrs_plus", nrrs.MODE_NET, plus),
                                      ("heuristic", nrrs.MODE_HEURISTIC, (default, 0))):
        r.set_mix_depth(mask)
        r.set_mix_depth_fixed(fixed)
        times, imgs = [], []
        for k in range(renders):
            r.set_guide(guide)          # every evaluation render sees the same previous frame
            r.reset_image()             # the pass counter keeps counting: fresh random numbers
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.render(spp, D, mode, stats=False)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            img, _ = r.read_image()
            imgs.append(img)
        res[name] = {"times": times, "imgs": imgs}
    r.set_guide(guide)
    r.set_mix_depth(default)
    r.set_mix_depth_fixed(0)
    # reference: plain path tracing with an independent seed (no random stream shared with the
    # evaluation renders)
    t0 = time.perf_counter()
    ref = make_reference(ref_spp)
    t_ref = time.perf_counter() - t0
    out = {"reference": f"plain path tracing, {ref_spp} spp, same depth, independent seed",
           "reference_s": round(t_ref, 2), "spp": spp, "renders": renders}
    for name, d in res.items():
        errs = [relmse(i, ref) for i in d["imgs"]]
        rm = float(np.mean(errs))
        t = float(np.median(d["times"]))
        out[name] = {"relmse": rm, "relmse_se": float(np.std(errs) / np.sqrt(len(errs))), "render_s": round(t, 5),
                     "efficiency": 1.0 / (rm * t)}
    out["nrrs_over_heuristic"] = out["nrrs"]["efficiency"] / out["heuristic"]["efficiency"]
    out["nrrs_plus_over_heuristic"] = out["nrrs_plus"]["efficiency"] / out["heuristic"]["efficiency"]
    out["mix_depth"] = {"search": "segmented, T_d = 5, methods network / heuristic / fixed rate",
                        "tables": n_tables, "search_s": round(t_search, 2),
                        "network_depths": [d + 1 for d, m in enumerate(table) if m == mixdepth.NET],
                        "fixed_rate_depths": [d + 1 for d, m in enumerate(table) if m == mixdepth.FIXED]}
    return out


def log_loss_study(nrrs, sc, torch, W, H, spp, D, prec, frames, renders, ref, p_train, tuning, heuristic_eff):
    """The same network, schedule and evaluation as the efficiency study, trained with the squared
    error of log radiance (the online-training configuration's loss) instead of the relative L2
    of Eq. (15): relMSE, render time and efficiency over the heuristic of the efficiency study."""
    rec_n, minibatch = 1 << 18, 1 << 13
    r = nrrs.Renderer(W, H, s_batch=spp, cap_factor=2.0, seed=0, net_max_depth=4, precision=prec,
                      records_cap=rec_n, p_train=p_train, max_tris=sc.n_tris, max_materials=len(sc.mat_type),
                      loss=nrrs.LOSS_LOG_MSE, ema_decay=0.99)
    r.upload_scene(sc)
    r.set_tuning(tuning["extend_variant"], tuning["extend_blocks_per_cu"], tuning["extend_refill"],
                 tuning["extend_leaf_batch"], tuning["extend_chunk"])
    for f in range(frames):
        st = r.render(spp, D, nrrs.MODE_NET)
        n = min(st["records"], rec_n) // minibatch * minibatch
        if n > 0:
            r.train_step(n, minibatch, 5e-3)
    guide = r.get_guide()
    times, errs = [], []
    for k in range(renders):
        r.set_guide(guide)
        r.reset_image()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.render(spp, D, nrrs.MODE_NET, stats=False)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        img, _ = r.read_image()
        errs.append(relmse(img, ref))
    r.close()
    rm, t = float(np.mean(errs)), float(np.median(times))
    eff = 1.0 / (rm * t)
    print(f"# log-loss network: relMSE {rm:.4f}, {t * 1e3:.2f} ms, {eff / heuristic_eff:.3f}x heuristic", flush=True)
    return {"loss": "squared error of log radiance", "trained_frames": frames, "relmse": rm,
            "relmse_se": float(np.std(errs) / np.sqrt(len(errs))), "render_s": round(t, 5), "efficiency": eff,
            "over_heuristic": eff / heuristic_eff}


def nrrs_proper_study(nrrs, sc, torch, W, H, spp, D, frames, renders, ref, p_train, tuning):
    """NRRS proper (Sec. 4.2): StatNet + RRSNet (NRRS inputs) and the AID-NRRS RRSNet, both trained
    online for `frames` frames (render + one train_step_nrrs each, both RRSNets per step; fitted
    to 1 for the first third, then by the pixel-variance loss of Eq. 16), then relMSE and
    1/(relMSE * t) at equal spp against heuristic normalized RRS on the same context, guide and
    reference: each with the factor at depths 1-4, and with the per-bounce table found by the
    segmented Mix-Depth search (Sec. 4.3) over {the factor, heuristic, fixed rate}."""
    from paper_2510_07868_amd import mixdepth

    rec_n = 1 << 18
    r = nrrs.Renderer(W, H, s_batch=spp, cap_factor=2.0, seed=0, net_max_depth=4, records_cap=rec_n,
                      p_train=p_train, max_tris=sc.n_tris, max_materials=len(sc.mat_type), ema_decay=0.99,
                      hash_log2=19)
    r.upload_scene(sc)
    if tuning:
        r.set_tuning(tuning["extend_variant"], tuning["extend_blocks_per_cu"], tuning["extend_refill"],
                     tuning["extend_leaf_batch"], tuning["extend_chunk"])
    step1 = max(1, frames // 3)
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_train = 0.0
    for f in range(frames):
        # frames alternate the two factors so that both RRSNets see their own renders' records
        st = r.render(spp, D, nrrs.MODE_NRRS if f % 2 == 0 else nrrs.MODE_AID)
        n = min(st["records"], rec_n)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lo = r.train_step_nrrs(n, 1 if f < step1 else 2, variant=2)
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t1
        if f % 20 == 0 or f == frames - 1:
            print(f"# nrrs frame {f}: records {n}, StatNet loss {lo['loss_stat']:.4f}, "
                  f"RRSNet loss {lo['loss_rrs']:.4g}, E_avg {lo['e_avg']:.4g}", flush=True)
            hist.append({"frame": f, "loss_stat": lo["loss_stat"], "loss_rrs": lo["loss_rrs"], "e_avg": lo["e_avg"]})
    t_frames = time.perf_counter() - t0
    guide = r.get_guide()
    default = r.get_mix_depth()
    tables = {}
    t0 = time.perf_counter()
    for name, mode in (("nrrs", nrrs.MODE_NRRS), ("aid", nrrs.MODE_AID)):
        score = mixdepth.render_efficiency_scorer(r, D, guide, mode)
        table, _, _ = mixdepth.heuristic_search(D - 1, 5, mixdepth.METHODS, score, fallback=mixdepth.FIXED)
        tables[name] = (mixdepth.table_to_mask(table, mixdepth.NET), mixdepth.table_to_mask(table, mixdepth.FIXED))
    t_search = time.perf_counter() - t0
    res = {}
    for name, mode, (mask, fixed) in (("nrrs", nrrs.MODE_NRRS, (default, 0)), ("nrrs_plus", nrrs.MODE_NRRS, tables["nrrs"]),
                                      ("aid", nrrs.MODE_AID, (default, 0)), ("aid_plus", nrrs.MODE_AID, tables["aid"]),
                                      ("heuristic", nrrs.MODE_HEURISTIC, (default, 0))):
        r.set_mix_depth(mask)
        r.set_mix_depth_fixed(fixed)
        times, errs = [], []
        for k in range(renders):
            r.set_guide(guide)
            r.reset_image()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.render(spp, D, mode, stats=False)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            img, _ = r.read_image()
            errs.append(relmse(img, ref))
        rm, t = float(np.mean(errs)), float(np.median(times))
        res[name] = {"relmse": rm, "relmse_se": float(np.std(errs) / np.sqrt(len(errs))), "render_s": round(t, 5),
                     "efficiency": 1.0 / (rm * t)}
        if mask != default or fixed:
            res[name]["factor_depths"] = [d + 1 for d in range(64) if (mask >> d) & 1 and not (fixed >> d) & 1]
            res[name]["fixed_rate_depths"] = [d + 1 for d in range(64) if (fixed >> d) & 1]
    r.set_mix_depth(default)
    r.set_mix_depth_fixed(0)
    # per-stage time of an NRRS render (the factor kernel is the network stage)
    r.set_timing(True)
    r.set_guide(guide)
    st = r.render(spp, D, nrrs.MODE_NRRS)
    r.set_timing(False)
    r.close()
    out = {"method": "StatNet (hash grid 8 x 2, 2^19 entries per level) + RRSNet with NRRS inputs, and the AID-NRRS "
                     "RRSNet (its own hash grid + one-blob inputs); 32-wide 3-hidden-layer MLPs, FP32; one Adam step "
                     "per frame (lr 5e-3 / 3e-4), gammas 0.01 / 0.05 / 0.01, error image mixed 0.5 and box-filtered "
                     "(radius 2)",
           "frames": frames, "step1_frames": step1, "train_s": round(t_frames, 2),
           "train_step_ms": round(1e3 * t_train / frames, 3), "mix_depth_search_s": round(t_search, 2),
           "history": hist, "stage_ms_nrrs": {k: round(v, 3) for k, v in st["stage_ms"].items()}}
    out.update(res)
    for k in ("nrrs", "nrrs_plus", "aid", "aid_plus"):
        out[f"{k}_over_heuristic"] = res[k]["efficiency"] / res["heuristic"]["efficiency"]
    return out


def _timed_render(r, torch, spp, D, mode, train=None):
    """One frame: render (+ one train_step when `train` = (records cap, minibatch, lr)); wall
    time with the stream drained on both sides."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = r.render(spp, D, mode)
    if train is not None:
        cap, mb, lr = train
        n = min(st["records"], cap) // mb * mb
        if n > 0:
            r.train_step(n, mb, lr)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, st


def _reference(nrrs, sc, W, H, s_batch, D, ref_spp, seed):
    """Plain path tracing (no roulette) with an independent seed, as two halves: their mean is the
    reference and their difference estimates the reference's own noise."""
    halves = []
    for k in range(2):
        rr = nrrs.Renderer(W, H, s_batch=s_batch, cap_factor=2.0, seed=seed + k, max_tris=sc.n_tris,
                           max_materials=len(sc.mat_type))
        rr.upload_scene(sc)
        rr.render(ref_spp // 2, D, nrrs.MODE_OFF, stats=False)
        img, _ = rr.read_image()
        rr.close()
        halves.append(img)
    return 0.5 * (halves[0] + halves[1]), 0.25 * (halves[0] - halves[1]) ** 2


def _relmse_pair(img, ref, ref_var):
    """relMSE against the reference, and the same with the reference's estimated variance taken out."""
    den = ref ** 2 + 0.01
    return float(np.mean((img - ref) ** 2 / den)), float(np.mean(((img - ref) ** 2 - ref_var) / den))


def room_study(nrrs, scenes, torch, frames=32, trials=3, ref_spp=1024):
    """The online-training configuration: 1024x1024 room (~2.1 M triangles) lit only through a
    0.5 m^2 ceiling opening, depth 24, 32 frames of 4 spp.  NRRS ("trained"): every NET frame is
    followed by one train_step on 2^18 records (minibatches of 2^13, BF16 inference, FP32
    masters).  "untrained": the same NET frames with the initial weights and no training.
    "heuristic": plain normalized RRS.  The image is the mean of the 32 frames (128 spp); time is
    render + training; efficiency = 1 / (relMSE * time).  Each method runs `trials` times on
    fresh random numbers, from the initial weights and no pixel estimate."""
    W = H = 1024
    spp, D = 4, 24
    rec_n, mb, lr = 1 << 18, 1 << 13, 5e-3
    t_setup = time.perf_counter()
    sc = scenes.room(0)
    r = nrrs.Renderer(W, H, s_batch=spp, cap_factor=2.0, seed=0, net_max_depth=4, precision=nrrs.PREC_BF16,
                      records_cap=rec_n, p_train=0.05, max_tris=sc.n_tris, max_materials=len(sc.mat_type),
                      loss=nrrs.LOSS_REL_L2, ema_decay=0.99)
    r.upload_scene(sc)
    tuning = r.autotune(D)
    t_setup = time.perf_counter() - t_setup
    w0, m0, v0, _ = r.get_params()
    none = np.full(W * H, -1.0, np.float32)
    res = {k: {"relmse": [], "relmse_ref_noise_removed": [], "seconds": [], "rays": []}
           for k in ("trained", "untrained", "heuristic")}
    imgs = {}
    for trial in range(trials):
        for name, mode, train in (("trained", nrrs.MODE_NET, (rec_n, mb, lr)), ("untrained", nrrs.MODE_NET, None),
                                  ("heuristic", nrrs.MODE_HEURISTIC, None)):
            r.set_params(w0, m0, v0, 0)
            r.set_state(infer=w0, alpha=1.0)
            r.set_guide(none)
            r.reset_image()
            secs = 0.0
            rays = 0
            for f in range(frames):
                dt, st = _timed_render(r, torch, spp, D, mode, train)
                secs += dt
                rays += st["rays"]
            img, n = r.read_image()
            imgs.setdefault(name, []).append(img)
            res[name]["seconds"].append(secs)
            res[name]["rays"].append(rays)
            print(f"# room trial {trial} {name}: {secs:.2f}s, {rays / secs / 1e6:.0f} Mpaths/s", flush=True)
    r.close()
    t_ref = time.perf_counter()
    ref, ref_var = _reference(nrrs, sc, W, H, 16, D, ref_spp, 0x5EED0000)
    t_ref = time.perf_counter() - t_ref
    out = {"workload": f"room {sc.n_tris} tris, {W}x{H}, {frames} frames x {spp} spp, max depth {D}",
           "reference": f"plain path tracing, {ref_spp} spp in two independent halves",
           "reference_s": round(t_ref, 1), "setup_s": round(t_setup, 1), "trials": trials,
           "traversal_launch": tuning}
    for name, d in res.items():
        for img in imgs[name]:
            a, b = _relmse_pair(img, ref, ref_var)
            d["relmse"].append(a)
            d["relmse_ref_noise_removed"].append(b)
        rm, rm_c, t = (float(np.mean(d[k])) for k in ("relmse", "relmse_ref_noise_removed", "seconds"))
        out[name] = {"relmse": rm, "relmse_se": float(np.std(d["relmse"]) / np.sqrt(trials)),
                     "relmse_ref_noise_removed": rm_c, "seconds": round(t, 3),
                     "mpaths_per_s": round(float(np.sum(d["rays"]) / np.sum(d["seconds"]) / 1e6), 1),
                     "efficiency": 1.0 / (rm * t)}
    out["trained_over_heuristic"] = out["trained"]["efficiency"] / out["heuristic"]["efficiency"]
    out["untrained_over_heuristic"] = out["untrained"]["efficiency"] / out["heuristic"]["efficiency"]
    out["trained_over_untrained"] = out["trained"]["efficiency"] / out["untrained"]["efficiency"]
    return out


def batched_study(nrrs, scenes, torch, spp=64, s_batch=8, D=32, train_frames=48, ref_spp=512):
    """The batched configuration: 1920x1080, ~5.0 M triangles (heightfield + 2000 boxes), depth
    32, 64 spp in passes of 8 spp (16.6 M-path wavefronts), one captured hipGraph per pass,
    autotuned traversal.  The network trains online for `train_frames` 8-spp frames, then the
    64-spp render runs with its FP8, BF16 and FP32 inference (same weights and pixel estimate)
    and with heuristic normalized RRS: time, Mpaths/s and relMSE against plain path tracing."""
    W, H = 1920, 1080
    rec_n, mb, lr = 1 << 18, 1 << 13, 5e-3
    t_setup = time.perf_counter()
    sc = scenes.terrain5m(0)
    r = nrrs.Renderer(W, H, s_batch=s_batch, cap_factor=2.0, seed=0, net_max_depth=4, precision=nrrs.PREC_FP8,
                      records_cap=rec_n, p_train=0.05 * 4194304 / (W * H * s_batch), max_tris=sc.n_tris,
                      max_materials=len(sc.mat_type), loss=nrrs.LOSS_REL_L2, ema_decay=0.99)
    r.upload_scene(sc)
    tuning = r.autotune(D)
    t_setup = time.perf_counter() - t_setup
    t_train = time.perf_counter()
    for f in range(train_frames):
        _timed_render(r, torch, s_batch, D, nrrs.MODE_NET, (rec_n, mb, lr))
    t_train = time.perf_counter() - t_train
    guide = r.get_guide()
    out = {"workload": f"terrain {sc.n_tris} tris, {W}x{H}, {spp} spp in passes of {s_batch} spp "
                       f"({W * H * s_batch}-path wavefronts), max depth {D}",
           "setup_s": round(t_setup, 1), "training_frames": train_frames, "training_s": round(t_train, 2),
           "traversal_launch": tuning}
    imgs = {}
    for name, mode, prec in (("fp8", nrrs.MODE_NET, nrrs.PREC_FP8), ("bf16", nrrs.MODE_NET, nrrs.PREC_BF16),
                             ("fp32", nrrs.MODE_NET, nrrs.PREC_FP32), ("heuristic", nrrs.MODE_HEURISTIC, None)):
        if prec is not None:
            r.set_precision(prec)
        r.set_guide(guide)
        r.reset_image()
        r.render(s_batch, D, mode, stats=False)   # capture this configuration's pass graph
        r.reset_image()
        dt, st = _timed_render(r, torch, spp, D, mode)
        img, n = r.read_image()
        imgs[name] = img
        out[name] = {"seconds": round(dt, 4), "mpaths_per_s": round(st["rays"] / dt / 1e6, 1), "rays": st["rays"]}
        print(f"# batched {name}: {dt:.3f}s, {st['rays'] / dt / 1e6:.0f} Mpaths/s", flush=True)
    r.close()
    # the same scene with its 2000 boxes as instances of one unit box (two-level traversal),
    # heuristic normalized RRS over the same 64 spp
    isc = scenes.terrain5m_instanced(0)
    ri = nrrs.Renderer(W, H, s_batch=s_batch, cap_factor=2.0, seed=0, max_tris=isc.workspace_tris,
                       max_materials=len(isc.base.mat_type))
    ri.upload_scene(isc)
    tuning_i = ri.autotune(D)
    ri.render(s_batch, D, nrrs.MODE_HEURISTIC, stats=False)
    ri.reset_image()
    dt, st = _timed_render(ri, torch, spp, D, nrrs.MODE_HEURISTIC)
    imgs["instanced_heuristic"], _ = ri.read_image()
    ri.close()
    out["instanced_heuristic"] = {"seconds": round(dt, 4), "mpaths_per_s": round(st["rays"] / dt / 1e6, 1),
                                  "rays": st["rays"], "traversal_launch": tuning_i,
                                  "triangles_stored": int(isc.base.n_tris + isc.mesh_tris.shape[0]),
                                  "instances": int(isc.inst_mesh.shape[0])}
    print(f"# batched instanced heuristic: {dt:.3f}s, {st['rays'] / dt / 1e6:.0f} Mpaths/s", flush=True)
    t_ref = time.perf_counter()
    ref, ref_var = _reference(nrrs, sc, W, H, s_batch, D, ref_spp, 0x5EED1000)
    out["reference"] = f"plain path tracing, {ref_spp} spp in two independent halves"
    out["reference_s"] = round(time.perf_counter() - t_ref, 1)
    for name, img in imgs.items():
        a, b = _relmse_pair(img, ref, ref_var)
        out[name]["relmse"] = a
        out[name]["relmse_ref_noise_removed"] = b
        out[name]["efficiency"] = 1.0 / (a * out[name]["seconds"])
    for name in ("fp8", "bf16", "fp32"):
        out[f"{name}_over_heuristic"] = out[name]["efficiency"] / out["heuristic"]["efficiency"]
    out["instanced_time_over_flat"] = out["instanced_heuristic"]["seconds"] / out["heuristic"]["seconds"]
    return out


def copy_calibration(torch):
    """A plain device copy of known size: 1 GiB read + 1 GiB written per launch, five launches."""
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n, "launches": 5}))


def cpu_baseline(sc, W, H, D, passes=16):
    import oracle

    osc = oracle.OracleScene(sc)
    cfg = oracle.make_cfg(W, H, 1, D, n_passes=passes, mode=oracle.MODE_HEUR, tau=0.0)
    t0 = time.perf_counter()
    o = oracle.render(osc, cfg)
    secs = time.perf_counter() - t0
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(o["rays"] / secs / 1e6, 3), "unit": "Mpaths/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": round(secs, 2), "cpu_model": cpu,
            "sample": f"{passes} spp of the same {W}x{H} heightfield workload ({passes} passes of one {W * H}-path "
                      f"wavefront, max depth {D}, heuristic normalized RRS), FP64 C oracle with OpenMP; BVH build "
                      "excluded"}


if __name__ == "__main__":
    main()
