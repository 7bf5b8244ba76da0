"""Thin ctypes binding of libnrrs.so (the C ABI of include/nrrs.h).

Argument marshalling only: every step of the render and of training runs in the
library's HIP kernels.  PyTorch provides the device workspace (one uint8 tensor) and
the HIP stream.  Importing this module does not touch the GPU; creating a Renderer
raises if the library is not built or no gfx950 device is present.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnrrs.so")
NPARAM = 9729
MAX_DEPTH = 64
MODE_OFF, MODE_HEURISTIC, MODE_NET, MODE_NRRS, MODE_AID = 0, 1, 2, 3, 4
STAT_NPARAM, RRS_NPARAM, AID_NPARAM = 3234, 2401, 3201
HG_LEVELS, HG_FEAT = 8, 2
NORM_TWO_SIDED, NORM_DOWNSCALE = 0, 1
PREC_FP32, PREC_BF16, PREC_FP8 = 0, 1, 2
LOSS_REL_L2, LOSS_LOG_MSE = 0, 1
MISS = 0xFFFFFFFF
NSTAGES = 8
STAGES = ["camera", "extend", "shade", "network", "sum_q", "roulette_scan", "expand", "pass_end"]

EXPORTS = [
    "nrrs_create", "nrrs_workspace_size", "nrrs_bind_workspace", "nrrs_upload_scene",
    "nrrs_upload_scene_instanced", "nrrs_render",
    "nrrs_set_timing", "nrrs_set_launch_mode", "nrrs_set_precision", "nrrs_set_mix_depth", "nrrs_get_mix_depth",
    "nrrs_set_mix_depth_fixed", "nrrs_get_mix_depth_fixed",
    "nrrs_set_pass_index", "nrrs_get_pass_index", "nrrs_get_tuning", "nrrs_set_tuning", "nrrs_autotune",
    "nrrs_train_step", "nrrs_read_image", "nrrs_reset_image", "nrrs_set_guide", "nrrs_get_guide",
    "nrrs_get_params", "nrrs_set_params", "nrrs_get_state", "nrrs_set_state", "nrrs_set_trace",
    "nrrs_read_trace", "nrrs_read_records", "nrrs_debug_rrs_expand", "nrrs_rrs_expand_noalloc",
    "nrrs_debug_set_norm_factors", "nrrs_debug_load_records", "nrrs_debug_read_queue", "nrrs_debug_trace",
    "nrrs_debug_philox", "nrrs_debug_mlp_forward", "nrrs_debug_mlp_codes", "nrrs_debug_mlp_grad",
    "nrrs_set_nrrs_params", "nrrs_get_nrrs_params", "nrrs_train_step_nrrs", "nrrs_debug_nrrs_forward",
    "nrrs_debug_nrrs_grads", "nrrs_debug_pixel_error", "nrrs_set_aid_params", "nrrs_get_aid_params",
    "nrrs_debug_aid_forward", "nrrs_debug_aid_grads", "nrrs_status_string",
    "nrrs_last_error", "nrrs_destroy",
]


class Tuning(C.Structure):
    _fields_ = [
        ("extend_variant", C.c_uint32), ("extend_blocks_per_cu", C.c_uint32), ("extend_refill", C.c_uint32),
        ("extend_leaf_batch", C.c_uint32), ("extend_chunk", C.c_uint32),
        ("extend_max_blocks_per_cu", C.c_uint32 * 5), ("extend_ms", C.c_float),
    ]

    def as_dict(self):
        return {"extend_variant": self.extend_variant, "extend_blocks_per_cu": self.extend_blocks_per_cu,
                "extend_refill": self.extend_refill, "extend_leaf_batch": self.extend_leaf_batch,
                "extend_chunk": self.extend_chunk,
                "extend_max_blocks_per_cu": list(self.extend_max_blocks_per_cu),
                "extend_ms": round(float(self.extend_ms), 4)}


class Config(C.Structure):
    _fields_ = [
        ("width", C.c_uint32), ("height", C.c_uint32), ("s_batch", C.c_uint32),
        ("cap_factor", C.c_double), ("f_rate", C.c_double), ("norm_mode", C.c_int32), ("seed", C.c_uint64),
        ("net_max_depth", C.c_int32), ("precision", C.c_int32), ("records_cap", C.c_uint32),
        ("p_train", C.c_double), ("loss", C.c_int32), ("ema_decay", C.c_double), ("trace_depth", C.c_uint32),
        ("hash_log2", C.c_uint32), ("nee", C.c_uint32),
    ]


class NrrsTrain(C.Structure):
    _fields_ = [
        ("lr_stat", C.c_float), ("lr_rrs", C.c_float), ("g_avg", C.c_float), ("g_min", C.c_float),
        ("g_rrs", C.c_float), ("a_mix", C.c_float), ("radius", C.c_int32), ("rrs_step", C.c_int32),
        ("variant", C.c_int32),
    ]


class NrrsLoss(C.Structure):
    _fields_ = [
        ("loss_stat", C.c_float), ("loss_rrs", C.c_float), ("e_avg", C.c_double), ("records", C.c_uint32),
        ("rrs_trained", C.c_uint32),
    ]


class Instances(C.Structure):
    """nrrs_instances: object-space meshes and their instances."""
    _fields_ = [
        ("mesh_verts", C.c_void_p), ("mesh_nv", C.c_uint64), ("mesh_tris", C.c_void_p),
        ("mesh_tri_mat", C.c_void_p), ("mesh_tri_begin", C.c_void_p), ("n_meshes", C.c_uint32),
        ("inst_mesh", C.c_void_p), ("inst_xform", C.c_void_p), ("inst_mat", C.c_void_p), ("n_inst", C.c_uint32),
    ]


class RenderStats(C.Structure):
    _fields_ = [
        ("max_depth", C.c_uint32), ("passes", C.c_uint32),
        ("n", C.c_uint64 * (MAX_DEPTH + 1)), ("S", C.c_uint64 * (MAX_DEPTH + 1)),
        ("retries", C.c_uint64 * (MAX_DEPTH + 1)), ("sumq", C.c_double * (MAX_DEPTH + 1)),
        ("F", C.c_double * (MAX_DEPTH + 1)), ("alpha", C.c_double), ("rays", C.c_uint64),
        ("nodes_visited", C.c_uint64), ("tris_tested", C.c_uint64),
        ("records", C.c_uint64), ("overflow", C.c_uint32), ("timed", C.c_uint32),
        ("stage_ms", C.c_double * NSTAGES), ("stage_launches", C.c_uint64 * NSTAGES),
    ]


class NrrsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nrrs error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libnrrs.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2510_07868_amd.build.build()")
    # torch first: its HIP runtime (SONAME libamdhip64.so.7) is then the one libnrrs binds to, so
    # the library, torch's allocator and torch's streams all live in one runtime instance.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, U32, U64, I32, D = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_double
    sig = {
        "nrrs_create": [P, P, P],
        "nrrs_workspace_size": [P, U64, U32, P],
        "nrrs_bind_workspace": [P, P, U64, U64, U32],
        "nrrs_upload_scene": [P, P, U64, P, U64, P, P, P, U32, P, P],
        "nrrs_upload_scene_instanced": [P, P, U64, P, U64, P, P, P, U32, P, P, P],
        "nrrs_render": [P, U32, U32, I32, P],
        "nrrs_set_timing": [P, I32],
        "nrrs_set_launch_mode": [P, I32],
        "nrrs_set_precision": [P, I32],
        "nrrs_set_mix_depth": [P, U64],
        "nrrs_get_mix_depth": [P, P],
        "nrrs_set_mix_depth_fixed": [P, U64],
        "nrrs_get_mix_depth_fixed": [P, P],
        "nrrs_set_pass_index": [P, U64],
        "nrrs_get_pass_index": [P, P],
        "nrrs_get_tuning": [P, P],
        "nrrs_set_tuning": [P, P],
        "nrrs_autotune": [P, U32, P, P, U32, P],
        "nrrs_train_step": [P, U32, U32, C.c_float, P],
        "nrrs_read_image": [P, P, P],
        "nrrs_reset_image": [P],
        "nrrs_set_guide": [P, P],
        "nrrs_get_guide": [P, P],
        "nrrs_get_params": [P, P, P, P, P],
        "nrrs_set_params": [P, P, P, P, P],
        "nrrs_get_state": [P, P, P],
        "nrrs_set_state": [P, P, P],
        "nrrs_set_trace": [P, I32],
        "nrrs_read_trace": [P, P],
        "nrrs_read_records": [P, P, P, P, P, P, P, P],
        "nrrs_debug_rrs_expand": [P, P, P, P, U32, U32, D, D, P, I32, U32, P, P, P, P, P, P, P],
        "nrrs_rrs_expand_noalloc": [P, P, P, U32, U32, D, D, D, I32, U32, P, P, P],
        "nrrs_debug_set_norm_factors": [P, P, U32],
        "nrrs_debug_load_records": [P, P, P, P, U32],
        "nrrs_debug_read_queue": [P, I32, U32, P, P, P, P],
        "nrrs_debug_trace": [P, P, P, U32, P, P, P, P],
        "nrrs_debug_philox": [P, P, P, U32, P],
        "nrrs_debug_mlp_forward": [P, P, U32, I32, P, P],
        "nrrs_debug_mlp_codes": [P, P, U32, I32, P, P, P],
        "nrrs_debug_mlp_grad": [P, P, P, U32, P, P],
        "nrrs_set_nrrs_params": [P, P, P, P],
        "nrrs_get_nrrs_params": [P, P, P, P],
        "nrrs_train_step_nrrs": [P, U32, P, P],
        "nrrs_debug_nrrs_forward": [P, P, P, P, U32, P, P, P],
        "nrrs_debug_nrrs_grads": [P, P, P, P, P, P, P, P, P, U32, P, P, U32, I32, C.c_float, P, P, P, P, P],
        "nrrs_debug_pixel_error": [P, P, P, P, U32, U32, I32, C.c_float, I32, C.c_float, C.c_float, C.c_float,
                                   P, P, P],
        "nrrs_set_aid_params": [P, P, P],
        "nrrs_get_aid_params": [P, P, P],
        "nrrs_debug_aid_forward": [P, P, P, P, U32, P, P],
        "nrrs_debug_aid_grads": [P, P, P, P, P, P, P, P, U32, P, P, U32, I32, C.c_float, P, P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = I32
    L.nrrs_status_string.argtypes = [I32]
    L.nrrs_status_string.restype = C.c_char_p
    L.nrrs_last_error.argtypes = [P]
    L.nrrs_last_error.restype = C.c_char_p
    L.nrrs_destroy.argtypes = [P]
    L.nrrs_destroy.restype = None
    _lib = L
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Renderer:
    """One rendering context bound to a torch-allocated workspace on ``device``."""

    def __init__(self, width, height, s_batch=1, cap_factor=2.0, f_rate=1.0, norm_mode=NORM_TWO_SIDED, seed=0,
                 net_max_depth=4, precision=PREC_FP32, records_cap=0, p_train=0.0, max_tris=1 << 16,
                 max_materials=4096, device="cuda:0", stream=None, loss=LOSS_REL_L2, ema_decay=0.0,
                 trace_depth=0, hash_log2=0, nee=0):
        import torch
        self.torch = torch
        self.L = load()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        # a stream of its own (default priority): hipGraph capture needs a non-null stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.cfg = Config(width, height, s_batch, cap_factor, f_rate, norm_mode, seed, net_max_depth, precision,
                          records_cap, p_train, loss, ema_decay, trace_depth, hash_log2, nee)
        self.trace_depth = trace_depth
        self.hash_log2 = hash_log2
        self.width, self.height, self.s_batch = width, height, s_batch
        self.records_cap = records_cap
        h = C.c_void_p()
        self._check(self.L.nrrs_create(C.byref(self.cfg), C.c_void_p(self.stream.cuda_stream), C.byref(h)), None)
        self.h = h
        nbytes = C.c_uint64()
        self._check(self.L.nrrs_workspace_size(self.h, max_tris, max_materials, C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self._check(self.L.nrrs_bind_workspace(self.h, C.c_void_p(self.workspace.data_ptr()), int(nbytes.value),
                                               max_tris, max_materials))
        self.max_tris = max_tris
        self.workspace_bytes = int(nbytes.value)

    # ---------------------------------------------------------------- plumbing
    def _check(self, code, h="self"):
        if code != 0:
            L = self.L
            msg = L.nrrs_status_string(code).decode()
            if h is not None and getattr(self, "h", None):
                msg += ": " + L.nrrs_last_error(self.h).decode()
            raise NrrsError(code, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.nrrs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- API
    def upload_scene(self, scene):
        if hasattr(scene, "inst_mesh"):
            return self._upload_instanced(scene)
        v = _c(scene.verts, np.float32)
        t = _c(scene.tris, np.uint32)
        tm = _c(scene.tri_mat, np.uint32)
        mt = _c(scene.mat_type, np.uint32)
        mp = _c(scene.mat_params, np.float32)
        cam = _c(scene.camera, np.float32)
        env = _c(scene.env, np.float32)
        self._check(self.L.nrrs_upload_scene(self.h, _p(v), v.shape[0], _p(t), t.shape[0], _p(tm), _p(mt), _p(mp),
                                             mt.shape[0], _p(cam), _p(env)))

    def _upload_instanced(self, scene):
        b = scene.base
        v = _c(b.verts, np.float32).reshape(-1, 3)
        t = _c(b.tris, np.uint32).reshape(-1, 3)
        tm = _c(b.tri_mat, np.uint32)
        mt = _c(b.mat_type, np.uint32)
        mp = _c(b.mat_params, np.float32)
        cam = _c(b.camera, np.float32)
        env = _c(b.env, np.float32)
        keep = [_c(scene.mesh_verts, np.float32).reshape(-1, 3), _c(scene.mesh_tris, np.uint32),
                _c(scene.mesh_tri_mat, np.uint32), _c(scene.mesh_tri_begin, np.uint64),
                _c(scene.inst_mesh, np.uint32), _c(scene.inst_xform, np.float32), _c(scene.inst_mat, np.uint32)]
        mv, mtr, mtm, mb, im, ix, imat = keep
        inst = Instances(_p(mv), mv.shape[0], _p(mtr), _p(mtm), _p(mb), mb.shape[0] - 1, _p(im), _p(ix), _p(imat),
                         im.shape[0])
        self._check(self.L.nrrs_upload_scene_instanced(
            self.h, _p(v), v.shape[0], _p(t), t.shape[0], _p(tm), _p(mt), _p(mp), mt.shape[0], _p(cam), _p(env),
            C.byref(inst)))

    def render(self, spp, max_depth, mode, stats=True):
        st = RenderStats()
        code = self.L.nrrs_render(self.h, spp, max_depth, mode, C.byref(st) if stats else None)
        if code != 0 and not (stats and code == -5):
            self._check(code)
        if not stats:
            return None
        D = max_depth
        return dict(status=int(code), n=np.array(st.n[: D + 1], np.uint64), S=np.array(st.S[: D + 1], np.uint64),
                    retries=np.array(st.retries[: D + 1], np.uint64), sumq=np.array(st.sumq[: D + 1]),
                    F=np.array(st.F[: D + 1]), alpha=st.alpha, rays=int(st.rays), records=int(st.records),
                    nodes_visited=int(st.nodes_visited), tris_tested=int(st.tris_tested),
                    overflow=int(st.overflow), passes=int(st.passes), timed=bool(st.timed),
                    stage_ms={k: float(st.stage_ms[i]) for i, k in enumerate(STAGES)},
                    stage_launches={k: int(st.stage_launches[i]) for i, k in enumerate(STAGES)})

    def set_launch_mode(self, graphs=True):
        self._check(self.L.nrrs_set_launch_mode(self.h, 1 if graphs else 0))

    def set_precision(self, precision):
        self._check(self.L.nrrs_set_precision(self.h, precision))

    def set_timing(self, enabled=True):
        self._check(self.L.nrrs_set_timing(self.h, 1 if enabled else 0))

    def set_mix_depth(self, net_depths):
        """Mix-Depth table: an int bitmask (bit d-1 = network at depth d) or an iterable of depths."""
        if not isinstance(net_depths, int):
            net_depths = sum(1 << (d - 1) for d in set(net_depths))
        self._check(self.L.nrrs_set_mix_depth(self.h, C.c_uint64(net_depths)))

    def set_pass_index(self, next_pass):
        self._check(self.L.nrrs_set_pass_index(self.h, C.c_uint64(next_pass)))

    def get_pass_index(self):
        m = C.c_uint64()
        self._check(self.L.nrrs_get_pass_index(self.h, C.byref(m)))
        return int(m.value)

    def set_mix_depth_fixed(self, fixed_depths):
        """Depths with the fixed-rate factor: an int bitmask (bit d-1 = depth d) or an iterable of depths."""
        if not isinstance(fixed_depths, int):
            fixed_depths = sum(1 << (d - 1) for d in set(fixed_depths))
        self._check(self.L.nrrs_set_mix_depth_fixed(self.h, C.c_uint64(fixed_depths)))

    def get_mix_depth_fixed(self):
        m = C.c_uint64()
        self._check(self.L.nrrs_get_mix_depth_fixed(self.h, C.byref(m)))
        return int(m.value)

    def get_mix_depth(self):
        m = C.c_uint64()
        self._check(self.L.nrrs_get_mix_depth(self.h, C.byref(m)))
        return int(m.value)

    def get_tuning(self):
        t = Tuning()
        self._check(self.L.nrrs_get_tuning(self.h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, extend_variant, extend_blocks_per_cu, extend_refill, extend_leaf_batch, extend_chunk=0, **_):
        t = Tuning(extend_variant, extend_blocks_per_cu, extend_refill, extend_leaf_batch, extend_chunk)
        self._check(self.L.nrrs_set_tuning(self.h, C.byref(t)))

    def autotune(self, max_depth, with_table=False):
        """Time the traversal kernel's launch candidates on the uploaded scene and keep the fastest
        (clears the accumulated image).  with_table: also return every candidate with its time."""
        t = Tuning()
        tried = (Tuning * 64)()
        n = C.c_uint32()
        self._check(self.L.nrrs_autotune(self.h, max_depth, C.byref(t), tried, 64, C.byref(n)))
        if with_table:
            return t.as_dict(), [tried[k].as_dict() for k in range(min(n.value, 64))]
        return t.as_dict()

    def read_image(self):
        img = np.zeros(self.width * self.height * 3)
        spp = C.c_uint64()
        self._check(self.L.nrrs_read_image(self.h, _p(img), C.byref(spp)))
        return img, int(spp.value)

    def reset_image(self):
        self._check(self.L.nrrs_reset_image(self.h))

    def set_guide(self, lum):
        g = _c(lum, np.float32)
        assert g.size == self.width * self.height
        self._check(self.L.nrrs_set_guide(self.h, _p(g)))

    def get_guide(self):
        g = np.zeros(self.width * self.height, np.float32)
        self._check(self.L.nrrs_get_guide(self.h, _p(g)))
        return g

    def get_params(self):
        w, m, v = (np.zeros(NPARAM, np.float32) for _ in range(3))
        step = C.c_uint64()
        self._check(self.L.nrrs_get_params(self.h, _p(w), _p(m), _p(v), C.byref(step)))
        return w, m, v, int(step.value)

    def set_params(self, master=None, m=None, v=None, step=None):
        arrs = [None if a is None else _c(a, np.float32) for a in (master, m, v)]
        for a in arrs:
            assert a is None or a.size == NPARAM
        st = None if step is None else C.byref(C.c_uint64(int(step)))
        self._check(self.L.nrrs_set_params(self.h, *[None if a is None else _p(a) for a in arrs], st))

    def get_state(self):
        """Inference (moving-average) weights and the overflow guard's alpha."""
        w = np.zeros(NPARAM, np.float32)
        a = C.c_double()
        self._check(self.L.nrrs_get_state(self.h, _p(w), C.byref(a)))
        return w, float(a.value)

    def set_state(self, infer=None, alpha=None):
        w = None if infer is None else _c(infer, np.float32)
        assert w is None or w.size == NPARAM
        self._check(self.L.nrrs_set_state(self.h, None if w is None else _p(w),
                                          None if alpha is None else C.byref(C.c_double(alpha))))

    def set_trace(self, enabled=True):
        """Per-path radiance by depth on (zeroes the sums) or off; needs trace_depth > 0 at creation."""
        self._check(self.L.nrrs_set_trace(self.h, 1 if enabled else 0))

    def read_trace(self):
        """Radiance per primary path and depth [W*H*s_batch, trace_depth, 3], summed over the passes
        since set_trace."""
        out = np.zeros(self.width * self.height * self.s_batch * self.trace_depth * 3)
        self._check(self.L.nrrs_read_trace(self.h, _p(out)))
        return out.reshape(-1, self.trace_depth, 3)

    def read_records(self):
        n = C.c_uint64()
        self._check(self.L.nrrs_read_records(self.h, C.byref(n), None, None, None, None, None, None))
        k = int(n.value)
        f = np.zeros((max(k, 1), 20), np.float32)
        lt, acc = np.zeros(max(k, 1), np.float32), np.zeros(max(k, 1), np.float32)
        d, px = np.zeros(max(k, 1), np.uint32), np.zeros(max(k, 1), np.uint32)
        lin = np.zeros(max(k, 1), np.uint64)
        self._check(self.L.nrrs_read_records(self.h, C.byref(n), _p(f), _p(lt), _p(acc), _p(d), _p(px), _p(lin)))
        return dict(feat=f[:k], lum_t=lt[:k], acc=acc[:k], depth=d[:k], pix=px[:k], id=lin[:k])

    def train_step(self, n_records, minibatch, lr):
        loss = C.c_float()
        self._check(self.L.nrrs_train_step(self.h, n_records, minibatch, C.c_float(lr), C.byref(loss)))
        return float(loss.value)

    # ---------------------------------------------------------------- test entry points
    def debug_rrs_expand(self, q, id_lo, id_hi, depth, budget_base, f_rate=1.0, alpha=1.0,
                         norm_mode=NORM_TWO_SIDED, cap=None):
        q = _c(q, np.float32)
        lo, hi = _c(id_lo, np.uint32), _c(id_hi, np.uint32)
        n = q.size
        cap = int(2 * budget_base) if cap is None else int(cap)
        X = np.zeros(max(n, 1), np.uint32)
        off = np.zeros(max(n, 1), np.uint32)
        par = np.zeros(max(cap, 1), np.uint32)
        S = C.c_uint32()
        F = C.c_double()
        a = C.c_double(alpha)
        qn = np.zeros(max(n, 1), np.float32)
        r = C.c_uint32()
        code = self.L.nrrs_debug_rrs_expand(self.h, _p(q), _p(lo), _p(hi), n, depth, float(budget_base),
                                            float(f_rate), C.byref(a), norm_mode, cap, _p(X), _p(off), _p(par),
                                            C.byref(S), C.byref(F), _p(qn), C.byref(r))
        if code not in (0, -5):
            self._check(code)
        return dict(status=int(code), X=X[:n], offset=off[:n], parent=par[: S.value].copy(), S=int(S.value),
                    F=float(F.value), q_norm=qn[:n], alpha=float(a.value), retries=int(r.value))

    def rrs_expand_noalloc(self, q, lineage, offset, result, depth, budget_base, f_rate=1.0, alpha=1.0,
                           norm_mode=NORM_TWO_SIDED, cap=None, parent=None):
        """nrrs_rrs_expand_noalloc on torch tensors of this context's device: q float32 [n], lineage
        int32 [n, 2] (lo, hi words), offset int32 [n] (out), result uint8 [32] (out), parent int32
        [cap] (out) or None.  Queued on the context's stream; nothing is allocated."""
        t = self.torch
        n = int(q.numel())
        assert q.dtype == t.float32 and lineage.dtype == t.int32 and offset.dtype == t.int32
        assert result.dtype == t.uint8 and result.numel() >= 32
        assert lineage.numel() == 2 * n and offset.numel() >= n
        assert q.is_contiguous() and lineage.is_contiguous() and offset.is_contiguous() and result.is_contiguous()
        cap = int(2 * budget_base) if cap is None else int(cap)
        if parent is not None:
            assert parent.dtype == t.int32 and parent.is_contiguous() and parent.numel() >= cap
        ptr = lambda x: C.c_void_p(x.data_ptr())  # noqa: E731
        self._check(self.L.nrrs_rrs_expand_noalloc(self.h, ptr(q), ptr(lineage), n, depth, float(budget_base),
                                                   float(f_rate), float(alpha), norm_mode, cap, ptr(offset),
                                                   None if parent is None else ptr(parent), ptr(result)))

    @staticmethod
    def decode_expand_result(result_bytes):
        """The nrrs_expand_result fields of 32 bytes copied to the host."""
        b = np.asarray(result_bytes, np.uint8)[:32].tobytes()
        F, alpha = np.frombuffer(b[:16], np.float64)
        S, retries, overflow, _ = np.frombuffer(b[16:], np.uint32)
        return dict(F=float(F), alpha=float(alpha), S=int(S), retries=int(retries), overflow=int(overflow))

    def debug_set_norm_factors(self, F=None):
        """Normalization factor per depth (F[d-1] at depth d) used instead of the computed one;
        None restores the computed factors."""
        if F is None:
            self._check(self.L.nrrs_debug_set_norm_factors(self.h, None, 0))
            return
        f = _c(F, np.float64)
        self._check(self.L.nrrs_debug_set_norm_factors(self.h, _p(f), f.size))

    def debug_load_records(self, feat, lum_t, acc):
        f = _c(feat, np.float32).reshape(-1, 20)
        lt, ac = _c(lum_t, np.float32), _c(acc, np.float32)
        assert lt.size == ac.size == f.shape[0]
        self._check(self.L.nrrs_debug_load_records(self.h, _p(f), _p(lt), _p(ac), f.shape[0]))

    def debug_read_queue(self, which, n):
        o, d, t, h = (np.zeros((n, 4), np.float32) for _ in range(4))
        self._check(self.L.nrrs_debug_read_queue(self.h, which, n, _p(o), _p(d), _p(t), _p(h)))
        return o, d, t, h

    def debug_trace(self, rays, exclude=None):
        rays = _c(rays, np.float32).reshape(-1, 6)
        n = rays.shape[0]
        ex = _c(exclude if exclude is not None else np.full(n, MISS), np.uint32)
        prim = np.zeros(n, np.uint32)
        t, b1, b2 = (np.zeros(n, np.float32) for _ in range(3))
        self._check(self.L.nrrs_debug_trace(self.h, _p(rays), _p(ex), n, _p(prim), _p(t), _p(b1), _p(b2)))
        return prim, t, b1, b2

    def debug_philox(self, ctr, key):
        ctr = _c(ctr, np.uint32).reshape(-1, 4)
        out = np.zeros_like(ctr)
        k = _c(key, np.uint32)
        self._check(self.L.nrrs_debug_philox(self.h, _p(ctr), _p(k), ctr.shape[0], _p(out)))
        return out

    def debug_mlp_forward(self, x, precision=PREC_FP32):
        x = _c(x, np.float32).reshape(-1, 20)
        n = x.shape[0]
        y, z = np.zeros(n, np.float32), np.zeros(n, np.float32)
        self._check(self.L.nrrs_debug_mlp_forward(self.h, _p(x), n, precision, _p(y), _p(z)))
        return y, z

    # ---------------------------------------------------------------- NRRS proper
    def table_size(self):
        return HG_LEVELS * HG_FEAT * (1 << self.hash_log2)

    def set_nrrs_params(self, stat=None, rrs=None, table=None):
        a = [None if v is None else _c(v, np.float32) for v in (stat, rrs, table)]
        for v, n in zip(a, (STAT_NPARAM, RRS_NPARAM, self.table_size())):
            if v is not None and v.size != n:
                raise ValueError(f"expected {n} values, got {v.size}")
        self._check(self.L.nrrs_set_nrrs_params(self.h, *[None if v is None else _p(v) for v in a]))

    def get_nrrs_params(self):
        st, rr, tb = np.zeros(STAT_NPARAM, np.float32), np.zeros(RRS_NPARAM, np.float32), \
            np.zeros(self.table_size(), np.float32)
        self._check(self.L.nrrs_get_nrrs_params(self.h, _p(st), _p(rr), _p(tb)))
        return st, rr, tb

    def train_step_nrrs(self, n_records, rrs_step, lr_stat=5e-3, lr_rrs=3e-4, g_avg=0.01, g_min=0.05, g_rrs=0.01,
                        a_mix=0.5, radius=2, variant=0):
        hp = NrrsTrain(lr_stat, lr_rrs, g_avg, g_min, g_rrs, a_mix, radius, rrs_step, variant)
        out = NrrsLoss()
        self._check(self.L.nrrs_train_step_nrrs(self.h, n_records, C.byref(hp), C.byref(out)))
        return dict(loss_stat=float(out.loss_stat), loss_rrs=float(out.loss_rrs), e_avg=float(out.e_avg),
                    records=int(out.records), rrs_trained=bool(out.rrs_trained))

    def set_aid_params(self, aid=None, table_r=None):
        a = [None if v is None else _c(v, np.float32) for v in (aid, table_r)]
        for v, n in zip(a, (AID_NPARAM, self.table_size())):
            if v is not None and v.size != n:
                raise ValueError(f"expected {n} values, got {v.size}")
        self._check(self.L.nrrs_set_aid_params(self.h, *[None if v is None else _p(v) for v in a]))

    def get_aid_params(self):
        pa, tr = np.zeros(AID_NPARAM, np.float32), np.zeros(self.table_size(), np.float32)
        self._check(self.L.nrrs_get_aid_params(self.h, _p(pa), _p(tr)))
        return pa, tr

    def debug_aid_forward(self, raw, t, I, with_enc=False):
        raw = _c(raw, np.float32).reshape(-1, 7)
        n = raw.shape[0]
        t = _c(t, np.float32).reshape(n, 3)
        I = _c(I, np.float32).reshape(n)
        q = np.zeros(max(n, 1), np.float32)
        enc = np.zeros((max(n, 1), 32), np.float32) if with_enc else None
        self._check(self.L.nrrs_debug_aid_forward(self.h, _p(raw), _p(t), _p(I), n, _p(q),
                                                  _p(enc) if with_enc else None))
        return (q[:n], enc[:n]) if with_enc else q[:n]

    def debug_aid_grads(self, raw, I, lum_t, t, q_norm, F, pix, wpx, k, rrs_step, g_rrs=0.01):
        raw = _c(raw, np.float32).reshape(-1, 7)
        n = raw.shape[0]
        arrs = [_c(I, np.float32), _c(lum_t, np.float32), _c(t, np.float32).reshape(n, 3), _c(q_norm, np.float32),
                _c(F, np.float32)]
        pix = _c(pix, np.uint32)
        wpx, k = _c(wpx, np.float32), _c(k, np.uint32)
        ga, gt = np.zeros(AID_NPARAM, np.float32), np.zeros(self.table_size(), np.float32)
        loss = C.c_float()
        self._check(self.L.nrrs_debug_aid_grads(self.h, _p(raw), *[_p(a) for a in arrs], _p(pix), n, _p(wpx), _p(k),
                                                wpx.size, rrs_step, float(g_rrs), _p(ga), _p(gt), C.byref(loss)))
        return dict(g_aid=ga, g_table_r=gt, loss=float(loss.value))

    def debug_nrrs_forward(self, raw, t, I, with_enc=False):
        raw = _c(raw, np.float32).reshape(-1, 7)
        n = raw.shape[0]
        t = _c(t, np.float32).reshape(n, 3)
        I = _c(I, np.float32).reshape(n)
        mv = np.zeros((max(n, 1), 2), np.float32)
        q = np.zeros(max(n, 1), np.float32)
        enc = np.zeros((max(n, 1), 32), np.float32) if with_enc else None
        self._check(self.L.nrrs_debug_nrrs_forward(self.h, _p(raw), _p(t), _p(I), n, _p(mv), _p(q),
                                                   _p(enc) if with_enc else None))
        return (mv[:n], q[:n], enc[:n]) if with_enc else (mv[:n], q[:n])

    def debug_nrrs_grads(self, raw, I, L, lum_t, t, q_norm, F, pix, wpx, k, rrs_step, g_rrs=0.01):
        raw = _c(raw, np.float32).reshape(-1, 7)
        n = raw.shape[0]
        arrs = [_c(I, np.float32), _c(L, np.float32), _c(lum_t, np.float32), _c(t, np.float32).reshape(n, 3),
                _c(q_norm, np.float32), _c(F, np.float32)]
        pix = _c(pix, np.uint32)
        wpx, k = _c(wpx, np.float32), _c(k, np.uint32)
        gs, gr = np.zeros(STAT_NPARAM, np.float32), np.zeros(RRS_NPARAM, np.float32)
        gt = np.zeros(self.table_size(), np.float32)
        ls, lr = C.c_float(), C.c_float()
        self._check(self.L.nrrs_debug_nrrs_grads(self.h, _p(raw), *[_p(a) for a in arrs], _p(pix), n, _p(wpx), _p(k),
                                                 wpx.size, rrs_step, float(g_rrs), _p(gs), _p(gr), _p(gt),
                                                 C.byref(ls), C.byref(lr)))
        return dict(g_stat=gs, g_rrs=gr, g_table=gt, loss_stat=float(ls.value), loss_rrs=float(lr.value))

    def debug_pixel_error(self, cur, acc, ref, w, h, first, a_mix=0.5, radius=2, var_scale=1.0, g_avg=0.01,
                          g_min=0.05):
        cur, ref = _c(cur, np.float32).ravel(), _c(ref, np.float32).ravel()
        acc = _c(acc, np.float32).ravel().copy()
        E, wpx = np.zeros(w * h, np.float32), np.zeros(w * h, np.float32)
        e = C.c_double()
        self._check(self.L.nrrs_debug_pixel_error(self.h, _p(cur), _p(acc), _p(ref), w, h, int(first), float(a_mix),
                                                  int(radius), float(var_scale), float(g_avg), float(g_min), _p(E),
                                                  _p(wpx), C.byref(e)))
        return float(e.value), E, wpx, acc

    def debug_mlp_codes(self, x, precision):
        """Matrix-core forward with the bit patterns of every quantized operand: y [n], codes
        [n, 3, 64] (uint16) and FP8 block-scale exponents [n, 3]."""
        xx = _c(x, np.float32).reshape(-1, 20)
        n = xx.shape[0]
        y = np.zeros(max(n, 1), np.float32)
        codes = np.zeros((max(n, 1), 3, 64), np.uint16)
        se = np.zeros((max(n, 1), 3), np.int8)
        self._check(self.L.nrrs_debug_mlp_codes(self.h, _p(xx), n, precision, _p(y), _p(codes), _p(se)))
        return y[:n], codes[:n], se[:n]

    def debug_mlp_grad(self, x, target):
        x = _c(x, np.float32).reshape(-1, 20)
        tg = _c(target, np.float32)
        g = np.zeros(NPARAM, np.float32)
        loss = C.c_float()
        self._check(self.L.nrrs_debug_mlp_grad(self.h, _p(x), _p(tg), x.shape[0], _p(g), C.byref(loss)))
        return float(loss.value), g
