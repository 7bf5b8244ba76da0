"""ctypes binding of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
NPARAM = 9729
MAXD = 64
MODE_OFF, MODE_HEUR, MODE_NET, MODE_NRRS, MODE_AID = 0, 1, 2, 3, 4
NORM_TWO_SIDED, NORM_DOWNSCALE = 0, 1
MISS = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain IEEE double: no -ffast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
             "-Wall", "-o", tmp, os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "nrrs_train.c"), "-lm"],
            check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Cfg(C.Structure):
    _fields_ = [
        ("width", C.c_uint32), ("height", C.c_uint32), ("s_batch", C.c_uint32), ("max_depth", C.c_uint32),
        ("pass_begin", C.c_uint32), ("n_passes", C.c_uint32),
        ("mode", C.c_int32), ("norm_mode", C.c_int32), ("net_max_depth", C.c_int32), ("frozen", C.c_int32),
        ("cap_factor", C.c_double), ("f_rate", C.c_double),
        ("seed", C.c_uint64),
        ("alpha", C.c_double), ("p_train", C.c_double),
        ("rec_cap", C.c_uint32), ("update_guide", C.c_uint32),
        ("tau", C.c_double), ("net_depths", C.c_uint64), ("fixed_depths", C.c_uint64),
        ("hash_log2", C.c_uint32), ("nee", C.c_uint32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("n", C.c_uint64 * (MAXD + 1)), ("active", C.c_uint64 * (MAXD + 1)), ("S", C.c_uint64 * (MAXD + 1)),
        ("retries", C.c_uint64 * (MAXD + 1)), ("sumq", C.c_double * (MAXD + 1)), ("F", C.c_double * (MAXD + 1)),
        ("rays", C.c_uint64), ("n_records", C.c_uint64), ("status", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.or_scene_create.restype = P
        L.or_scene_create.argtypes = [P, C.c_uint64, P, C.c_uint64, P, P, P, C.c_uint32, P, P, C.c_int32]
        L.or_scene_destroy.argtypes = [P]
        L.or_philox.argtypes = [P, P, P]
        L.or_philox_batch.argtypes = [P, P, C.c_uint64, P]
        L.or_trace.argtypes = [P, P, P, C.c_uint64, P, P, P, P, C.c_int32, C.c_double, P]
        L.or_rrs_expand.restype = C.c_int32
        L.or_rrs_expand.argtypes = [P, P, C.c_uint64, C.c_double, C.c_double, P, C.c_int32, C.c_uint64,
                                    P, P, P, P, P, P, P]
        L.or_render.restype = C.c_int32
        L.or_render.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.or_enumerate.restype = C.c_int32
        L.or_enumerate.argtypes = [P, P, P, P, P, P, P, P, P]
        L.or_mlp_forward.argtypes = [P, P, C.c_uint64, P, P]
        L.or_mlp_forward_quant.argtypes = [P, P, C.c_uint64, C.c_int32, P, P, P]
        L.or_mlp_forward_quant_codes.argtypes = [P, P, C.c_uint64, C.c_int32, P, P, P, P, P, P]
        L.or_round_bf16.restype = C.c_double
        L.or_round_bf16.argtypes = [C.c_double]
        L.or_round_e4m3.restype = C.c_double
        L.or_round_e4m3.argtypes = [C.c_double]
        L.or_fp8_dot_error_bound.restype = C.c_double
        L.or_fp8_dot_error_bound.argtypes = [P, P, C.c_int32]
        L.or_mlp_loss_grad.restype = C.c_double
        L.or_mlp_loss_grad.argtypes = [P, P, P, C.c_uint64, C.c_double, C.c_int32, P]
        L.or_adam.argtypes = [P, P, P, P, C.c_uint64, C.c_uint64, C.c_double, C.c_double, C.c_double,
                              C.c_double]
        L.or_softplus_mod.restype = C.c_double
        L.or_softplus_mod.argtypes = [C.c_double]
        L.or_softplus_mod_grad.restype = C.c_double
        L.or_softplus_mod_grad.argtypes = [C.c_double]
        L.or_num_threads.restype = C.c_int32
        L.or_ggx_D.restype = C.c_double
        L.or_ggx_D.argtypes = [C.c_double, P]
        L.or_ggx_G1.restype = C.c_double
        L.or_ggx_G1.argtypes = [C.c_double, P]
        L.or_ggx_G2.restype = C.c_double
        L.or_ggx_G2.argtypes = [C.c_double, P, P]
        L.or_ggx_sample.restype = C.c_int32
        L.or_ggx_sample.argtypes = [C.c_double, C.c_double, P, C.c_double, C.c_double, P, P, P]
        L.or_ggx_eval_cos.restype = C.c_double
        L.or_ggx_eval_cos.argtypes = [C.c_double, C.c_double, P, P]
        L.or_ggx_pdf.restype = C.c_double
        L.or_ggx_pdf.argtypes = [C.c_double, P, P]
        L.or_lambert_sample.argtypes = [C.c_double, C.c_double, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class OracleScene:
    def __init__(self, scene, bvh: bool = True):
        self._keep = [_c(scene.verts, np.float32), _c(scene.tris, np.uint32), _c(scene.tri_mat, np.uint32),
                      _c(scene.mat_type, np.uint32), _c(scene.mat_params, np.float32),
                      _c(scene.camera, np.float32), _c(scene.env, np.float32)]
        v, t, tm, mt, mp, cam, env = self._keep
        self.h = lib().or_scene_create(_p(v), v.shape[0], _p(t), t.shape[0], _p(tm), _p(mt), _p(mp), mt.shape[0],
                                       _p(cam), _p(env), 1 if bvh else 0)
        if not self.h:
            raise ValueError("oracle rejected the scene")
        self.bvh = bvh
        self.n_tris = t.shape[0]

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_scene_destroy(self.h)
            self.h = None


def num_threads() -> int:
    return int(lib().or_num_threads())


def philox(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox(_p(c), _p(k), _p(out))
    return out


def philox_batch(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32).reshape(-1, 4)
    k = _c(key, np.uint32)
    out = np.zeros_like(c)
    lib().or_philox_batch(_p(c), _p(k), c.shape[0], _p(out))
    return out


def trace(sc: OracleScene, rays: np.ndarray, exclude=None, bvh=None, tau=0.0, with_fragile=False):
    rays = _c(rays, np.float64).reshape(-1, 6)
    n = rays.shape[0]
    ex = _c(exclude if exclude is not None else np.full(n, MISS), np.uint32)
    prim = np.zeros(n, np.uint32)
    t, b1, b2 = (np.zeros(n) for _ in range(3))
    frag = np.zeros(n, np.uint8)
    use = sc.bvh if bvh is None else bvh
    lib().or_trace(sc.h, _p(rays), _p(ex), n, _p(prim), _p(t), _p(b1), _p(b2), 1 if use else 0, float(tau),
                   _p(frag))
    if with_fragile:
        return prim, t, b1, b2, frag.astype(bool)
    return prim, t, b1, b2


def rrs_expand(q, u, budget_base, f_rate=1.0, alpha=1.0, norm_mode=NORM_TWO_SIDED, cap=None):
    q = _c(q, np.float64)
    u = _c(u, np.float64)
    n = q.shape[0]
    if cap is None:
        cap = 2 * int(budget_base)
    X = np.zeros(n, np.uint32)
    off = np.zeros(n, np.uint64)
    # parent map can be as long as S <= cap
    poc = np.zeros(max(int(cap), 1), np.uint32)
    S = np.zeros(1, np.uint64)
    F = np.zeros(1, np.float64)
    qn = np.zeros(n, np.float32)
    a = np.array([alpha], np.float64)
    retries = np.zeros(1, np.uint32)
    st = lib().or_rrs_expand(_p(q), _p(u), n, float(budget_base), float(f_rate), _p(a), int(norm_mode), int(cap),
                             _p(X), _p(off), _p(poc), _p(S), _p(F), _p(qn), _p(retries))
    return dict(status=int(st), X=X, offset=off, parent=poc[: int(S[0])].copy(), S=int(S[0]), F=float(F[0]),
                q_norm=qn, alpha=float(a[0]), retries=int(retries[0]))


def make_cfg(width, height, s_batch=1, max_depth=8, pass_begin=0, n_passes=1, mode=MODE_HEUR,
             norm_mode=NORM_TWO_SIDED, net_max_depth=4, cap_factor=2.0, f_rate=1.0, seed=0, alpha=1.0,
             p_train=0.0, rec_cap=0, update_guide=0, tau=1e-4, frozen=0, net_depths=None,
             fixed_depths=0, hash_log2=0, nee=0) -> Cfg:
    # Mix-Depth table (Sec. 4.3): bit d-1 set = network at depth d; default = depths 1..net_max_depth;
    # a bit of fixed_depths gives its depth the fixed rate instead (it wins over the network bit)
    if net_depths is None:
        net_depths = (1 << net_max_depth) - 1
    return Cfg(width, height, s_batch, max_depth, pass_begin, n_passes, mode, norm_mode, net_max_depth, frozen,
               cap_factor, f_rate, seed, alpha, p_train, rec_cap, update_guide, tau, net_depths, fixed_depths,
               hash_log2, nee)


def render(sc: OracleScene, cfg: Cfg, params=None, guide=None, image=None, records=False, paths=False):
    """Run passes [pass_begin, pass_begin + n_passes); returns a dict with the FP64 radiance sums.
    paths: also the radiance of every primary path by vertex depth (path_rgb [nprim, D, 3], summed
    over the passes) and the first depth a near-tie decision may change (path_first [nprim],
    D + 1 = none)."""
    npx = cfg.width * cfg.height
    img = np.zeros(npx * 3) if image is None else image
    assert img.dtype == np.float64 and img.size == npx * 3
    frag = np.zeros(npx, np.uint8)
    st = Stats()
    pr = None if params is None else _c(params, np.float64)
    gd = None if guide is None else guide
    if gd is not None:
        assert gd.dtype == np.float64 and gd.size == npx
    cap = cfg.rec_cap if records else 0
    cfg.rec_cap = cap
    rf = np.zeros((max(cap, 1), 20))
    rl, ra = np.zeros(max(cap, 1)), np.zeros(max(cap, 1))
    rd, rp = np.zeros(max(cap, 1), np.uint32), np.zeros(max(cap, 1), np.uint32)
    ri = np.zeros(max(cap, 1), np.uint64)
    N = None
    nprim = npx * cfg.s_batch
    prgb = np.zeros(nprim * cfg.max_depth * 3) if paths else None
    pfrag = np.zeros(nprim, np.uint8) if paths else None
    status = lib().or_render(sc.h, C.byref(cfg), N if pr is None else _p(pr), N if gd is None else _p(gd), _p(img),
                             _p(frag), C.byref(st), _p(rf), _p(rl), _p(ra), _p(rd), _p(rp), _p(ri),
                             N if prgb is None else _p(prgb), N if pfrag is None else _p(pfrag))
    D = cfg.max_depth
    out = dict(status=int(status), image=img, fragile=frag.astype(bool), alpha=cfg.alpha,
               n=np.array(st.n[: D + 1]), active=np.array(st.active[: D + 1]), S=np.array(st.S[: D + 1]),
               retries=np.array(st.retries[: D + 1]), sumq=np.array(st.sumq[: D + 1]), F=np.array(st.F[: D + 1]),
               rays=int(st.rays), n_records=int(st.n_records))
    if paths:
        out["path_rgb"] = prgb.reshape(nprim, cfg.max_depth, 3)
        out["path_first"] = pfrag.astype(np.int64)
    if records:
        k = int(st.n_records)
        out["records"] = dict(feat=rf[:k].copy(), lum_t=rl[:k].copy(), acc=ra[:k].copy(), depth=rd[:k].copy(),
                              pix=rp[:k].copy(), id=ri[:k].copy())
    return out


def enumerate_expectation(sc: OracleScene, cfg: Cfg, with_pmf=False):
    npx = cfg.width * cfg.height
    nprim = npx * cfg.s_batch
    cap = int(np.floor(cfg.cap_factor * nprim))
    ie, io = np.zeros(npx * 3), np.zeros(npx * 3)
    ms, br = np.zeros(1, np.uint64), np.zeros(1, np.uint64)
    pmf = np.zeros((cfg.max_depth + 1) * (cap + 2))
    live = np.zeros(cfg.max_depth + 1)
    qn1 = np.zeros(nprim, np.float32)
    st = lib().or_enumerate(sc.h, C.byref(cfg), _p(ie), _p(io), _p(ms), _p(br), _p(pmf), _p(live), _p(qn1))
    if st != 0:
        raise RuntimeError(f"or_enumerate failed: {st}")
    if with_pmf:
        return ie, io, int(ms[0]), int(br[0]), pmf.reshape(cfg.max_depth + 1, cap + 2), live, qn1
    return ie, io, int(ms[0]), int(br[0])


def mlp_forward(params, x):
    P = _c(params, np.float64)
    x = _c(x, np.float64).reshape(-1, 20)
    n = x.shape[0]
    y, z = np.zeros(n), np.zeros(n)
    lib().or_mlp_forward(_p(P), _p(x), n, _p(y), _p(z))
    return y, z


LOSS_REL_L2, LOSS_LOG_MSE = 0, 1


def round_bf16(x):
    return float(lib().or_round_bf16(float(x)))


def round_e4m3(x):
    return float(lib().or_round_e4m3(float(x)))


def fp8_dot_error_bound(w, x):
    w = _c(w, np.float64)
    x = _c(x, np.float64)
    assert w.size == x.size
    return float(lib().or_fp8_dot_error_bound(_p(w), _p(x), int(w.size)))


def mlp_forward_quant(params, x, prec, with_fragile=False):
    P = _c(params, np.float64)
    x = _c(x, np.float64).reshape(-1, 20)
    n = x.shape[0]
    y, z = np.zeros(n), np.zeros(n)
    frag = np.zeros(n, np.uint8)
    lib().or_mlp_forward_quant(_p(P), _p(x), n, int(prec), _p(y), _p(z), _p(frag))
    if with_fragile:
        return y, z, frag.astype(bool)
    return y, z


def mlp_forward_quant_codes(params, x, prec):
    """Quantized forward with the codes of every quantized layer (inputs, hidden 1, hidden 2):
    returns y, z, row near-tie flags, codes [n, 3, 64] (uint16 bit patterns), per-activation
    near-tie flags [n, 3, 64] and FP8 block-scale exponents [n, 3]."""
    P = _c(params, np.float64)
    x = _c(x, np.float64).reshape(-1, 20)
    n = x.shape[0]
    y, z = np.zeros(n), np.zeros(n)
    frag = np.zeros(n, np.uint8)
    codes = np.zeros((n, 3, 64), np.uint16)
    near = np.zeros((n, 3, 64), np.uint8)
    se = np.zeros((n, 3), np.int8)
    lib().or_mlp_forward_quant_codes(_p(P), _p(x), n, int(prec), _p(y), _p(z), _p(frag), _p(codes), _p(near), _p(se))
    return y, z, frag.astype(bool), codes, near.astype(bool), se


def mlp_loss_grad(params, x, target, eps=0.01, kind=LOSS_LOG_MSE):
    P = _c(params, np.float64)
    x = _c(x, np.float64).reshape(-1, 20)
    tg = _c(target, np.float64)
    g = np.zeros(NPARAM)
    loss = lib().or_mlp_loss_grad(_p(P), _p(x), _p(tg), x.shape[0], float(eps), int(kind), _p(g))
    return float(loss), g


def adam(params, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(grad, np.float64)
    lib().or_adam(_p(params), _p(m), _p(v), _p(g), params.size, int(step), float(lr), float(b1), float(b2), float(eps))


def softplus_mod(z: float) -> float:
    return float(lib().or_softplus_mod(float(z)))


def softplus_mod_grad(z: float) -> float:
    return float(lib().or_softplus_mod_grad(float(z)))


def ggx_D(alpha, h):
    return float(lib().or_ggx_D(float(alpha), _p(_c(h, np.float64))))


def ggx_G1(alpha, w):
    return float(lib().or_ggx_G1(float(alpha), _p(_c(w, np.float64))))


def ggx_G2(alpha, wo, wi):
    return float(lib().or_ggx_G2(float(alpha), _p(_c(wo, np.float64)), _p(_c(wi, np.float64))))


def ggx_sample(alpha, f0, wo, u1, u2):
    wi = np.zeros(3)
    w = np.zeros(1)
    pdf = np.zeros(1)
    ok = lib().or_ggx_sample(float(alpha), float(f0), _p(_c(wo, np.float64)), float(u1), float(u2), _p(wi), _p(w),
                             _p(pdf))
    return bool(ok), wi, float(w[0]), float(pdf[0])


def ggx_pdf(alpha, wo, wi):
    return float(lib().or_ggx_pdf(float(alpha), _p(_c(wo, np.float64)), _p(_c(wi, np.float64))))


def ggx_eval_cos(alpha, f0, wo, wi):
    return float(lib().or_ggx_eval_cos(float(alpha), float(f0), _p(_c(wo, np.float64)), _p(_c(wi, np.float64))))


def lambert_sample(u1, u2):
    wi = np.zeros(3)
    pdf = np.zeros(1)
    lib().or_lambert_sample(float(u1), float(u2), _p(wi), _p(pdf))
    return wi, float(pdf[0])
