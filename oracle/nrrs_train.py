"""Python wrappers of the FP64 oracle of NRRS training proper (oracle/nrrs_train.c): StatNet,
the NRRS variant of RRSNet, gradient transfer and the pixel error (Sec. 4.2, Sec. 5).

TEST INFRASTRUCTURE ONLY: loaded by the tests and the benchmark's CPU-baseline leg, never by the
HIP product path."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _c, _p, lib as _base_lib

HG_LEVELS, HG_FEAT, HG_BASE = 8, 2, 16
STAT_RAW, STAT_IN, STAT_OUT, RRS_IN, AID_IN = 7, 32, 2, 7, 32

_ready = False


def lib():
    global _ready
    L = _base_lib()
    if not _ready:
        P, D, U32, U64, I32 = C.c_void_p, C.c_double, C.c_uint32, C.c_uint64, C.c_int32
        L.or_oneblob.argtypes = [D, I32, P]
        L.or_hashgrid_encode.argtypes = [P, U32, P, P]
        L.or_hashgrid_backward.argtypes = [U32, P, P, P]
        L.or_hashgrid_cell_margin.restype = D
        L.or_hashgrid_cell_margin.argtypes = [P]
        L.or_statnet_encode.argtypes = [P, U32, P, P]
        L.or_mlp32_nparams.restype = U64
        L.or_mlp32_nparams.argtypes = [I32, I32]
        L.or_mlp32_forward.argtypes = [P, I32, I32, P, P]
        L.or_mlp32_backward.argtypes = [P, I32, I32, P, P, P, P]
        L.or_statnet_forward.argtypes = [P, P, U32, P, P]
        L.or_statnet_loss_grad.restype = D
        L.or_statnet_loss_grad.argtypes = [P, P, U32, P, P, U64, D, P, P]
        L.or_rrs_inputs.argtypes = [P, P, D, D, P]
        L.or_nrrs_factor.restype = D
        L.or_nrrs_factor.argtypes = [P, P, P, U32, P, P, D, P, P]
        L.or_nrrs_dloss_dq.restype = D
        L.or_nrrs_dloss_dq.argtypes = [D, U32, D, P, D, D, D, D]
        L.or_nrrs_pixel_weights.restype = D
        L.or_nrrs_pixel_weights.argtypes = [P, P, P, U32, U32, I32, D, I32, D, D, D, D, P, P]
        L.or_rrsnet_nrrs_grad.restype = D
        L.or_rrsnet_nrrs_grad.argtypes = [P, P, P, U32, P, P, P, P, P, P, P, P, P, U64, I32, D, D, P]
        L.or_aid_encode.argtypes = [P, U32, P, P, D, P]
        L.or_aid_factor.restype = D
        L.or_aid_factor.argtypes = [P, P, U32, P, P, D, P]
        L.or_aid_grad.restype = D
        L.or_aid_grad.argtypes = [P, P, P, P, U32, P, P, P, P, P, P, P, P, P, U64, I32, D, D, P, P]
        _ready = True
    return L


def mlp32_nparams(n_in: int, n_out: int) -> int:
    return int(lib().or_mlp32_nparams(n_in, n_out))


def oneblob(s: float, bins: int) -> np.ndarray:
    out = np.zeros(bins)
    lib().or_oneblob(float(s), int(bins), _p(out))
    return out


def hashgrid_encode(table, log2T: int, p) -> np.ndarray:
    t = _c(table, np.float64)
    p = _c(p, np.float64).reshape(-1, 3)
    out = np.zeros((p.shape[0], HG_LEVELS * HG_FEAT))
    for r in range(p.shape[0]):
        lib().or_hashgrid_encode(_p(t), int(log2T), _p(p[r]), _p(out[r]))
    return out


def hashgrid_backward(log2T: int, p, dout) -> np.ndarray:
    p = _c(p, np.float64).reshape(-1, 3)
    d = _c(dout, np.float64).reshape(-1, HG_LEVELS * HG_FEAT)
    dt = np.zeros(HG_LEVELS * (1 << log2T) * HG_FEAT)
    for r in range(p.shape[0]):
        lib().or_hashgrid_backward(int(log2T), _p(p[r]), _p(d[r]), _p(dt))
    return dt


def cell_margin(p) -> np.ndarray:
    p = _c(p, np.float64).reshape(-1, 3)
    return np.array([lib().or_hashgrid_cell_margin(_p(p[r])) for r in range(p.shape[0])])


def statnet_encode(table, log2T: int, raw) -> np.ndarray:
    t = _c(table, np.float64)
    raw = _c(raw, np.float64).reshape(-1, STAT_RAW)
    out = np.zeros((raw.shape[0], STAT_IN))
    for r in range(raw.shape[0]):
        lib().or_statnet_encode(_p(t), int(log2T), _p(raw[r]), _p(out[r]))
    return out


def mlp32_forward(P, n_in: int, n_out: int, x) -> np.ndarray:
    P = _c(P, np.float64)
    x = _c(x, np.float64).reshape(-1, n_in)
    y = np.zeros((x.shape[0], n_out))
    for r in range(x.shape[0]):
        lib().or_mlp32_forward(_p(P), n_in, n_out, _p(x[r]), _p(y[r]))
    return y


def mlp32_backward(P, n_in: int, n_out: int, x, dy):
    """Summed parameter gradient over the rows, and the input gradients."""
    P = _c(P, np.float64)
    x = _c(x, np.float64).reshape(-1, n_in)
    dy = _c(dy, np.float64).reshape(-1, n_out)
    dP = np.zeros_like(P)
    dx = np.zeros_like(x)
    for r in range(x.shape[0]):
        lib().or_mlp32_backward(_p(P), n_in, n_out, _p(x[r]), _p(dy[r]), _p(dP), _p(dx[r]))
    return dP, dx


def statnet_forward(Ps, table, log2T: int, raw) -> np.ndarray:
    Ps, t = _c(Ps, np.float64), _c(table, np.float64)
    raw = _c(raw, np.float64).reshape(-1, STAT_RAW)
    mv = np.zeros((raw.shape[0], STAT_OUT))
    for r in range(raw.shape[0]):
        lib().or_statnet_forward(_p(Ps), _p(t), int(log2T), _p(raw[r]), _p(mv[r]))
    return mv


def statnet_loss_grad(Ps, table, log2T: int, raw, target, eps: float = 0.01):
    Ps, t = _c(Ps, np.float64), _c(table, np.float64)
    raw = _c(raw, np.float64).reshape(-1, STAT_RAW)
    tg = _c(target, np.float64)
    dP, dT = np.zeros_like(Ps), np.zeros_like(t)
    loss = lib().or_statnet_loss_grad(_p(Ps), _p(t), int(log2T), _p(raw), _p(tg), raw.shape[0], float(eps),
                                      _p(dP), _p(dT))
    return float(loss), dP, dT


def rrs_inputs(mv, t, I, rho) -> np.ndarray:
    mv, t = _c(mv, np.float64).reshape(-1, 2), _c(t, np.float64).reshape(-1, 3)
    I, rho = _c(I, np.float64).ravel(), _c(rho, np.float64).ravel()
    x = np.zeros((mv.shape[0], RRS_IN))
    for r in range(mv.shape[0]):
        lib().or_rrs_inputs(_p(mv[r]), _p(t[r]), float(I[r]), float(rho[r]), _p(x[r]))
    return x


def nrrs_factor(Ps, Pr, table, log2T: int, raw, t, I):
    """q, (m, v) and the pre-activation z per vertex."""
    Ps, Pr, tb = _c(Ps, np.float64), _c(Pr, np.float64), _c(table, np.float64)
    raw = _c(raw, np.float64).reshape(-1, STAT_RAW)
    t = _c(t, np.float64).reshape(-1, 3)
    I = _c(I, np.float64).ravel()
    n = raw.shape[0]
    q, mv, z = np.zeros(n), np.zeros((n, 2)), np.zeros(n)
    zz = C.c_double()
    for r in range(n):
        q[r] = lib().or_nrrs_factor(_p(Ps), _p(Pr), _p(tb), int(log2T), _p(raw[r]), _p(t[r]), float(I[r]),
                                    _p(mv[r]), C.byref(zz))
        z[r] = zz.value
    return q, mv, z


def nrrs_dloss_dq(wpx, k, lum_t, mv, q_norm, F, q_nrrs, g_rrs) -> float:
    mv = _c(mv, np.float64)
    return float(lib().or_nrrs_dloss_dq(float(wpx), int(k), float(lum_t), _p(mv), float(q_norm), float(F),
                                        float(q_nrrs), float(g_rrs)))


def pixel_weights(cur, acc, ref, w: int, h: int, first: bool, a_mix=0.5, radius=2, var_scale=1.0,
                  g_avg=0.01, g_min=0.05, eps=0.01):
    """Returns (E_avg, E, wpx, acc_new)."""
    cur, ref = _c(cur, np.float64).ravel(), _c(ref, np.float64).ravel()
    acc = _c(acc, np.float64).ravel().copy()
    E, wpx = np.zeros(w * h), np.zeros(w * h)
    e = lib().or_nrrs_pixel_weights(_p(cur), _p(acc), _p(ref), w, h, int(first), float(a_mix), int(radius),
                                    float(var_scale), float(g_avg), float(g_min), float(eps), _p(E), _p(wpx))
    return float(e), E, wpx, acc


def rrsnet_nrrs_grad(Pr, Ps, table, log2T: int, raw, t_rgb, I_px, lum_t, q_norm, F, pix, k_pix, wpx, step: int,
                     g_rrs=0.01, eps=0.01):
    Pr, Ps, tb = _c(Pr, np.float64), _c(Ps, np.float64), _c(table, np.float64)
    raw = _c(raw, np.float64).reshape(-1, STAT_RAW)
    n = raw.shape[0]
    args = [_c(t_rgb, np.float64).reshape(-1, 3), _c(I_px, np.float64), _c(lum_t, np.float64),
            _c(q_norm, np.float64), _c(F, np.float64)]
    pix, k_pix, wpx = _c(pix, np.uint32), _c(k_pix, np.uint32), _c(wpx, np.float64)
    dPr = np.zeros_like(Pr)
    loss = lib().or_rrsnet_nrrs_grad(_p(Pr), _p(Ps), _p(tb), int(log2T), _p(raw), *[_p(a) for a in args],
                                     _p(pix), _p(k_pix), _p(wpx), n, int(step), float(g_rrs), float(eps), _p(dPr))
    return float(loss), dPr


def aid_encode(table, log2T: int, raw, t, I) -> np.ndarray:
    tb = _c(table, np.float64)
    raw = _c(raw, np.float64).reshape(-1, STAT_RAW)
    t = _c(t, np.float64).reshape(-1, 3)
    I = _c(I, np.float64).ravel()
    out = np.zeros((raw.shape[0], AID_IN))
    for r in range(raw.shape[0]):
        lib().or_aid_encode(_p(tb), int(log2T), _p(raw[r]), _p(t[r]), float(I[r]), _p(out[r]))
    return out


def aid_factor(Pa, table, log2T: int, raw, t, I):
    """AID-NRRS factor q and pre-activation z per vertex."""
    Pa, tb = _c(Pa, np.float64), _c(table, np.float64)
    raw = _c(raw, np.float64).reshape(-1, STAT_RAW)
    t = _c(t, np.float64).reshape(-1, 3)
    I = _c(I, np.float64).ravel()
    n = raw.shape[0]
    q, z = np.zeros(n), np.zeros(n)
    zz = C.c_double()
    for r in range(n):
        q[r] = lib().or_aid_factor(_p(Pa), _p(tb), int(log2T), _p(raw[r]), _p(t[r]), float(I[r]), C.byref(zz))
        z[r] = zz.value
    return q, z


def aid_grad(Pa, table_r, Ps, table_s, log2T: int, raw, t_rgb, I_px, lum_t, q_norm, F, pix, k_pix, wpx, step: int,
             g_rrs=0.01, eps=0.01):
    Pa, tr, Ps, ts = (_c(a, np.float64) for a in (Pa, table_r, Ps, table_s))
    raw = _c(raw, np.float64).reshape(-1, STAT_RAW)
    n = raw.shape[0]
    args = [_c(t_rgb, np.float64).reshape(-1, 3), _c(I_px, np.float64), _c(lum_t, np.float64),
            _c(q_norm, np.float64), _c(F, np.float64)]
    pix, k_pix, wpx = _c(pix, np.uint32), _c(k_pix, np.uint32), _c(wpx, np.float64)
    dPa, dT = np.zeros_like(Pa), np.zeros_like(tr)
    loss = lib().or_aid_grad(_p(Pa), _p(tr), _p(Ps), _p(ts), int(log2T), _p(raw), *[_p(a) for a in args], _p(pix),
                             _p(k_pix), _p(wpx), n, int(step), float(g_rrs), float(eps), _p(dPa), _p(dT))
    return float(loss), dPa, dT
