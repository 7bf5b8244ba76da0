/* FP64 CPU oracle of NRRS training proper: StatNet, the NRRS variant of RRSNet, and the
 * losses that train them through gradient transfer.
 *
 * TEST INFRASTRUCTURE ONLY (part of liboracle.so; see oracle.h).  Written from the paper's
 * definitions with plain loops in double precision; shares no code with the HIP path.
 *
 * Paper references (NRRS, arXiv 2510.07868):
 *   variance of splitting / RR and their derivatives   Sec. 3, Eqs. (4)-(7)
 *   StatNet, RRSNet (NRRS inputs)                      Sec. 4.2.1
 *   StatNet loss (relative L2, stop-gradient)          Sec. 4.2.2, Eq. (15)
 *   RRSNet loss gamma1 L_avg + gamma2 L_min + gamma3 L_rrs, Eq. (16); Eqs. (19)-(21)
 *   gradient transfer (one-sample estimates)           Sec. 4.2.2, Eqs. (17)-(18)
 *   per-sample sharing of the pixel loss               Sec. 4.2.2 (end)
 *   3 hidden layers of 32, leaky ReLU; encodings       Sec. 5 "Network Architecture", "Input Encoding"
 *   two-step training schedule                         Sec. 5 "Training"
 *   temporal accumulation of the error image           Sec. 5 "Tackle Low Spp", Eq. (23)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"


/* ----------------------------------------------------------------- one-blob encoding
 * Sec. 5 "Input Encoding" (one-blob encoding of Mueller et al. 2019): a Gaussian kernel of
 * width sigma = 1 / bins centred at s in [0, 1], read at the centre of each of the bins. */
void or_oneblob(double s, int32_t bins, double* out) {
  if (s < 0.0) s = 0.0;
  if (s > 1.0) s = 1.0;
  const double sigma = 1.0 / bins;
  for (int i = 0; i < bins; ++i) {
    const double c = (i + 0.5) / bins;
    out[i] = exp(-(s - c) * (s - c) / (2.0 * sigma * sigma));
  }
}

/* ------------------------------------------------------ multiresolution hash grid
 * Sec. 5 "Input Encoding": 8 levels of 2 trainable features, coarsest resolution 16, doubling
 * per level (the hash grid of Mueller et al. 2022).  Level l has resolution R = 16 * 2^l:
 * the point p in [0, 1]^3 lies in cell c = min(floor(p R), R - 1) per axis, and its value is
 * the trilinear interpolation of the features stored at the cell's 8 corners.  A corner
 * (x, y, z) is stored densely at x + (R + 1)(y + (R + 1) z) when the level's (R + 1)^3
 * corners fit the table of T = 2^log2T entries, else at the spatial hash
 * (x * 1 ^ y * 2654435761 ^ z * 805459861) mod T in 32-bit unsigned arithmetic.
 * Table layout: [level][T][2]. */
static uint32_t hg_index(uint32_t R, uint32_t log2T, uint32_t x, uint32_t y, uint32_t z) {
  const uint64_t T = 1ull << log2T;
  const uint64_t side = (uint64_t)R + 1;
  if (side * side * side <= T) return (uint32_t)(x + side * (y + side * z));
  const uint32_t h = (x * 1u) ^ (y * 2654435761u) ^ (z * 805459861u);
  return h & (uint32_t)(T - 1);
}

/* Corners and trilinear weights of p at level l. */
static void hg_corners(const double* p, int l, uint32_t log2T, uint32_t idx[8], double w[8]) {
  const uint32_t R = (uint32_t)OR_HG_BASE << l;
  uint32_t c[3];
  double f[3];
  for (int a = 0; a < 3; ++a) {
    double u = p[a];
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
    u *= (double)R;
    double fl = floor(u);
    if (fl > (double)(R - 1)) fl = (double)(R - 1);
    c[a] = (uint32_t)fl;
    f[a] = u - fl;
  }
  for (int k = 0; k < 8; ++k) {
    const uint32_t dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    idx[k] = hg_index(R, log2T, c[0] + dx, c[1] + dy, c[2] + dz);
    w[k] = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
  }
}

void or_hashgrid_encode(const double* table, uint32_t log2T, const double* p, double* out) {
  const uint64_t T = 1ull << log2T;
  for (int l = 0; l < OR_HG_LEVELS; ++l) {
    uint32_t idx[8];
    double w[8];
    hg_corners(p, l, log2T, idx, w);
    const double* tl = table + (uint64_t)l * T * OR_HG_FEAT;
    for (int f = 0; f < OR_HG_FEAT; ++f) {
      double v = 0.0;
      for (int k = 0; k < 8; ++k) v += w[k] * tl[(uint64_t)idx[k] * OR_HG_FEAT + f];
      out[OR_HG_FEAT * l + f] = v;
    }
  }
}

void or_hashgrid_backward(uint32_t log2T, const double* p, const double* dout, double* dtable) {
  const uint64_t T = 1ull << log2T;
  for (int l = 0; l < OR_HG_LEVELS; ++l) {
    uint32_t idx[8];
    double w[8];
    hg_corners(p, l, log2T, idx, w);
    double* tl = dtable + (uint64_t)l * T * OR_HG_FEAT;
    for (int k = 0; k < 8; ++k)
      for (int f = 0; f < OR_HG_FEAT; ++f) tl[(uint64_t)idx[k] * OR_HG_FEAT + f] += w[k] * dout[OR_HG_FEAT * l + f];
  }
}

/* Distance of p * R to the nearest integer over all axes and levels: below a small margin
 * the float32 cell choice of another implementation may differ (near-tie flag). */
double or_hashgrid_cell_margin(const double* p) {
  double m = 1e300;
  for (int l = 0; l < OR_HG_LEVELS; ++l) {
    const double R = (double)(OR_HG_BASE << l);
    for (int a = 0; a < 3; ++a) {
      const double u = p[a] * R;
      const double d = fabs(u - nearbyint(u));
      if (d < m) m = d;
    }
  }
  return m;
}

/* ------------------------------------------------------------ StatNet input encoding
 * Raw record: p in [0, 1]^3 (position in the scene box), w_o (unit, world space), remapped
 * roughness rho = 1 - exp(-alpha).  Encoding (Sec. 5 "Input Encoding"): hash grid of p (16),
 * one-blob of the spherical coordinates of w_o, theta / pi and phi / (2 pi) + 1/2, with 4 bins
 * each (8), one-blob of rho with 8 bins (8): 32 inputs. */
void or_statnet_encode(const double* table, uint32_t log2T, const double* raw, double* enc) {
  or_hashgrid_encode(table, log2T, raw, enc);
  double wz = raw[5];
  if (wz > 1.0) wz = 1.0;
  if (wz < -1.0) wz = -1.0;
  const double theta = acos(wz);
  const double phi = atan2(raw[4], raw[3]);
  or_oneblob(theta / M_PI, 4, enc + 16);
  or_oneblob(phi / (2.0 * M_PI) + 0.5, 4, enc + 20);
  or_oneblob(raw[6], 8, enc + 24);
}

/* ------------------------------------------------------------------ 32-wide MLP
 * Sec. 5 "Network Architecture": in -> 32 -> 32 -> 32 -> out, leaky ReLU (slope 0.01) after
 * each hidden layer, linear output.  Parameters: W1[32][in], b1[32], W2[32][32], b2[32],
 * W3[32][32], b3[32], W4[out][32], b4[out]. */
#define LEAK 0.01
#define HW 32

uint64_t or_mlp32_nparams(int32_t in, int32_t out) {
  return (uint64_t)HW * in + HW + 2ull * (HW * HW + HW) + (uint64_t)out * HW + out;
}

typedef struct {
  const double *W[4], *b[4];
} mlp32_view;

static mlp32_view mlp32_split(const double* P, int in, int out) {
  mlp32_view v;
  const int fan_in[4] = {in, HW, HW, HW}, fan_out[4] = {HW, HW, HW, out};
  uint64_t o = 0;
  for (int L = 0; L < 4; ++L) {
    v.W[L] = P + o;
    o += (uint64_t)fan_in[L] * fan_out[L];
    v.b[L] = P + o;
    o += fan_out[L];
  }
  return v;
}

/* Forward of one row; pre[3][32] and act[3][32] (may be NULL) keep the hidden layers. */
static void mlp32_fwd(const double* P, int in, int out, const double* x, double* y, double pre[3][HW],
                      double act[3][HW]) {
  const mlp32_view v = mlp32_split(P, in, out);
  double h[HW], g[HW];
  const double* src = x;
  int k = in;
  for (int L = 0; L < 3; ++L) {
    for (int o = 0; o < HW; ++o) {
      double a = v.b[L][o];
      for (int i = 0; i < k; ++i) a += v.W[L][(uint64_t)o * k + i] * src[i];
      if (pre) pre[L][o] = a;
      g[o] = a > 0.0 ? a : LEAK * a;
    }
    memcpy(h, g, sizeof(h));
    if (act) memcpy(act[L], h, sizeof(h));
    src = h;
    k = HW;
  }
  for (int o = 0; o < out; ++o) {
    double a = v.b[3][o];
    for (int i = 0; i < HW; ++i) a += v.W[3][(uint64_t)o * HW + i] * h[i];
    y[o] = a;
  }
}

void or_mlp32_forward(const double* P, int32_t in, int32_t out, const double* x, double* y) {
  mlp32_fwd(P, in, out, x, y, NULL, NULL);
}

/* Backward of one row: dP += dL/dP for the output gradient dy; dx (may be NULL) = dL/dx. */
void or_mlp32_backward(const double* P, int32_t in, int32_t out, const double* x, const double* dy, double* dP,
                       double* dx) {
  double pre[3][HW], act[3][HW], y[64];
  mlp32_fwd(P, in, out, x, y, pre, act);
  const mlp32_view v = mlp32_split(P, in, out);
  const mlp32_view d = mlp32_split(dP, in, out);
  double* dW[4];
  double* db[4];
  for (int L = 0; L < 4; ++L) {
    dW[L] = (double*)d.W[L];
    db[L] = (double*)d.b[L];
  }
  /* output layer */
  double dh[HW];
  for (int i = 0; i < HW; ++i) dh[i] = 0.0;
  for (int o = 0; o < out; ++o) {
    db[3][o] += dy[o];
    for (int i = 0; i < HW; ++i) {
      dW[3][(uint64_t)o * HW + i] += dy[o] * act[2][i];
      dh[i] += dy[o] * v.W[3][(uint64_t)o * HW + i];
    }
  }
  /* hidden layers 3, 2, 1 */
  for (int L = 2; L >= 0; --L) {
    double da[HW];
    for (int o = 0; o < HW; ++o) da[o] = dh[o] * (pre[L][o] > 0.0 ? 1.0 : LEAK);
    const int k = L == 0 ? in : HW;
    const double* src = L == 0 ? x : act[L - 1];
    double dsrc[HW > 64 ? HW : 64];
    for (int i = 0; i < k; ++i) dsrc[i] = 0.0;
    for (int o = 0; o < HW; ++o) {
      db[L][o] += da[o];
      for (int i = 0; i < k; ++i) {
        dW[L][(uint64_t)o * k + i] += da[o] * src[i];
        dsrc[i] += da[o] * v.W[L][(uint64_t)o * k + i];
      }
    }
    if (L > 0) {
      for (int i = 0; i < HW; ++i) dh[i] = dsrc[i];
    } else if (dx) {
      for (int i = 0; i < in; ++i) dx[i] = dsrc[i];
    }
  }
}

/* ------------------------------------------------------------------------ StatNet
 * Outputs m (luminance mean of the reflected radiance) and v (its variance) (Sec. 4.2.1).
 * Loss per record (Eq. 15): L2(m, L) + L2(v, (L - sg(m))^2), L2(a, b) = (a - b)^2 / (sg(b)^2 + eps),
 * averaged over the n records.  Gradients accumulate into dP (MLP) and dtable (hash grid). */
void or_statnet_forward(const double* P, const double* table, uint32_t log2T, const double* raw, double* mv) {
  double enc[OR_STAT_IN];
  or_statnet_encode(table, log2T, raw, enc);
  or_mlp32_forward(P, OR_STAT_IN, OR_STAT_OUT, enc, mv);
}

double or_statnet_loss_grad(const double* P, const double* table, uint32_t log2T, const double* raw,
                            const double* target, uint64_t n, double eps, double* dP, double* dtable) {
  double loss = 0.0;
  for (uint64_t r = 0; r < n; ++r) {
    const double* rr = raw + OR_STAT_RAW * r;
    double enc[OR_STAT_IN], mv[OR_STAT_OUT], denc[OR_STAT_IN];
    or_statnet_encode(table, log2T, rr, enc);
    or_mlp32_forward(P, OR_STAT_IN, OR_STAT_OUT, enc, mv);
    const double L = target[r];
    const double v1 = (L - mv[0]) * (L - mv[0]); /* one-sample variance about sg(m) */
    const double em = (mv[0] - L), ev = (mv[1] - v1);
    loss += em * em / (L * L + eps) + ev * ev / (v1 * v1 + eps);
    double dy[OR_STAT_OUT];
    dy[0] = 2.0 * em / (L * L + eps) / (double)n;
    dy[1] = 2.0 * ev / (v1 * v1 + eps) / (double)n;
    or_mlp32_backward(P, OR_STAT_IN, OR_STAT_OUT, enc, dy, dP, denc);
    if (dtable) or_hashgrid_backward(log2T, rr, denc, dtable);
  }
  return n ? loss / (double)n : 0.0;
}

/* ------------------------------------------------------------- RRSNet (NRRS variant)
 * Inputs (Sec. 5 "Input Encoding", NRRS): Box-Cox (lambda = 1/2: 2 (sqrt(x) - 1)) of the
 * StatNet mean m, of the second moment E[L^2] = v + m^2, of the throughput t (RGB) and of the
 * pixel value I; the remapped roughness rho as is.  Negative StatNet outputs count as 0. */
static double box_cox(double x) { return 2.0 * (sqrt(x > 0.0 ? x : 0.0) - 1.0); }

void or_rrs_inputs(const double* mv, const double* t, double I, double rho, double* x) {
  const double m = mv[0] > 0.0 ? mv[0] : 0.0;
  const double v = mv[1] > 0.0 ? mv[1] : 0.0;
  x[0] = box_cox(m);
  x[1] = box_cox(v + m * m);
  x[2] = box_cox(t[0]);
  x[3] = box_cox(t[1]);
  x[4] = box_cox(t[2]);
  x[5] = box_cox(I);
  x[6] = rho;
}

/* RRS factor at a vertex: StatNet, then RRSNet with the modified softplus output (Eq. 22). */
double or_nrrs_factor(const double* Ps, const double* Pr, const double* table, uint32_t log2T, const double* raw,
                      const double* t, double I, double* mv_out, double* z_out) {
  double mv[OR_STAT_OUT], x[OR_RRS_IN], z;
  or_statnet_forward(Ps, table, log2T, raw, mv);
  or_rrs_inputs(mv, t, I, raw[6], x);
  or_mlp32_forward(Pr, OR_RRS_IN, 1, x, &z);
  if (mv_out) {
    mv_out[0] = mv[0];
    mv_out[1] = mv[1];
  }
  if (z_out) *z_out = z;
  return or_softplus_mod(z);
}

/* ------------------------------------------------------------ gradient transfer
 * One-sample estimates of the derivative of the pixel variance with respect to the RRS factor
 * of a sample (Eqs. 17-18): with the prefix weight g/p (the luminance of the vertex's
 * throughput) and the StatNet statistics of the suffix H,
 *   RR (q < 1):         dVar/dq = -(g/p)^2 E[H^2] / q^2,  E[H^2] = v + m^2
 *   splitting (q >= 1): dVar/dq = -(g/p)^2 Var[H] / q^2,  Var[H] = v.
 * The factor the renderer used is q_norm = F q_nrrs (normalization, Eq. 10), so
 * dVar/dq_nrrs = F dVar/dq_norm.  The pixel loss is shared equally by the pixel's k samples,
 * and L_rrs (Eq. 21) adds 2 gamma3 (q_nrrs - sg(q_norm)). */
double or_nrrs_dloss_dq(double wpx, uint32_t k, double lum_t, const double* mv, double q_norm, double F,
                        double q_nrrs, double g_rrs) {
  const double m = mv[0] > 0.0 ? mv[0] : 0.0;
  const double v = mv[1] > 0.0 ? mv[1] : 0.0;
  const double S = q_norm < 1.0 ? v + m * m : v;
  const double dvar = -(lum_t * lum_t) * S / (q_norm * q_norm);
  return (k ? wpx / (double)k : 0.0) * dvar * F + 2.0 * g_rrs * (q_nrrs - q_norm);
}

/* ----------------------------------------------------------------- pixel error
 * Sec. 5 "Tackle Low Spp" and Eqs. (19)-(20).  Per pixel (luminance): the temporal mix
 * acc = (1 - a) acc + a cur (Eq. 23; acc = cur on the first frame), the relative error
 * E'_i = var_scale (acc_i - ref_i)^2 / (ref_i^2 + eps) against the accumulated image of the
 * previous frames ref, a box filter of radius `radius` over the pixels inside the image (in
 * place of the paper's denoiser), E_avg = mean of E, and the derivative of
 * gamma1 L_avg + gamma2 L_min with respect to the pixel variance,
 *   wpx_i = (gamma2 + 2 gamma1 (E_i - E_avg)) / (ref_i^2 + eps).
 * Pixels with ref < 0 (no previous frame) get wpx = 0 and E = 0 and do not enter E_avg. */
double or_nrrs_pixel_weights(const double* cur, double* acc, const double* ref, uint32_t w, uint32_t h,
                             int32_t first, double a_mix, int32_t radius, double var_scale, double g_avg,
                             double g_min, double eps, double* E, double* wpx) {
  const uint64_t npx = (uint64_t)w * h;
  double* Ep = (double*)malloc(sizeof(double) * (npx ? npx : 1));
  for (uint64_t i = 0; i < npx; ++i) {
    acc[i] = first ? cur[i] : (1.0 - a_mix) * acc[i] + a_mix * cur[i];
    Ep[i] = ref[i] < 0.0 ? 0.0 : var_scale * (acc[i] - ref[i]) * (acc[i] - ref[i]) / (ref[i] * ref[i] + eps);
  }
  double sum = 0.0;
  uint64_t cnt = 0;
  for (uint32_t y = 0; y < h; ++y)
    for (uint32_t x = 0; x < w; ++x) {
      const uint64_t i = (uint64_t)y * w + x;
      if (ref[i] < 0.0) {
        E[i] = 0.0;
        continue;
      }
      double s = 0.0;
      int n = 0;
      for (int dy = -radius; dy <= radius; ++dy)
        for (int dx = -radius; dx <= radius; ++dx) {
          const int64_t xx = (int64_t)x + dx, yy = (int64_t)y + dy;
          if (xx < 0 || yy < 0 || xx >= (int64_t)w || yy >= (int64_t)h) continue;
          const uint64_t j = (uint64_t)yy * w + (uint64_t)xx;
          if (ref[j] < 0.0) continue;
          s += Ep[j];
          ++n;
        }
      E[i] = s / n;
      sum += E[i];
      ++cnt;
    }
  const double Eavg = cnt ? sum / (double)cnt : 0.0;
  for (uint64_t i = 0; i < npx; ++i)
    wpx[i] = ref[i] < 0.0 ? 0.0 : (g_min + 2.0 * g_avg * (E[i] - Eavg)) / (ref[i] * ref[i] + eps);
  free(Ep);
  return Eavg;
}

/* ------------------------------------------------------------- RRSNet gradient
 * Step 1 of the schedule (Sec. 5 "Training"): RRSNet is fitted to the output 1 with the
 * relative L2 loss (q - 1)^2 / (1 + eps), averaged over the records.  Step 2: the gradient of
 * Eq. (16) reaches q through or_nrrs_dloss_dq (sums over pixels and samples).  StatNet runs
 * forward only: no gradient flows into it.  Returns the step-1 loss, or the L_rrs term in
 * step 2.  Records with q_norm <= 0 are skipped in step 2. */
double or_rrsnet_nrrs_grad(const double* Pr, const double* Ps, const double* table, uint32_t log2T,
                           const double* raw, const double* t_rgb, const double* I_px, const double* lum_t,
                           const double* q_norm, const double* F, const uint32_t* pix, const uint32_t* k_pix,
                           const double* wpx, uint64_t n, int32_t step, double g_rrs, double eps, double* dPr) {
  double loss = 0.0;
  for (uint64_t r = 0; r < n; ++r) {
    double mv[OR_STAT_OUT], x[OR_RRS_IN], z;
    const double* rr = raw + OR_STAT_RAW * r;
    or_statnet_forward(Ps, table, log2T, rr, mv);
    or_rrs_inputs(mv, t_rgb + 3 * r, I_px[r], rr[6], x);
    or_mlp32_forward(Pr, OR_RRS_IN, 1, x, &z);
    const double q = or_softplus_mod(z);
    double dq;
    if (step == 1) {
      loss += (q - 1.0) * (q - 1.0) / (1.0 + eps);
      dq = 2.0 * (q - 1.0) / (1.0 + eps) / (double)n;
    } else {
      if (!(q_norm[r] > 0.0)) continue;
      loss += g_rrs * (q - q_norm[r]) * (q - q_norm[r]);
      dq = or_nrrs_dloss_dq(wpx[pix[r]], k_pix[pix[r]], lum_t[r], mv, q_norm[r], F[r], q, g_rrs);
    }
    const double dz = dq * or_softplus_mod_grad(z);
    or_mlp32_backward(Pr, OR_RRS_IN, 1, x, &dz, dPr, NULL);
  }
  return step == 1 ? (n ? loss / (double)n : 0.0) : loss;
}

/* ------------------------------------------------------------- RRSNet (AID-NRRS variant)
 * Sec. 4.2.1 and Sec. 5 "Input Encoding": RRSNet reads the vertex itself instead of StatNet's
 * statistics, through an input module of its own: a hash grid of p (same shape as StatNet's,
 * separate trainable table) (16), one-blob of w_o's spherical coordinates with 4 bins each (8),
 * Box-Cox of the throughput (3) and of the pixel value (1), one-blob of the remapped roughness
 * with 4 bins (4): 32 inputs -> 32 -> 32 -> 32 -> 1, modified softplus.  StatNet only
 * supervises: its statistics enter the gradient transfer, not the factor. */
void or_aid_encode(const double* table, uint32_t log2T, const double* raw, const double* t, double I, double* enc) {
  or_hashgrid_encode(table, log2T, raw, enc);
  double wz = raw[5];
  if (wz > 1.0) wz = 1.0;
  if (wz < -1.0) wz = -1.0;
  or_oneblob(acos(wz) / M_PI, 4, enc + 16);
  or_oneblob(atan2(raw[4], raw[3]) / (2.0 * M_PI) + 0.5, 4, enc + 20);
  enc[24] = box_cox(t[0]);
  enc[25] = box_cox(t[1]);
  enc[26] = box_cox(t[2]);
  enc[27] = box_cox(I);
  or_oneblob(raw[6], 4, enc + 28);
}

double or_aid_factor(const double* Pa, const double* table, uint32_t log2T, const double* raw, const double* t,
                     double I, double* z_out) {
  double enc[OR_AID_IN], z;
  or_aid_encode(table, log2T, raw, t, I, enc);
  or_mlp32_forward(Pa, OR_AID_IN, 1, enc, &z);
  if (z_out) *z_out = z;
  return or_softplus_mod(z);
}

/* AID-NRRS RRSNet gradient: as or_rrsnet_nrrs_grad (step 1 toward 1, step 2 the transfer of
 * Eqs. 17-18 with StatNet's statistics), into the MLP (dPa) and its own hash grid (dtable). */
double or_aid_grad(const double* Pa, const double* table_r, const double* Ps, const double* table_s, uint32_t log2T,
                   const double* raw, const double* t_rgb, const double* I_px, const double* lum_t,
                   const double* q_norm, const double* F, const uint32_t* pix, const uint32_t* k_pix,
                   const double* wpx, uint64_t n, int32_t step, double g_rrs, double eps, double* dPa,
                   double* dtable_r) {
  double loss = 0.0;
  for (uint64_t r = 0; r < n; ++r) {
    const double* rr = raw + OR_STAT_RAW * r;
    double enc[OR_AID_IN], denc[OR_AID_IN], z;
    or_aid_encode(table_r, log2T, rr, t_rgb + 3 * r, I_px[r], enc);
    or_mlp32_forward(Pa, OR_AID_IN, 1, enc, &z);
    const double q = or_softplus_mod(z);
    double dq;
    if (step == 1) {
      loss += (q - 1.0) * (q - 1.0) / (1.0 + eps);
      dq = 2.0 * (q - 1.0) / (1.0 + eps) / (double)n;
    } else {
      if (!(q_norm[r] > 0.0)) continue;
      double mv[OR_STAT_OUT];
      or_statnet_forward(Ps, table_s, log2T, rr, mv);
      loss += g_rrs * (q - q_norm[r]) * (q - q_norm[r]);
      dq = or_nrrs_dloss_dq(wpx[pix[r]], k_pix[pix[r]], lum_t[r], mv, q_norm[r], F[r], q, g_rrs);
    }
    const double dz = dq * or_softplus_mod_grad(z);
    or_mlp32_backward(Pa, OR_AID_IN, 1, enc, &dz, dPa, denc);
    if (dtable_r) or_hashgrid_backward(log2T, rr, denc, dtable_r);
  }
  return step == 1 ? (n ? loss / (double)n : 0.0) : loss;
}
