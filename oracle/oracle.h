/* FP64 CPU oracle of the normalized-RRS wavefront path tracer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP path: everything here (random numbers, intersection, sampling,
 * normalization, roulette, network) is written separately from the paper's
 * definitions, in double precision, with plain loops.
 *
 * Paper references (NRRS, arXiv 2510.07868):
 *   rendering equation / MC estimator          Sec. 3, Eqs. (1)-(2)
 *   stochastic rounding of the RRS factor      Sec. 3, Eq. (8)
 *   wavefront stages, terminate on light/miss  Sec. 3, "Wavefront Architecture"
 *   per-depth normalization                    Sec. 4.1.2, Eqs. (9)-(11)
 *   rate control / adaptive alpha              Sec. 4.1.4, Eqs. (12)-(14)
 *   downscale-only compromise                  Sec. 5, "Compromise"
 *   modified softplus output                   Sec. 5, Eq. (22)
 *   Box-Cox / roughness remap input encodings  Sec. 5, "Input Encoding"
 *   ADRRS ratio for q                          Sec. 2.2 (ADRRS paragraph)
 */
#ifndef NRRS_ORACLE_H
#define NRRS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_NPARAM 9729   /* 20-64-64-64-1 MLP */
#define OR_STAT_NPARAM 3234 /* StatNet: 32 -> 32 -> 32 -> 32 -> 2 */
#define OR_RRS_NPARAM 2401  /* RRSNet (NRRS): 7 -> 32 -> 32 -> 32 -> 1 */
#define OR_AID_NPARAM 3201  /* RRSNet (AID-NRRS): 32 -> 32 -> 32 -> 32 -> 1 */
#define OR_NFEAT 20
#define OR_MAXD 64

enum { OR_MODE_OFF = 0, OR_MODE_HEUR = 1, OR_MODE_NET = 2, OR_MODE_NRRS = 3, OR_MODE_AID = 4 };
enum { OR_NORM_TWO_SIDED = 0, OR_NORM_DOWNSCALE = 1 };

typedef struct or_scene or_scene;

typedef struct {
  uint32_t width, height, s_batch, max_depth;
  uint32_t pass_begin, n_passes;
  int32_t mode, norm_mode, net_max_depth, frozen;
  double cap_factor, f_rate;
  uint64_t seed;
  double alpha;          /* in: adaptive rate alpha; out: value after the render */
  double p_train;        /* probability that a primary path records training vertices */
  uint32_t rec_cap;      /* capacity of the record arrays (0 = no records) */
  uint32_t update_guide; /* 1: refresh the guide image from the running mean after each pass */
  double tau;            /* near-tie margin for the fragile-pixel flags */
  uint64_t net_depths;   /* Mix-Depth table (Sec. 4.3): NET mode evaluates the network at depth d
                            when bit d-1 is set and keeps the heuristic factor at the other depths */
  uint64_t fixed_depths; /* Mix-Depth's fixed rate: at depth d with bit d-1 set every vertex that
                            continues gets the raw factor 1 (HEUR and NET modes; before the network) */
  uint32_t hash_log2;    /* NRRS mode (Sec. 4.2): params = StatNet (OR_STAT_NPARAM), RRSNet
                            (OR_RRS_NPARAM) and the hash grid [8][2^hash_log2][2], concatenated; the
                            NRRS factor replaces the heuristic at the depths of net_depths; AID mode:
                            params = the AID-NRRS RRSNet (OR_AID_NPARAM) and its hash grid */
  uint32_t nee;          /* 1: next-event estimation at every vertex that may continue (one light
                            sample, shadow ray, power-heuristic MIS with the BSDF-sampled hits) */
} or_cfg;

typedef struct {
  uint64_t n[OR_MAXD + 1];        /* queue entries entering extend at depth d (summed over passes) */
  uint64_t active[OR_MAXD + 1];   /* entries with q > 0 */
  uint64_t S[OR_MAXD + 1];        /* children emitted at depth d (summed) */
  uint64_t retries[OR_MAXD + 1];  /* overflow-guard retries */
  double sumq[OR_MAXD + 1];       /* last pass: FP64 sum of q_orig */
  double F[OR_MAXD + 1];          /* last pass: normalization factor */
  uint64_t rays;                  /* rays traced (non-dead entries extended) */
  uint64_t n_records;             /* records written (<= rec_cap) */
  int32_t status;                 /* 0 ok, -5 alpha fell below 1e-3 */
} or_stats;

/* Scene from the generator's arrays; build_bvh=0 forces brute-force closest hit. */
or_scene* or_scene_create(const float* verts, uint64_t nv, const uint32_t* tris, uint64_t nt,
                          const uint32_t* tri_mat, const uint32_t* mat_type, const float* mat_params,
                          uint32_t nm, const float* camera, const float* env, int32_t build_bvh);
void or_scene_destroy(or_scene* s);

/* Philox4x32-10 (Salmon et al., SC'11). */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_philox_batch(const uint32_t* ctr, const uint32_t key[2], uint64_t n, uint32_t* out);

/* Closest hit for n rays (origin xyz, dir xyz, exclude prim) -> prim (0xffffffff = miss), t, b1, b2.
 * fragile[i] (may be NULL) flags decisions within tau of changing (near-ties). */
void or_trace(const or_scene* s, const double* rays, const uint32_t* exclude, uint64_t n,
              uint32_t* prim, double* t, double* b1, double* b2, int32_t use_bvh, double tau,
              uint8_t* fragile);

/* Normalization + roulette + exclusive scan on a host array of q_orig (Eqs. 8-14).
 * Outputs X, offsets, parent_of_child[S], S, F, q_norm (FP32 values as doubles),
 * the alpha after the overflow guard and the retry count.  u[i] are the uniforms.
 * Returns 0, or -5 when alpha falls below 1e-3. */
int32_t or_rrs_expand(const double* q_orig, const double* u, uint64_t n, double budget_base,
                      double f_rate, double* alpha, int32_t norm_mode, uint64_t cap,
                      uint32_t* X, uint64_t* offset, uint32_t* parent_of_child, uint64_t* S,
                      double* F, float* q_norm, uint32_t* retries);

/* Full render: accumulates radiance sums into image[W*H*3] (not divided by spp).
 * Optional per-path outputs (may be NULL): path_rgb[nprim][max_depth][3] accumulates the
 * radiance that primary path k of a pass (sample k mod s_batch of pixel k / s_batch) and its
 * split descendants collect at each vertex depth (summed over passes); path_first[nprim] is
 * the smallest depth whose radiance a near-tie decision of the path or a descendant may
 * change (max_depth + 1 = none). */
int32_t or_render(const or_scene* s, or_cfg* cfg, const double* params, double* guide,
                  double* image, uint8_t* fragile, or_stats* stats,
                  double* rec_feat, double* rec_lumt, double* rec_acc, uint32_t* rec_depth,
                  uint32_t* rec_pix, uint64_t* rec_id, double* path_rgb, uint8_t* path_first);

/* Exhaustive expectation over all roulette outcomes with frozen continuous samples
 * (every child of a vertex reuses the sample of child 0).  Writes the outcome-weighted
 * mean image of one pass and the OFF-mode image on the same samples.  Also returns the
 * largest S seen on any branch and the number of branches.  Optional (may be NULL):
 * pmf_S[(max_depth + 1) * (C + 2)] with C = floor(cap_factor * nprim): the probability that
 * depth d emits S children (entry d * (C + 2) + S; S > C goes to entry C + 1);
 * live[max_depth + 1]: the probability that depth d has a positive factor sum;
 * q_norm1[nprim]: the float32 normalized factors of depth 1 (a single branch). */
int32_t or_enumerate(const or_scene* s, const or_cfg* cfg, double* image_expect, double* image_off,
                     uint64_t* max_S, uint64_t* branches, double* pmf_S, double* live, float* q_norm1);

/* Network (Sec. 5): 20 -> 64 -> 64 -> 64 (ReLU) -> 1, modified softplus output. */
void or_mlp_forward(const double* params, const double* x, uint64_t n, double* y, double* z);
/* The same network evaluated with the quantization of the matrix-core paths (test reading):
 * prec 1: weights, inputs and hidden activations rounded to bfloat16 (ties to even);
 * prec 2: weights as OCP E4M3 with one scale per layer (amax / 448), inputs and hidden
 *         activations as E4M3 with one power-of-two scale per vertex and layer (the smallest
 *         2^e >= amax / 448).  Arithmetic otherwise in double.
 * fragile[r] (may be NULL) flags rows where a hidden activation lies within 2e-4 (BF16) or
 * 5e-5 (E4M3) grid steps of
 * a rounding midpoint (or the scale choice is near a power of two): a float32 evaluation may
 * round those the other way. */
double or_round_bf16(double x);
double or_round_e4m3(double x);
/* Bound on the distance of an FP8 matrix-core dot product of E4M3 codes w[n], x[n] from its
 * exact value (the near-tie margin of the FP8 quantized forward). */
double or_fp8_dot_error_bound(const double* w, const double* x, int32_t n);
void or_mlp_forward_quant(const double* params, const double* x, uint64_t n, int32_t prec, double* y, double* z,
                          uint8_t* fragile);
/* As or_mlp_forward_quant, also giving per row (each may be NULL): codes[192] = the bit
 * patterns (E4M3 in the low byte, or BF16) of the quantized inputs (0..19) and of the two
 * quantized hidden layers (64..127, 128..191); near_act[192] = 1 where that activation's
 * rounding, or its layer's power-of-two scale, is a near-tie; scale_exp[3] = the FP8 block
 * scale exponent of the inputs and of each hidden layer. */
void or_mlp_forward_quant_codes(const double* params, const double* x, uint64_t n, int32_t prec, double* y,
                                double* z, uint8_t* fragile, uint16_t* codes, uint8_t* near_act, int8_t* scale_exp);

/* Training losses of the radiance estimate y against the one-sample target L:
 *   OR_LOSS_REL_L2:  mean((y - L)^2 / (sg(y)^2 + eps)), the relative L2 of Sec. 4.2.2 (Eq. 15)
 *                    with the prediction held constant in the denominator (its minimiser is the
 *                    mean of L);
 *   OR_LOSS_LOG_MSE: mean((ln(y + eps) - ln(L + eps))^2).
 * Returns the loss and writes the gradient w.r.t. all parameters. */
enum { OR_LOSS_REL_L2 = 0, OR_LOSS_LOG_MSE = 1 };
double or_mlp_loss_grad(const double* params, const double* x, const double* target, uint64_t n,
                        double eps, int32_t kind, double* grad);
void or_adam(double* params, double* m, double* v, const double* grad, uint64_t np, uint64_t step,
             double lr, double b1, double b2, double eps);
double or_softplus_mod(double z);
int32_t or_num_threads(void);
double or_softplus_mod_grad(double z);

/* BSDF helpers exposed for the closed-form pins.  Directions are in the local frame (n = +z). */
double or_ggx_D(double alpha, const double h[3]);
double or_ggx_G1(double alpha, const double w[3]);
double or_ggx_G2(double alpha, const double wo[3], const double wi[3]);
/* Sample: returns 1 if wi is above the surface; w_out = f*cos/pdf (scalar F0 channel). */
int32_t or_ggx_sample(double alpha, double f0, const double wo[3], double u1, double u2,
                      double wi[3], double* weight, double* pdf);
double or_ggx_eval_cos(double alpha, double f0, const double wo[3], const double wi[3]);
/* Solid-angle pdf of the visible-normal sampling of or_ggx_sample for the direction wi. */
double or_ggx_pdf(double alpha, const double wo[3], const double wi[3]);
void or_lambert_sample(double u1, double u2, double wi[3], double* pdf);

/* ------------------------------------------------ NRRS training proper (nrrs_train.c)
 * StatNet and the NRRS variant of RRSNet (Sec. 4.2.1), their losses (Sec. 4.2.2, Eqs. 15-21)
 * and encodings (Sec. 5).  Records: raw[7] = position in the scene box scaled to [0, 1]^3,
 * unit outgoing direction w_o (world), remapped roughness 1 - exp(-alpha). */
#define OR_HG_LEVELS 8
#define OR_HG_FEAT 2
#define OR_HG_BASE 16
#define OR_STAT_RAW 7
#define OR_STAT_IN 32   /* 16 hash grid + 8 one-blob direction + 8 one-blob roughness */
#define OR_STAT_OUT 2   /* luminance mean and variance of the reflected radiance */
#define OR_RRS_IN 7     /* Box-Cox of m, E[L^2], t (RGB), I; remapped roughness */
void or_oneblob(double s, int32_t bins, double* out);
void or_hashgrid_encode(const double* table, uint32_t log2T, const double* p, double* out);
void or_hashgrid_backward(uint32_t log2T, const double* p, const double* dout, double* dtable);
double or_hashgrid_cell_margin(const double* p);
void or_statnet_encode(const double* table, uint32_t log2T, const double* raw, double* enc);
uint64_t or_mlp32_nparams(int32_t in, int32_t out);
void or_mlp32_forward(const double* P, int32_t in, int32_t out, const double* x, double* y);
void or_mlp32_backward(const double* P, int32_t in, int32_t out, const double* x, const double* dy, double* dP,
                       double* dx);
void or_statnet_forward(const double* P, const double* table, uint32_t log2T, const double* raw, double* mv);
double or_statnet_loss_grad(const double* P, const double* table, uint32_t log2T, const double* raw,
                            const double* target, uint64_t n, double eps, double* dP, double* dtable);
void or_rrs_inputs(const double* mv, const double* t, double I, double rho, double* x);
double or_nrrs_factor(const double* Ps, const double* Pr, const double* table, uint32_t log2T, const double* raw,
                      const double* t, double I, double* mv_out, double* z_out);
double or_nrrs_dloss_dq(double wpx, uint32_t k, double lum_t, const double* mv, double q_norm, double F,
                        double q_nrrs, double g_rrs);
double or_nrrs_pixel_weights(const double* cur, double* acc, const double* ref, uint32_t w, uint32_t h,
                             int32_t first, double a_mix, int32_t radius, double var_scale, double g_avg,
                             double g_min, double eps, double* E, double* wpx);
#define OR_AID_IN 32    /* AID-NRRS RRSNet inputs: 16 hash grid + 8 one-blob w_o + 4 Box-Cox + 4 one-blob */
void or_aid_encode(const double* table, uint32_t log2T, const double* raw, const double* t, double I, double* enc);
double or_aid_factor(const double* Pa, const double* table, uint32_t log2T, const double* raw, const double* t,
                     double I, double* z_out);
double or_aid_grad(const double* Pa, const double* table_r, const double* Ps, const double* table_s, uint32_t log2T,
                   const double* raw, const double* t_rgb, const double* I_px, const double* lum_t,
                   const double* q_norm, const double* F, const uint32_t* pix, const uint32_t* k_pix,
                   const double* wpx, uint64_t n, int32_t step, double g_rrs, double eps, double* dPa,
                   double* dtable_r);
double or_rrsnet_nrrs_grad(const double* Pr, const double* Ps, const double* table, uint32_t log2T,
                           const double* raw, const double* t_rgb, const double* I_px, const double* lum_t,
                           const double* q_norm, const double* F, const uint32_t* pix, const uint32_t* k_pix,
                           const double* wpx, uint64_t n, int32_t step, double g_rrs, double eps, double* dPr);

#ifdef __cplusplus
}
#endif
#endif
