// Host-side launchers of the gfx950 kernels (one translation unit per kernel family).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bvh_layout.hpp"
#include "device_common.hpp"

namespace nrrs {

// Values that change from pass to pass live on the device so that a captured pass can be
// replayed as is: k_begin_pass advances them at the start of every pass.
struct PassState {
  uint32_t pass;   // pass index keying the random numbers
  uint32_t pad;
  double spp;      // samples per pixel accumulated in the image after this pass
};

// Everything the per-depth kernels read about the render in progress.

struct RenderArgs {
  DevScene sc;
  Queue qin, qout;
  float4* hit;        // per slot: t, b1, b2, triangle (BVH index) bits
  float4* vpos;       // per slot: hit point, triangle bits
  float4* vnrm;       // per slot: face-forwarded normal, material bits
  float* q;           // per slot: raw RRS factor (0 = no children)
  uint32_t* offs;     // per slot: first child slot
  double* partial;    // [kScanBlocks] FP64 partial sums of q
  uint32_t* bsum;     // [kScanBlocks] children per block
  uint32_t* boff;     // [kScanBlocks] exclusive scan of bsum
  uint32_t* gsum;     // [kScanBlocks * kGuardSteps] guard candidate counts
  DepthCtl* ctl;      // [max_depth + 2]
  double* alpha;      // persistent adaptive-rate alpha
  uint32_t* overflow; // set when no guard candidate fits
  unsigned long long* rays;  // [3] rays traced, BVH nodes visited, triangles tested (accumulated)
  double* image;      // [npx * 3] FP64 radiance sums
  const float* guide; // [npx] luminance of the previous mean (negative = none)
  double* trace;      // [nprim][trace_depth][3] radiance per primary path and depth, or null
  uint32_t trace_depth;
  Records rec;
  uint2 key;
  uint32_t width, height, nprim, cap, depth, max_depth, pass, mode, norm_mode, net_max_depth;
  uint32_t records_on;
  float p_train;
  double f_rate;
  double budget_base;   // N_px of Eq. (10): primary paths of the pass
  const double* F_fixed;  // test entry point: normalization factor per depth given by the caller
                          // (used as is in place of Eqs. 10-14), or null: computed
  uint32_t* dbg_parent; // when set, the expansion also writes each child's parent index
  uint32_t* spill;      // traversal stack spill area [spill depth][trace_blocks * threads]
  uint32_t* work;       // traversal claim counters [max_depth + 2][kWorkSlices][kWorkStride]
  uint32_t trace_blocks;  // persistent traversal grid (blocks)
  uint32_t ext_variant;   // 0: leaves intersected at once, 1: leaves parked and batched per wave
  uint32_t ext_refill;    // idle lanes (1..64) at which a traversal wave fetches new rays
  uint32_t ext_leaf_batch;  // parked leaves (1..64) at which a wave intersects them (variants 1, 2)
  uint32_t ext_chunk;     // queue entries a traversal wave claims at once (0: just what it needs)
  uint32_t count_work;    // 1: the traversal also counts BVH nodes visited and triangles tested
  uint32_t nee;           // 1: next-event estimation (shadow rays through the traversal kernel)
  uint32_t* work_nee;     // the shadow rays' claim counters (shape of work)
  PassState* pass_state;  // pass index and samples per pixel so far (advanced on the device)
};

void launch_camera(const RenderArgs& a, hipStream_t s);
void launch_extend(const RenderArgs& a, hipStream_t s);
void launch_shade(const RenderArgs& a, hipStream_t s);
// Next-event estimation of one depth after launch_shade: the shadow rays shade wrote into the
// out-queue slots (origin, direction, contribution, shortened light distance) traced by the
// traversal kernel, then the unoccluded contributions added to image, records and paths.
void launch_nee(const RenderArgs& a, hipStream_t s);
void launch_record_features(const RenderArgs& a, uint64_t records_cap, hipStream_t s);  // after shade, same depth
void launch_fixed_factor(const RenderArgs& a, hipStream_t s);  // Mix-Depth fixed rate, after shade
void launch_sum_q(const RenderArgs& a, hipStream_t s);
void launch_roulette(const RenderArgs& a, hipStream_t s);  // count, scan, guard, offsets
void launch_expand(const RenderArgs& a, hipStream_t s);
void launch_parents(const RenderArgs& a, hipStream_t s);  // parent map only (test entry point)
void launch_guide(const RenderArgs& a, float* guide, hipStream_t s);
void launch_begin_pass(const RenderArgs& a, double spp_per_pass, hipStream_t s);
void launch_set_pass_state(PassState* ps, uint32_t pass, double spp, hipStream_t s);
void launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s);
void launch_zero_f64(double* p, uint64_t n, hipStream_t s);
void launch_fill_f32(float* p, uint64_t n, float v, hipStream_t s);
void launch_set_f64(double* p, double v, hipStream_t s);
void launch_accumulate_stats(const DepthCtl* ctl, uint32_t max_depth, unsigned long long* n_sum,
                             unsigned long long* s_sum, unsigned long long* r_sum, double* sumq_last,
                             double* f_last, hipStream_t s);

uint32_t extend_blocks_per_cu(uint32_t variant, bool inst);  // inst: the two-level traversal
uint32_t extend_threads_per_block();
uint32_t extend_spill_depth();

// Debug / test launchers.
void launch_philox(const uint4* ctr, uint2 key, uint4* out, uint32_t n, hipStream_t s);

// Network (mlp.hip).
struct NetArgs {
  const float* master;       // FP32 inference parameters
  const uint16_t* bf16;      // BF16 weights (RNE) packed in matrix-core operand order
  const uint8_t* fp8;        // FP8 E4M3 weights packed in matrix-core operand order
  const float* fp8_scale;    // per-layer FP8 weight scales [3]
  int32_t precision;
};
void launch_rrsnet(const RenderArgs& a, const NetArgs& n, hipStream_t s);
void launch_mlp_forward_rows(const float* x, uint32_t n, const NetArgs& net, float* y, float* z, hipStream_t s);
void launch_mlp_grad(const float* x, const float* target, const uint32_t* index, uint32_t n, const float* master,
                     int32_t loss_kind, float* grad_partial, float* loss_partial, uint32_t* nblocks_out,
                     hipStream_t s);
void launch_grad_reduce(const float* grad_partial, uint32_t nblocks, float* grad, const float* loss_partial,
                        float* loss_accum, uint32_t n_rows_total, hipStream_t s);
// Gradient sum (fixed order) + Adam on `master` + infer = decay * infer + (1 - decay) * master
// (decay 0: copy) — the tail of one training step in one launch.
void launch_grad_adam_ema(const float* grad_partial, uint32_t nblocks, float* grad, const float* loss_partial,
                          float* loss_accum, uint32_t n_rows_total, float* master, float* m, float* v, uint64_t step,
                          float lr, float* infer, float decay, hipStream_t s);
void launch_quantize(const float* master, uint16_t* bf16, uint8_t* fp8, float* fp8_scale, hipStream_t s);
void launch_record_targets(const Records& r, float* target, uint32_t n, hipStream_t s);
// Matrix-core inference (mlp_mfma.hip): precision 1 = BF16, 2 = FP8-E4M3.
uint32_t packed_bf16_elems();
uint32_t packed_fp8_bytes();
void launch_pack_weights(const float* master, uint16_t* bf16, uint8_t* fp8, float* fp8_scale, hipStream_t s);
void launch_rrsnet_mfma(const RenderArgs& a, const NetArgs& n, hipStream_t s);
void launch_rows_mfma(const float* x, uint32_t n, const NetArgs& net, float* y, float* z, hipStream_t s);
// Test entry point: also the bit patterns of every quantized layer's values ([n][3][64]: inputs,
// hidden 1, hidden 2) and, for FP8, their block-scale exponents ([n][3]).
void launch_codes_mfma(const float* x, uint32_t n, const NetArgs& net, float* y, uint16_t* codes, int8_t* scale_exp,
                       hipStream_t s);
void warm_mfma_launch_cache();  // occupancy queries done before any stream capture

// NRRS proper (nrrs_net.hip): StatNet and the NRRS variant of RRSNet, both in -> 32 -> 32 -> 32
// -> out with leaky ReLU, and the multiresolution hash grid of StatNet's position input.
constexpr int kHgLevels = 8, kHgFeat = 2, kHgBase = 16;
constexpr int kStatRaw = 7, kStatIn = 32, kStatOut = 2, kRrsIn = 7;
constexpr uint32_t mlp32_params(int in, int out) { return 32u * in + 32u + 2u * (32u * 32u + 32u) + 32u * out + out; }
constexpr uint32_t kStatParams = mlp32_params(kStatIn, kStatOut);  // 3234
constexpr uint32_t kRrsParams = mlp32_params(kRrsIn, 1);           // 2401
constexpr int kAidIn = 32;                                         // AID-NRRS RRSNet inputs
constexpr uint32_t kAidParams = mlp32_params(kAidIn, 1);           // 3201
struct NrrsNet {
  const float* stat;     // StatNet parameters
  const float* rrs;      // RRSNet parameters (NRRS inputs)
  const float* table;    // StatNet's hash grid [kHgLevels][2^log2T][kHgFeat]
  const float* aid;      // RRSNet parameters (AID-NRRS inputs)
  const float* table_r;  // the AID-NRRS RRSNet's own hash grid (same shape)
  uint32_t log2T;
};
// aid = false: StatNet + NRRS RRSNet; true: the AID-NRRS RRSNet alone.
void launch_nrrs_factor(const RenderArgs& a, const NrrsNet& n, uint32_t blocks, bool aid, hipStream_t s);
void launch_aid_rows(const float* raw, const float* t, const float* I, uint32_t n, const NrrsNet& net, float* q,
                     float* enc, hipStream_t s);  // test entry point
void launch_record_qnorm(const RenderArgs& a, hipStream_t s);  // after the roulette of the depth
// Test entry point: StatNet outputs, RRS factor and (optional) StatNet encodings of n vertices.
void launch_nrrs_rows(const float* raw, const float* t, const float* I, uint32_t n, const NrrsNet& net, float* mv,
                      float* q, float* enc, hipStream_t s);
// Training records as the gradient kernels read them (device arrays; n rows).
struct NrrsRows {
  const float* raw;     // [n][8] (stride 8): raw StatNet inputs (7), pixel value I
  const float* lum_t;   // [n]
  const float* acc;     // [n] descendant emission luminance (StatNet target = acc / lum_t), or null
  const float* target;  // [n] StatNet target given directly (used when acc is null)
  const float4* tq;     // [n] throughput rgb
  const float2* qf;     // [n] q_norm, F
  const uint32_t* pix;  // [n]
  uint32_t n;
};
uint32_t nrrs_grad_blocks(uint32_t n);
// StatNet gradient of Eq. (15) (mean over the rows): block partials [blocks][kStatParams], block
// losses, and hash-grid gradients added atomically into gtable (zeroed by the caller).
void launch_statnet_grad(const NrrsRows& r, const float* stat, const float* table, uint32_t log2T, float eps,
                         float* partial, float* loss_part, float* gtable, hipStream_t s);
// RRSNet gradient: step 1 fits the output 1 (mean relative L2); step 2 transfers the pixel
// gradient wpx / k (Eqs. 17-18) and adds the bound loss (Eq. 21).
void launch_rrsnet_grad(const NrrsRows& r, const float* stat, const float* table, uint32_t log2T, const float* rrs,
                        int32_t step, const float* wpx, const uint32_t* kpix, float g_rrs, float eps, float* partial,
                        float* loss_part, hipStream_t s);
// AID-NRRS RRSNet gradient (steps as launch_rrsnet_grad; StatNet's statistics only in step 2):
// block partials [blocks][kAidParams] and its hash-grid gradients added into gtable_r.
void launch_aid_grad(const NrrsRows& r, const float* stat, const float* table, uint32_t log2T, const float* aid,
                     const float* table_r, int32_t step, const float* wpx, const uint32_t* kpix, float g_rrs,
                     float eps, float* partial, float* loss_part, float* gtable_r, hipStream_t s);
// Fixed-order sum of the block partials into grad (through group_sums, scratch of
// nrrs_sum_groups() * np floats), and of the block losses into *loss.
void launch_partial_sum(const float* partial, uint32_t nblocks, uint32_t np, float* grad, const float* loss_part,
                        float* loss, float* group_sums, hipStream_t s);
uint32_t nrrs_sum_groups();
// Adam (bias-corrected, step >= 1) on np parameters, the moving average of the inference copy
// (decay 0: copy) and, when zero_grad, the gradient cleared for the next step.
void launch_adam(float* w, float* m, float* v, float* grad, uint64_t np, uint64_t step, float lr, float* infer,
                 float decay, bool zero_grad, hipStream_t s);
// Pixel error of the frame (Sec. 5 "Tackle Low Spp", Eqs. 19-20, 23): from the luminance of the
// current frame cur and of the previous frames ref (< 0: none) per pixel, with the temporally
// mixed acc updated in place: E (box filter of radius r), E_avg into *eavg (double), and the
// derivative wpx of gamma1 L_avg + gamma2 L_min with respect to the pixel variance.
struct PixelErrArgs {
  const float* cur;
  const float* ref;
  float* acc;
  float* Ep;     // scratch [npx]
  float* E;      // [npx]
  float* wpx;    // [npx]
  double* part;  // scratch [2 * pixel blocks]
  double* eavg;  // [1]
  uint32_t w, h, first;
  int32_t radius;
  float a_mix, var_scale, g_avg, g_min, eps;
};
void launch_pixel_error(const PixelErrArgs& p, hipStream_t s);
// Frame luminances from the FP64 image sums: cur = (lum(image) - lum_start) / spp_frame,
// ref = lum_start / spp_start (or -1 when spp_start = 0); lum_start <- lum(image).
void launch_frame_lum(const double* image, double* lum_start, uint32_t npx, double spp_frame, double spp_start,
                      float* cur, float* ref, hipStream_t s);
// Records per pixel: kpix zeroed, then one count per row.
void launch_count_pix(const uint32_t* pix, uint32_t n, uint32_t* kpix, uint32_t npx, hipStream_t s);
uint32_t mlp_grad_blocks(uint32_t n);
uint32_t mlp_grad_scratch_floats(uint32_t max_rows);  // partials + reduction groups

}  // namespace nrrs
