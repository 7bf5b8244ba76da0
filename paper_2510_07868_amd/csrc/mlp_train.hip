// Training gradient of the RRS network on the gfx950 FP32 matrix cores (v_mfma_f32_32x32x2_f32):
// forward, loss, backward and the weight gradients of one minibatch (Sec. 5 "Training"),
// with the statistic loss of Eq. (15) (relative L2, prediction in the denominator held
// constant) or the squared error of log radiance.
//
// Layout.  A wave owns 32 rows and keeps every activation "units x rows": in the 32x32 MFMA
// accumulator, lane l holds row l % 32 and 16 units per 32-unit tile, unit
// 8 (v / 4) + 4 (l / 32) + v % 4 of register v.  A layer's output registers are the next
// product's B operand unchanged: the K order of that product follows the same unit order,
// and the weights are read from LDS in that order.  The weight gradients (K = rows) need units
// along the lanes instead, so deltas and activations go through a padded LDS transpose.  For
// the weight gradients each of the four waves owns one 32x32 output tile and runs K over the
// rows of all four waves in order; bias sums are per-wave partials added in wave order.  The
// block writes one partial gradient; partials are summed in a fixed order, so results are
// deterministic.
#include <algorithm>
#include <cmath>

#include "launch.hpp"

namespace nrrs {

namespace {

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kTWaves = 4;
constexpr int kTThreads = 64 * kTWaves;
constexpr int kTRows = 32 * kTWaves;     // rows per block
constexpr int kS1 = 21, kS2 = 65, kST = 33;  // padded LDS row strides (distinct banks per lane)
constexpr int kRedGroups = 16;           // first-level groups of the partial-gradient sum

// LDS carve (floats)
constexpr int kOffW1 = 0;                         // W1 [64][kS1]
constexpr int kOffW2 = kOffW1 + 64 * kS1;         // W2 [64][kS2]
constexpr int kOffW3 = kOffW2 + 64 * kS2;         // W3 [64][kS2]
constexpr int kOffB = kOffW3 + 64 * kS2;          // b1, b2, b3, w4 [64 each], b4
constexpr int kOffScratch = kOffB + 4 * 64 + 4;   // per wave: X [32][kS1], D [64][kST], H [64][kST]
constexpr int kWaveScratch = 32 * kS1 + 2 * 64 * kST;
constexpr int kOffBias = kOffScratch + kTWaves * kWaveScratch;  // per-wave bias sums [kTWaves][kBiasPart]
constexpr int kBiasPart = 4 * 64 + 4;                            // b3, w4, b2, b1 [64 each], b4
constexpr int kOffRow = kOffBias + kTWaves * kBiasPart;          // per-row loss and dz [2][kTRows]
static_assert(kTWaves == 4, "one 32x32 weight-gradient tile per wave");
constexpr int kLdsFloats = kOffRow + 2 * kTRows;

__device__ __forceinline__ float softplus_mod(float z) { return z < 0.0f ? log1pf(expf(z)) : 0.5f * z + 0.69314718055994531f; }
__device__ __forceinline__ float softplus_mod_grad(float z) { return z < 0.0f ? 1.0f / (1.0f + expf(-z)) : 0.5f; }

// hidden unit held by register v of tile t in lane half h
__device__ __forceinline__ int unit_of(int t, int v, int h) { return 32 * t + 8 * (v >> 2) + 4 * h + (v & 3); }

// LDS offset (floats) of parameter p; four consecutive parameters starting at a multiple of 4
// stay in one row of one section, so they land at consecutive offsets.
__device__ __forceinline__ int param_lds(int p) {
  static_assert(kB1 % 4 == 0 && kW2 % 4 == 0 && kB2 % 4 == 0 && kW3 % 4 == 0 && kB3 % 4 == 0 && kW4 % 4 == 0 &&
                    kB4 % 4 == 0 && kW4 == kB3 + 64 && kB4 == kW4 + 64,
                "parameter sections not float4-aligned");
  if (p < kB1) return kOffW1 + (p / 20) * kS1 + p % 20;
  if (p < kW2) return kOffB + (p - kB1);
  if (p < kB2) return kOffW2 + ((p - kW2) >> 6) * kS2 + ((p - kW2) & 63);
  if (p < kW3) return kOffB + 64 + (p - kB2);
  if (p < kB3) return kOffW3 + ((p - kW3) >> 6) * kS2 + ((p - kW3) & 63);
  return kOffB + 128 + (p - kB3);  // b3, w4, b4
}

__device__ __forceinline__ f32x16 mfma(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// out = W x (units x rows) for a 64-unit input held as registers in[32] (tile-major), weights
// W[o][i] at Ws[o * ld + i]; `transposed` reads W[i][o] instead (the backward product W^T d).
__device__ __forceinline__ void layer64(const float* Ws, int ld, bool transposed, const float (&in)[32], int h,
                                        int c, f32x16 (&acc)[2]) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f32x16 r = {};
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const int k = unit_of(s >> 4, s & 15, h);
      const int o = 32 * t + c;
      const float a = transposed ? Ws[k * ld + o] : Ws[o * ld + k];
      r = mfma(a, in[s], r);
    }
    acc[t] = r;
  }
}

// One 32x32 tile of a weight gradient, dW[32 mt + m][32 nt + n] = sum_r D[.][r] H[.][r] over the
// rows of all waves of the block (wave w's D and H at scratch + w * kWaveScratch, as
// [unit][kST]; H = X rows-major [row][kS1] when `x_input`), K in wave-then-row order.
template <bool x_input>
__device__ __forceinline__ f32x16 weight_grad_tile(const float* scratch, int mt, int nt, int h, int c) {
  f32x16 r = {};
#pragma unroll
  for (int w = 0; w < kTWaves; ++w) {
    const float* X = scratch + w * kWaveScratch;
    const float* D = X + 32 * kS1;
    const float* H = D + 64 * kST;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int rr = 2 * s + h;
      const float b = x_input ? (c < 20 ? X[rr * kS1 + c] : 0.0f) : H[(32 * nt + c) * kST + rr];
      r = mfma(D[(32 * mt + c) * kST + rr], b, r);
    }
  }
  return r;
}

__global__ __launch_bounds__(kTThreads) void k_mlp_grad_mfma(const float* x, const float* target,
                                                            const uint32_t* index, uint32_t n, uint32_t n_total,
                                                            const float* master, int32_t loss_kind,
                                                            float* grad_partial, float* loss_partial) {
  extern __shared__ float lds[];
  float* W1s = lds + kOffW1;
  float* W2s = lds + kOffW2;
  float* W3s = lds + kOffW3;
  float* Bs = lds + kOffB;  // b1 [0,64), b2 [64,128), b3 [128,192), w4 [192,256), b4 [256]
  float* BiasPart = lds + kOffBias;
  float* RowLoss = lds + kOffRow;
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, h = l >> 5, c = l & 31;
  {
    // every parameter but b4 as float4 (all section boundaries are multiples of 4), loads
    // issued together before the LDS stores
    constexpr int kVec = (kNParam - 1) / 4;
    constexpr int kPer = (kVec + kTThreads - 1) / kTThreads;
    const float4* m4 = reinterpret_cast<const float4*>(master);
    float4 wv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + j * kTThreads;
      wv[j] = q < kVec ? m4[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + j * kTThreads;
      if (q < kVec) {
        float* dst = lds + param_lds(4 * q);
        dst[0] = wv[j].x;
        dst[1] = wv[j].y;
        dst[2] = wv[j].z;
        dst[3] = wv[j].w;
      }
    }
    if (tid == 0) Bs[256] = master[kB4];
  }
  float* Xs = lds + kOffScratch + wave * kWaveScratch;  // [32 rows][kS1]
  float* Ds = Xs + 32 * kS1;                            // [64 units][kST]
  float* Hs = Ds + 64 * kST;                            // [64 units][kST]
  const uint32_t row = blockIdx.x * kTRows + wave * 32 + c;
  const bool valid = row < n;
  const uint32_t src = valid ? (index ? index[row] : row) : 0u;
  float xf[10];
#pragma unroll
  for (int s = 0; s < 10; ++s) {
    xf[s] = valid ? x[20ull * src + 2 * s + h] : 0.0f;
    Xs[c * kS1 + 2 * s + h] = xf[s];
  }
  __syncthreads();

  // ---- forward: H1, H2 (post-ReLU), H3
  f32x16 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f32x16 r = {};
#pragma unroll
    for (int s = 0; s < 10; ++s) r = mfma(W1s[(32 * t + c) * kS1 + 2 * s + h], xf[s], r);
    acc[t] = r;
  }
  float H1[32], H2[32], H3[32];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) H1[16 * t + v] = fmaxf(acc[t][v] + Bs[unit_of(t, v, h)], 0.0f);
  layer64(W2s, kS2, false, H1, h, c, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) H2[16 * t + v] = fmaxf(acc[t][v] + Bs[64 + unit_of(t, v, h)], 0.0f);
  layer64(W3s, kS2, false, H2, h, c, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) H3[16 * t + v] = fmaxf(acc[t][v] + Bs[128 + unit_of(t, v, h)], 0.0f);

  // ---- output, loss, dL/dz per row
  float zp = 0.0f;
#pragma unroll
  for (int s = 0; s < 32; ++s) zp = fmaf(Bs[192 + unit_of(s >> 4, s & 15, h)], H3[s], zp);
  const float z = zp + __shfl_xor(zp, 32) + Bs[256];
  float dz = 0.0f, ls = 0.0f;
  if (valid) {
    const float y = softplus_mod(z);
    const float L = target[src];
    float dy;
    if (loss_kind == 1) {  // squared error of log radiance
      const float diff = logf(y + 0.01f) - logf(L + 0.01f);
      ls = diff * diff;
      dy = 2.0f * diff / (y + 0.01f);
    } else {               // relative L2 with the prediction held constant in the denominator
      const float den = y * y + 0.01f;
      const float diff = y - L;
      ls = diff * diff / den;
      dy = 2.0f * diff / den;
    }
    dz = dy / (float)n_total * softplus_mod_grad(z);
  }
  if (h == 0) {
    RowLoss[wave * 32 + c] = ls;
    RowLoss[kTRows + wave * 32 + c] = dz;
  }

  // ---- layer 3 delta, output-layer gradients (dW4 = sum_r dz H3, db4 = sum_r dz)
  float D[32];
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    const int u = unit_of(s >> 4, s & 15, h);
    D[s] = H3[s] > 0.0f ? dz * Bs[192 + u] : 0.0f;
    Hs[u * kST + c] = H3[s] * dz;
    Ds[u * kST + c] = D[s];
  }
  __syncthreads();
  // lane u sums its unit over the wave's 32 rows: dW4[u], db3[u]
  float gw4 = 0.0f, gb3 = 0.0f, gb4 = 0.0f;
  for (int r = 0; r < 32; ++r) {
    gw4 += Hs[l * kST + r];
    gb3 += Ds[l * kST + r];
    gb4 += RowLoss[kTRows + wave * 32 + r];
  }
  __syncthreads();
  float* bp = BiasPart + wave * kBiasPart;
  bp[l] = gb3;
  bp[64 + l] = gw4;
  if (l == 0) bp[256] = gb4;
  float* gp = grad_partial + (uint64_t)blockIdx.x * kNParam;
  const int mt = wave >> 1, nt = wave & 1;  // this wave's weight-gradient tile
  // dW3 = D3 H2^T
#pragma unroll
  for (int s = 0; s < 32; ++s) Hs[unit_of(s >> 4, s & 15, h) * kST + c] = H2[s];
  __syncthreads();
  f32x16 g = weight_grad_tile<false>(lds + kOffScratch, mt, nt, h, c);
  // D2 = (W3^T D3) * relu'(H2)
  layer64(W3s, kS2, true, D, h, c, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) D[16 * t + v] = H2[16 * t + v] > 0.0f ? acc[t][v] : 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) gp[kW3 + 64 * unit_of(mt, v, h) + 32 * nt + c] = g[v];
  __syncthreads();
  // ---- layer 2: dW2 = D2 H1^T, db2, D1 = (W2^T D2) * relu'(H1)
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    const int u = unit_of(s >> 4, s & 15, h);
    Ds[u * kST + c] = D[s];
    Hs[u * kST + c] = H1[s];
  }
  __syncthreads();
  float gb2 = 0.0f;
  for (int r = 0; r < 32; ++r) gb2 += Ds[l * kST + r];
  bp[128 + l] = gb2;
  g = weight_grad_tile<false>(lds + kOffScratch, mt, nt, h, c);
  layer64(W2s, kS2, true, D, h, c, acc);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) D[16 * t + v] = H1[16 * t + v] > 0.0f ? acc[t][v] : 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) gp[kW2 + 64 * unit_of(mt, v, h) + 32 * nt + c] = g[v];
  __syncthreads();
  // ---- layer 1: dW1 = D1 X^T (20 inputs in one 32-wide tile, waves 0 and 1), db1
#pragma unroll
  for (int s = 0; s < 32; ++s) Ds[unit_of(s >> 4, s & 15, h) * kST + c] = D[s];
  __syncthreads();
  float gb1 = 0.0f;
  for (int r = 0; r < 32; ++r) gb1 += Ds[l * kST + r];
  bp[192 + l] = gb1;
  if (wave < 2) {
    g = weight_grad_tile<true>(lds + kOffScratch, wave, 0, h, c);
    if (c < 20) {
#pragma unroll
      for (int v = 0; v < 16; ++v) gp[kW1 + 20 * unit_of(wave, v, h) + c] = g[v];
    }
  }
  __syncthreads();
  // biases: per-wave sums added in wave order
  if (wave == 0) {
    float s3 = 0.0f, s4 = 0.0f, s2 = 0.0f, s1 = 0.0f;
#pragma unroll
    for (int w = 0; w < kTWaves; ++w) {
      const float* q = BiasPart + w * kBiasPart;
      s3 += q[l];
      s4 += q[64 + l];
      s2 += q[128 + l];
      s1 += q[192 + l];
    }
    gp[kB3 + l] = s3;
    gp[kW4 + l] = s4;
    gp[kB2 + l] = s2;
    gp[kB1 + l] = s1;
    if (l == 0) {
      float s0 = 0.0f;
      for (int w = 0; w < kTWaves; ++w) s0 += BiasPart[w * kBiasPart + 256];
      gp[kB4] = s0;
    }
  }
  if (tid == 0) {
    float sum = 0.0f;
    for (int r = 0; r < kTRows; ++r) sum += RowLoss[r];
    loss_partial[blockIdx.x] = sum;
  }
}

// Partial gradients summed in two fixed-order levels: kRedGroups groups of consecutive
// partials, then the groups.
__global__ void k_grad_reduce_groups(const float* gp, uint32_t nb, float* tmp) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (uint32_t)kNParam) return;
  const uint32_t per = (nb + kRedGroups - 1) / kRedGroups;
  const uint32_t b0 = blockIdx.y * per, b1 = min(nb, b0 + per);
  float acc = 0.0f;
  for (uint32_t b = b0; b < b1; ++b) acc += gp[(uint64_t)b * kNParam + k];
  tmp[(uint64_t)blockIdx.y * kNParam + k] = acc;
}

__global__ void k_grad_reduce_final(const float* tmp, float* grad, const float* lp, uint32_t nb, float* loss_accum,
                                    uint32_t n_rows_total) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < (uint32_t)kNParam) {
    float acc = 0.0f;
    for (int g = 0; g < kRedGroups; ++g) acc += tmp[(uint64_t)g * kNParam + k];
    grad[k] = acc;
  }
  if (k == 0 && loss_accum) {
    float s = 0.0f;
    for (uint32_t b = 0; b < nb; ++b) s += lp[b];
    *loss_accum += s / (float)n_rows_total;
  }
}

// Adam (bias-corrected) on one parameter; returns the new weight.
__device__ __forceinline__ float adam_update(float w, float& m, float& v, float g, float c1, float c2, float lr) {
  const float mk = 0.9f * m + 0.1f * g;
  const float vk = 0.999f * v + 0.001f * g * g;
  m = mk;
  v = vk;
  return w - lr * (mk / c1) / (sqrtf(vk / c2) + 1e-8f);
}

__device__ __forceinline__ float ema_update(float infer, float w, float decay) {
  return decay > 0.0f ? fmaf(decay, infer - w, w) : w;
}

// One training step's tail in one launch: the block partials summed in block order, the loss,
// Adam on the master weights and the moving average of the inference weights.
// A block handles 64 parameters with 4 waves: wave s sums the partials b = s, s + 4, ...
// (consecutive lanes read consecutive parameters), the four sums are added in wave order.
constexpr int kTailParams = 64;
__global__ __launch_bounds__(256) void k_grad_adam_ema(const float* gp, uint32_t nb, float* grad, const float* lp,
                                                       float* loss_accum, uint32_t n_rows_total, float* w, float* m,
                                                       float* v, float c1, float c2, float lr, float* infer,
                                                       float decay) {
  __shared__ float part[4][kTailParams];
  const uint32_t j = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const uint32_t k = blockIdx.x * kTailParams + j;
  float g = 0.0f;
  if (k < (uint32_t)kNParam) {
#pragma unroll 8
    for (uint32_t b = sl; b < nb; b += 4) g += gp[(uint64_t)b * kNParam + k];
  }
  part[sl][j] = g;
  __syncthreads();
  if (sl == 0 && k < (uint32_t)kNParam) {
    g = ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j];
    grad[k] = g;
    const float wn = adam_update(w[k], m[k], v[k], g, c1, c2, lr);
    w[k] = wn;
    infer[k] = ema_update(infer[k], wn, decay);
  }
  if (blockIdx.x == 0 && threadIdx.x == 64 && loss_accum) {
    float s = 0.0f;
#pragma unroll 8
    for (uint32_t b = 0; b < nb; ++b) s += lp[b];
    *loss_accum += s / (float)n_rows_total;
  }
}

// Bias corrections of Adam step `step` (1-based), in double before rounding.
inline void adam_corrections(uint64_t step, float& c1, float& c2) {
  const double t = (double)step;
  c1 = (float)(1.0 - std::pow(0.9, t));
  c2 = (float)(1.0 - std::pow(0.999, t));
}

}  // namespace

void launch_grad_adam_ema(const float* grad_partial, uint32_t nblocks, float* grad, const float* loss_partial,
                          float* loss_accum, uint32_t n_rows_total, float* master, float* m, float* v, uint64_t step,
                          float lr, float* infer, float decay, hipStream_t s) {
  float c1, c2;
  adam_corrections(step, c1, c2);
  hipLaunchKernelGGL(k_grad_adam_ema, dim3((kNParam + kTailParams - 1) / kTailParams), dim3(256), 0, s, grad_partial,
                     nblocks, grad, loss_partial, loss_accum, n_rows_total, master, m, v, c1, c2, lr, infer, decay);
}

uint32_t mlp_grad_blocks(uint32_t n) { return (n + kTRows - 1) / kTRows; }
uint32_t mlp_grad_scratch_floats(uint32_t max_rows) {
  return (mlp_grad_blocks(max_rows) + kRedGroups) * (uint32_t)kNParam;
}

void launch_mlp_grad(const float* x, const float* target, const uint32_t* index, uint32_t n, const float* master,
                     int32_t loss_kind, float* grad_partial, float* loss_partial, uint32_t* nblocks_out,
                     hipStream_t s) {
  const uint32_t nb = mlp_grad_blocks(n);
  *nblocks_out = nb;
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute((const void*)k_mlp_grad_mfma, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(sizeof(float) * kLdsFloats));
    attr = true;
  }
  hipLaunchKernelGGL(k_mlp_grad_mfma, dim3(nb), dim3(kTThreads), sizeof(float) * kLdsFloats, s, x, target, index, n,
                     n, master, loss_kind, grad_partial, loss_partial);
}

void launch_grad_reduce(const float* grad_partial, uint32_t nblocks, float* grad, const float* loss_partial,
                        float* loss_accum, uint32_t n_rows_total, hipStream_t s) {
  float* tmp = const_cast<float*>(grad_partial) + (uint64_t)nblocks * kNParam;
  const uint32_t bx = (kNParam + 255) / 256;
  hipLaunchKernelGGL(k_grad_reduce_groups, dim3(bx, kRedGroups), dim3(256), 0, s, grad_partial, nblocks, tmp);
  hipLaunchKernelGGL(k_grad_reduce_final, dim3(bx), dim3(256), 0, s, tmp, grad, loss_partial, nblocks, loss_accum,
                     n_rows_total);
}

}  // namespace nrrs
