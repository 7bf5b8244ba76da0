// RRS network on gfx950: 20 -> 64 -> 64 -> 64 (ReLU) -> 1 with the modified softplus of
// the paper (Sec. 5, Eq. 22), inference inside the bounce loop (Mix-Depth gated, Sec. 4.3)
// and online training with the log-radiance loss, its backward pass and Adam.
//
// The factor a vertex receives from the network is the ADRRS ratio of the estimated
// reflected radiance to the pixel estimate (Sec. 2.2): q = lum(t) * y / (I_px + 0.01), with
// the previous mean image as I_px (Sec. 5 "Compromise").
#include <algorithm>

#include "features.hpp"
#include "launch.hpp"

namespace nrrs {

namespace {

constexpr int kNetThreads = 256;
constexpr int kGradRows = 64;      // rows per training block
constexpr int kGradThreads = 256;

__device__ __forceinline__ float softplus_mod(float z) { return z < 0.0f ? log1pf(expf(z)) : 0.5f * z + 0.69314718055994531f; }
__device__ __forceinline__ float softplus_mod_grad(float z) { return z < 0.0f ? 1.0f / (1.0f + expf(-z)) : 0.5f; }

// FP32 forward of one row with the weights in LDS; returns the pre-activation output z.
__device__ __forceinline__ float mlp_row_f32(const float* W, const float f[20]) {
  float h1[64];
#pragma unroll
  for (int o = 0; o < 64; ++o) {
    float acc = W[kB1 + o];
#pragma unroll
    for (int i = 0; i < 20; ++i) acc = fmaf(W[kW1 + 20 * o + i], f[i], acc);
    h1[o] = fmaxf(acc, 0.0f);
  }
  float h2[64];
#pragma unroll 4
  for (int o = 0; o < 64; ++o) {
    float acc = W[kB2 + o];
#pragma unroll
    for (int i = 0; i < 64; ++i) acc = fmaf(W[kW2 + 64 * o + i], h1[i], acc);
    h2[o] = fmaxf(acc, 0.0f);
  }
  float z = W[kB4];
#pragma unroll 4
  for (int o = 0; o < 64; ++o) {
    float acc = W[kB3 + o];
#pragma unroll
    for (int i = 0; i < 64; ++i) acc = fmaf(W[kW3 + 64 * o + i], h2[i], acc);
    z = fmaf(W[kW4 + o], fmaxf(acc, 0.0f), z);
  }
  return z;
}

__device__ __forceinline__ void load_weights(float* sw, const float* master) {
  for (int k = threadIdx.x; k < kNParam; k += blockDim.x) sw[k] = master[k];
  __syncthreads();
}

__global__ __launch_bounds__(kNetThreads) void k_rrsnet_f32(RenderArgs a, const float* master) {
  __shared__ float sw[kNParam];
  load_weights(sw, master);
  const uint32_t n = a.ctl[a.depth].n;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float q0 = a.q[i];
  if (!(q0 > 0.0f)) return;
  const float4 dr = a.qin.dir[i];
  const uint32_t pix = __float_as_uint(dr.w);
  const float g = a.guide[pix];
  if (!(g >= 0.0f)) return;  // no pixel history: keep the heuristic factor
  const float4 th = a.qin.thr[i], vp = a.vpos[i], vn = a.vnrm[i];
  const uint32_t mid = __float_as_uint(vn.w);
  const float4 m0 = a.sc.mat[2 * mid], m1 = a.sc.mat[2 * mid + 1];
  float f[20];
  vertex_features(a.sc, xyz(vp), xyz(vn), v3(-dr.x, -dr.y, -dr.z), xyz(th), m0, __float_as_uint(m1.w), a.depth,
                  a.max_depth, f);
  const float y = softplus_mod(mlp_row_f32(sw, f));
  const float q = lum(xyz(th)) * y / (g + 0.01f);
  if (isfinite(q) && q > 0.0f) a.q[i] = q;
}

__global__ __launch_bounds__(kNetThreads) void k_forward_rows_f32(const float* x, uint32_t n, const float* master,
                                                                float* y, float* z) {
  __shared__ float sw[kNParam];
  load_weights(sw, master);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float f[20];
#pragma unroll
  for (int k = 0; k < 20; ++k) f[k] = x[20ull * i + k];
  const float zz = mlp_row_f32(sw, f);
  y[i] = softplus_mod(zz);
  if (z) z[i] = zz;
}

// ------------------------------------------------------------------------ training
// One block: forward of kGradRows rows with activations kept in LDS, loss
// mean((ln(y+eps) - ln(L+eps))^2), backward through softplus and ReLU (ReLU'(0) = 0), and
// the block's partial weight gradients summed over its rows (fixed order, deterministic).
__global__ __launch_bounds__(kGradThreads) void k_mlp_grad(const float* x, const float* target,
                                                          const uint32_t* index, uint32_t n, uint32_t n_total,
                                                          const float* master, int32_t loss_kind,
                                                          float* grad_partial, float* loss_partial) {
  extern __shared__ float lds[];
  float* W = lds;                              // kNParam
  float* X = W + kNParam + 3;                  // [64][20]
  float* A1 = X + kGradRows * 20;              // pre-activations [64 rows][64]
  float* A2 = A1 + kGradRows * 64;
  float* A3 = A2 + kGradRows * 64;
  float* D1 = A3 + kGradRows * 64;             // deltas
  float* D2 = D1 + kGradRows * 64;
  float* D3 = D2 + kGradRows * 64;
  float* DZ = D3 + kGradRows * 64;             // [64]
  float* LS = DZ + kGradRows;                  // [64] per-row loss
  const int tid = threadIdx.x;
  const uint32_t row0 = blockIdx.x * kGradRows;
  const uint32_t rows = min((uint32_t)kGradRows, n - row0);
  for (int k = tid; k < kNParam; k += kGradThreads) W[k] = master[k];
  for (int k = tid; k < kGradRows * 20; k += kGradThreads) {
    const uint32_t r = k / 20;
    float v = 0.0f;
    if (r < rows) {
      const uint32_t src = index ? index[row0 + r] : row0 + r;
      v = x[20ull * src + (k % 20)];
    }
    X[k] = v;
  }
  __syncthreads();
  // layer 1..3 pre-activations: thread handles (row, 16 outputs)
  for (int layer = 0; layer < 3; ++layer) {
    float* dst = layer == 0 ? A1 : (layer == 1 ? A2 : A3);
    const float* src = layer == 0 ? X : (layer == 1 ? A1 : A2);
    const int kin = layer == 0 ? 20 : 64;
    const float* Wl = W + (layer == 0 ? kW1 : (layer == 1 ? kW2 : kW3));
    const float* bl = W + (layer == 0 ? kB1 : (layer == 1 ? kB2 : kB3));
    for (int e = tid; e < kGradRows * 64; e += kGradThreads) {
      const int r = e / 64, o = e % 64;
      float acc = bl[o];
      for (int i = 0; i < kin; ++i) {
        float h = src[r * kin + i];
        if (layer > 0) h = fmaxf(h, 0.0f);
        acc = fmaf(Wl[o * kin + i], h, acc);
      }
      dst[e] = acc;
    }
    __syncthreads();
  }
  if (tid < kGradRows) {
    const int r = tid;
    float dz = 0.0f, ls = 0.0f;
    if ((uint32_t)r < rows) {
      float z = W[kB4];
      for (int i = 0; i < 64; ++i) z = fmaf(W[kW4 + i], fmaxf(A3[r * 64 + i], 0.0f), z);
      const float y = softplus_mod(z);
      const uint32_t src = index ? index[row0 + r] : row0 + r;
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
    DZ[r] = dz;
    LS[r] = ls;
  }
  __syncthreads();
  for (int e = tid; e < kGradRows * 64; e += kGradThreads) {
    const int r = e / 64, i = e % 64;
    D3[e] = A3[e] > 0.0f ? DZ[r] * W[kW4 + i] : 0.0f;
  }
  __syncthreads();
  for (int e = tid; e < kGradRows * 64; e += kGradThreads) {
    const int r = e / 64, i = e % 64;
    float acc = 0.0f;
    for (int o = 0; o < 64; ++o) acc = fmaf(W[kW3 + 64 * o + i], D3[r * 64 + o], acc);
    D2[e] = A2[e] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  for (int e = tid; e < kGradRows * 64; e += kGradThreads) {
    const int r = e / 64, i = e % 64;
    float acc = 0.0f;
    for (int o = 0; o < 64; ++o) acc = fmaf(W[kW2 + 64 * o + i], D2[r * 64 + o], acc);
    D1[e] = A1[e] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  float* gp = grad_partial + (uint64_t)blockIdx.x * kNParam;
  for (int k = tid; k < kNParam; k += kGradThreads) {
    float acc = 0.0f;
    if (k < kB1) {  // W1[o][i]
      const int o = k / 20, i = k % 20;
      for (int r = 0; r < kGradRows; ++r) acc = fmaf(D1[r * 64 + o], X[r * 20 + i], acc);
    } else if (k < kW2) {
      const int o = k - kB1;
      for (int r = 0; r < kGradRows; ++r) acc += D1[r * 64 + o];
    } else if (k < kB2) {
      const int o = (k - kW2) / 64, i = (k - kW2) % 64;
      for (int r = 0; r < kGradRows; ++r) acc = fmaf(D2[r * 64 + o], fmaxf(A1[r * 64 + i], 0.0f), acc);
    } else if (k < kW3) {
      const int o = k - kB2;
      for (int r = 0; r < kGradRows; ++r) acc += D2[r * 64 + o];
    } else if (k < kB3) {
      const int o = (k - kW3) / 64, i = (k - kW3) % 64;
      for (int r = 0; r < kGradRows; ++r) acc = fmaf(D3[r * 64 + o], fmaxf(A2[r * 64 + i], 0.0f), acc);
    } else if (k < kW4) {
      const int o = k - kB3;
      for (int r = 0; r < kGradRows; ++r) acc += D3[r * 64 + o];
    } else if (k < kB4) {
      const int i = k - kW4;
      for (int r = 0; r < kGradRows; ++r) acc = fmaf(DZ[r], fmaxf(A3[r * 64 + i], 0.0f), acc);
    } else {
      for (int r = 0; r < kGradRows; ++r) acc += DZ[r];
    }
    gp[k] = acc;
  }
  if (tid == 0) {
    float s = 0.0f;
    for (int r = 0; r < kGradRows; ++r) s += LS[r];
    loss_partial[blockIdx.x] = s;
  }
}

__global__ void k_grad_reduce(const float* gp, uint32_t nb, float* grad, const float* lp, float* loss_accum,
                              uint32_t n_rows_total) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < (uint32_t)kNParam) {
    float acc = 0.0f;
    for (uint32_t b = 0; b < nb; ++b) acc += gp[(uint64_t)b * kNParam + k];
    grad[k] = acc;
  }
  if (k == 0 && loss_accum) {
    float s = 0.0f;
    for (uint32_t b = 0; b < nb; ++b) s += lp[b];
    *loss_accum += s / (float)n_rows_total;
  }
}

__global__ void k_adam(float* w, float* m, float* v, const float* g, uint64_t step, float lr) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (uint32_t)kNParam) return;
  const double t = (double)step;
  const float c1 = (float)(1.0 - pow(0.9, t));
  const float c2 = (float)(1.0 - pow(0.999, t));
  const float gk = g[k];
  const float mk = 0.9f * m[k] + 0.1f * gk;
  const float vk = 0.999f * v[k] + 0.001f * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + 1e-8f);
}

__global__ void k_ema(float* infer, const float* master, float decay) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < (uint32_t)kNParam) infer[k] = decay > 0.0f ? fmaf(decay, infer[k] - master[k], master[k]) : master[k];
}

__global__ void k_record_targets(Records r, float* target, uint32_t n) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float lt = r.lum_t[k];
  target[k] = lt > 0.0f ? fmaxf(r.acc[k], 0.0f) / lt : 0.0f;
}

}  // namespace

uint32_t mlp_grad_blocks(uint32_t n) { return (n + kGradRows - 1) / kGradRows; }

static size_t grad_lds_bytes() {
  return sizeof(float) * (kNParam + 3 + kGradRows * 20 + 6 * kGradRows * 64 + 2 * kGradRows);
}

void launch_rrsnet(const RenderArgs& a, const NetArgs& n, hipStream_t s) {
  if (n.precision != 0) {
    launch_rrsnet_mfma(a, n, s);
    return;
  }
  const uint32_t blocks = (a.cap + kNetThreads - 1) / kNetThreads;
  hipLaunchKernelGGL(k_rrsnet_f32, dim3(blocks), dim3(kNetThreads), 0, s, a, n.master);
}

void launch_mlp_forward_rows(const float* x, uint32_t n, const NetArgs& net, float* y, float* z, hipStream_t s) {
  if (!n) return;
  if (net.precision != 0) {
    launch_rows_mfma(x, n, net, y, z, s);
    return;
  }
  hipLaunchKernelGGL(k_forward_rows_f32, dim3((n + kNetThreads - 1) / kNetThreads), dim3(kNetThreads), 0, s, x, n,
                     net.master, y, z);
}

void launch_mlp_grad(const float* x, const float* target, const uint32_t* index, uint32_t n, const float* master,
                     int32_t loss_kind, float* grad_partial, float* loss_partial, uint32_t* nblocks_out,
                     hipStream_t s) {
  const uint32_t nb = mlp_grad_blocks(n);
  *nblocks_out = nb;
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute((const void*)k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize, (int)grad_lds_bytes());
    attr = true;
  }
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(kGradThreads), grad_lds_bytes(), s, x, target, index, n, n, master,
                     loss_kind, grad_partial, loss_partial);
}

void launch_grad_reduce(const float* grad_partial, uint32_t nblocks, float* grad, const float* loss_partial,
                        float* loss_accum, uint32_t n_rows_total, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_reduce, dim3((kNParam + 255) / 256), dim3(256), 0, s, grad_partial, nblocks, grad,
                     loss_partial, loss_accum, n_rows_total);
}

void launch_adam(float* master, float* m, float* v, const float* grad, uint64_t step, float lr, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((kNParam + 255) / 256), dim3(256), 0, s, master, m, v, grad, step, lr);
}

void launch_ema(float* infer, const float* master, float decay, hipStream_t s) {
  hipLaunchKernelGGL(k_ema, dim3((kNParam + 255) / 256), dim3(256), 0, s, infer, master, decay);
}

void launch_quantize(const float* master, uint16_t* bf16, uint8_t* fp8, float* fp8_scale, hipStream_t s) {
  launch_pack_weights(master, bf16, fp8, fp8_scale, s);
}

void launch_record_targets(const Records& r, float* target, uint32_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_record_targets, dim3((n + 255) / 256), dim3(256), 0, s, r, target, n);
}

}  // namespace nrrs
