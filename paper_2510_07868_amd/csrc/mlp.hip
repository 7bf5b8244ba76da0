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
  a.q[i] = network_factor(lum(xyz(th)), y, g, q0);
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
// (gradient kernels: mlp_train.hip)
__global__ void k_record_targets(Records r, float* target, uint32_t n) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float lt = r.lum_t[k];
  target[k] = lt > 0.0f ? fmaxf(r.acc[k], 0.0f) / lt : 0.0f;
}

}  // namespace

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

void launch_quantize(const float* master, uint16_t* bf16, uint8_t* fp8, float* fp8_scale, hipStream_t s) {
  launch_pack_weights(master, bf16, fp8, fp8_scale, s);
}

void launch_record_targets(const Records& r, float* target, uint32_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_record_targets, dim3((n + 255) / 256), dim3(256), 0, s, r, target, n);
}

}  // namespace nrrs
