// NRRS proper on gfx950 (Sec. 4.2, Sec. 5).  StatNet predicts the luminance mean m and
// variance v of the radiance reflected at a vertex from a multiresolution hash grid of its
// position and one-blob encodings of its outgoing direction and roughness; RRSNet (NRRS
// variant) maps Box-Cox(m), Box-Cox(v + m^2), Box-Cox(throughput), Box-Cox(pixel value) and the
// remapped roughness to the RRS factor through the modified softplus (Eq. 22).  Both networks
// are in -> 32 -> 32 -> 32 -> out with leaky ReLU (Sec. 5 "Network Architecture").
//
// Training (one Adam step per frame over all its records, the paper's batch of 2^19):
// StatNet by the relative L2 of Eq. (15); RRSNet first toward the output 1, then by the
// pixel-variance loss of Eq. (16), whose gradient reaches each sample's factor through the
// one-sample transfer of Eqs. (17)-(18), shared by the pixel's samples, plus the bound loss of
// Eq. (21).  The per-pixel error uses the temporal mix of Eq. (23) and a box filter.
//
// Layout: inference evaluates 64 vertices per wave, each lane encoding its own vertex, with the
// networks' layers on the FP32 matrix cores; training runs one thread per record with the
// weights in LDS (read by all lanes at once); the hash grid lives in HBM ([level][2^log2T][2]
// floats, gathered per corner).  Weight gradients are
// reduced per block through LDS tiles of the per-record activations and deltas in a fixed
// order, then over blocks in block order; hash-grid gradients are added atomically.
#include <algorithm>
#include <cmath>

#include "features.hpp"
#include "launch.hpp"

namespace nrrs {

namespace {

constexpr int kT = 256;       // threads per block
constexpr int kPad = 33;      // LDS row stride (floats) of the per-record tiles
constexpr float kLeak = 0.01f;

__device__ __forceinline__ float leaky(float x) { return x > 0.0f ? x : kLeak * x; }
// derivative of the leaky ReLU from its output (same sign as its input)
__device__ __forceinline__ float dleaky(float h) { return h > 0.0f ? 1.0f : kLeak; }
__device__ __forceinline__ float softplus_mod(float z) { return z < 0.0f ? log1pf(expf(z)) : 0.5f * z + 0.69314718055994531f; }
__device__ __forceinline__ float softplus_mod_grad(float z) { return z < 0.0f ? 1.0f / (1.0f + expf(-z)) : 0.5f; }
__device__ __forceinline__ float box_cox(float x) { return 2.0f * (sqrtf(fmaxf(x, 0.0f)) - 1.0f); }

// Parameter offsets of an in -> 32 -> 32 -> 32 -> out network.
template <int IN, int OUT>
struct L32 {
  static constexpr int W1 = 0, B1 = 32 * IN, W2 = B1 + 32, B2 = W2 + 1024, W3 = B2 + 32, B3 = W3 + 1024,
                       W4 = B3 + 32, B4 = W4 + 32 * OUT, N = B4 + OUT;
};
static_assert(L32<kStatIn, kStatOut>::N == (int)kStatParams, "StatNet layout");
static_assert(L32<kRrsIn, 1>::N == (int)kRrsParams, "RRSNet layout");

// y = leaky(W x + b) for one 32-wide hidden layer (W row-major [32][K], in LDS).
template <int K>
__device__ __forceinline__ void hidden(const float* __restrict__ W, const float* __restrict__ b, const float (&x)[K],
                                       float (&y)[32]) {
#pragma unroll
  for (int o = 0; o < 32; ++o) {
    float acc = b[o];
#pragma unroll
    for (int i = 0; i < K; ++i) acc = fmaf(W[o * K + i], x[i], acc);
    y[o] = leaky(acc);
  }
}

// Forward through the three hidden layers and the linear output; keeps the activations.
template <int IN, int OUT>
__device__ __forceinline__ void mlp32(const float* P, const float (&x)[IN], float (&h1)[32], float (&h2)[32],
                                      float (&h3)[32], float (&y)[OUT]) {
  using Lo = L32<IN, OUT>;
  // the empty asm statements keep each layer's weight reads from LDS within the layer: hoisted
  // ahead, thousands of them would each hold a register
  hidden<IN>(P + Lo::W1, P + Lo::B1, x, h1);
  asm volatile("" ::: "memory");
  hidden<32>(P + Lo::W2, P + Lo::B2, h1, h2);
  asm volatile("" ::: "memory");
  hidden<32>(P + Lo::W3, P + Lo::B3, h2, h3);
  asm volatile("" ::: "memory");
#pragma unroll
  for (int k = 0; k < OUT; ++k) {
    float acc = P[Lo::B4 + k];
#pragma unroll
    for (int i = 0; i < 32; ++i) acc = fmaf(P[Lo::W4 + 32 * k + i], h3[i], acc);
    y[k] = acc;
  }
}

// ------------------------------------------------------------------ matrix-core inference
// A wave evaluates 64 vertices, one per lane, as two tiles of 32 on the FP32 matrix cores
// (v_mfma_f32_32x32x2_f32): M = the 32 units of a layer, N = a tile's 32 vertices, K = the
// layer's inputs two at a time.  Lane l computes the inputs of vertex l (tile l / 32, column
// l % 32) and, as an MFMA operand, serves column c = l % 32 of both tiles in lane half h = l / 32:
// A[m = c][k = h] (weights) and B[k = h][n = c] (inputs).  Register v of an accumulator holds
// unit 8 (v / 4) + 4 h + v % 4 of column c, so a layer's leaky-ReLU outputs are the next layer's
// B operands unchanged when that layer's weights are taken in the same unit order.  The first
// layer's inputs of a tile's column come from the two lanes of that column: one exchange across
// the lane halves per input pair.  The weights sit in LDS in operand order (each lane reads its
// own contiguous run).  FP32 products and FP32 accumulation, as the vector path; only the order
// of the additions differs.
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int acc_unit(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// LDS image of an in -> 32 -> 32 -> 32 -> out network in operand order (floats):
//   W1 [h][c][S]: W1[c][2s + h] (0 past the inputs), S = ceil(in / 2) input pairs
//   W2, W3 [h][c][16]: W[c][acc_unit(s, h)];  B1, B2, B3 [h][16]: b[acc_unit(v, h)]
//   W4 [o][h][16]: W4[o][acc_unit(v, h)];  B4 [o]
template <int IN, int OUT>
struct Img {
  static constexpr int S = (IN + 1) / 2;
  static constexpr int W1 = 0, W2 = W1 + 64 * S, W3 = W2 + 1024, B1 = W3 + 1024, B2 = B1 + 32, B3 = B2 + 32,
                       W4 = B3 + 32, B4 = W4 + 32 * OUT, N = B4 + OUT;
};

template <int IN, int OUT>
__device__ __forceinline__ void load_img(float* dst, const float* P) {
  using Lo = L32<IN, OUT>;
  using Im = Img<IN, OUT>;
  for (int d = threadIdx.x; d < Im::N; d += blockDim.x) {
    float v = 0.0f;
    if (d < Im::W2) {
      const int s = d % Im::S, c = (d / Im::S) % 32, h = d / (Im::S * 32), k = 2 * s + h;
      if (k < IN) v = P[Lo::W1 + c * IN + k];
    } else if (d < Im::B1) {
      const bool second = d < Im::W3;
      const int j = d - (second ? Im::W2 : Im::W3);
      const int s = j % 16, c = (j / 16) % 32, h = j / 512;
      v = P[(second ? Lo::W2 : Lo::W3) + c * 32 + acc_unit(s, h)];
    } else if (d < Im::W4) {
      const int L = (d - Im::B1) / 32, j = (d - Im::B1) % 32;
      v = P[(L == 0 ? Lo::B1 : L == 1 ? Lo::B2 : Lo::B3) + acc_unit(j % 16, j / 16)];
    } else if (d < Im::B4) {
      const int j = d - Im::W4, o = j / 32, h = (j / 16) % 2;
      v = P[Lo::W4 + o * 32 + acc_unit(j % 16, h)];
    } else {
      v = P[Lo::B4 + (d - Im::B4)];
    }
    dst[d] = v;
  }
}

__device__ __forceinline__ f32x16 mfma_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// The network on the wave's 64 vertices: x = this lane's vertex's inputs; returns the outputs
// of this lane's vertex.  All 64 lanes must call it together (inactive lanes with finite
// inputs, e.g. zeros).
template <int IN, int OUT>
__device__ __forceinline__ void mlp_mfma(const float* I, const float (&x)[IN], float (&y)[OUT]) {
  using Im = Img<IN, OUT>;
  const int l = (int)__lane_id(), h = l >> 5, c = l & 31;
  f32x16 a0, a1;
  // layer 1: the pair (2s, 2s + 1) of tile 0 is (own, partner's) in half 0 and (partner's, own)
  // in half 1; the lane sends the value its partner lacks
  {
    const float* w = I + Im::W1 + (h * 32 + c) * Im::S;
#pragma unroll
    for (int v = 0; v < 16; ++v) a0[v] = a1[v] = I[Im::B1 + h * 16 + v];
#pragma unroll
    for (int s = 0; s < Im::S; ++s) {
      const float lo = x[2 * s], hi = 2 * s + 1 < IN ? x[2 * s + 1] : 0.0f;
      const float recv = __shfl_xor(h ? lo : hi, 32);
      const float wk = w[s];
      a0 = mfma_f32(wk, h ? recv : lo, a0);  // tile 0: vertex c's input 2s + h
      a1 = mfma_f32(wk, h ? hi : recv, a1);  // tile 1: vertex 32 + c's input 2s + h
    }
  }
  float h0[16], h1[16];
#pragma unroll
  for (int L = 0; L < 2; ++L) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      h0[v] = leaky(a0[v]);
      h1[v] = leaky(a1[v]);
    }
    asm volatile("" ::: "memory");
    const float* w = I + (L == 0 ? Im::W2 : Im::W3) + (h * 32 + c) * 16;
    const float* b = I + (L == 0 ? Im::B2 : Im::B3) + h * 16;
#pragma unroll
    for (int v = 0; v < 16; ++v) a0[v] = a1[v] = b[v];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const float wk = w[s];
      a0 = mfma_f32(wk, h0[s], a0);
      a1 = mfma_f32(wk, h1[s], a1);
    }
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    h0[v] = leaky(a0[v]);
    h1[v] = leaky(a1[v]);
  }
#pragma unroll
  for (int o = 0; o < OUT; ++o) {
    const float* w = I + Im::W4 + (o * 2 + h) * 16;
    float p0 = 0.0f, p1 = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      p0 = fmaf(w[v], h0[v], p0);
      p1 = fmaf(w[v], h1[v], p1);
    }
    p0 += __shfl_xor(p0, 32);
    p1 += __shfl_xor(p1, 32);
    y[o] = (h ? p1 : p0) + I[Im::B4 + o];
  }
}

// ------------------------------------------------------------------ encodings
// Hash grid (Sec. 5 "Input Encoding"): level l has resolution R = 16 * 2^l; p lies in cell
// c = min(floor(p R), R - 1) per axis and reads the trilinear interpolation of its 8 corners.
// A corner is stored densely when the level's (R + 1)^3 corners fit the table, else at the
// spatial hash (x ^ y * 2654435761 ^ z * 805459861) mod 2^log2T.
struct Corner8 {
  uint32_t idx[8];
  float w[8];
};

__device__ __forceinline__ void hg_corners(float px, float py, float pz, int l, uint32_t log2T, Corner8& c) {
  const uint32_t R = (uint32_t)kHgBase << l;
  const float Rf = (float)R;
  float f[3];
  uint32_t ci[3];
  const float p[3] = {px, py, pz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float u = fminf(fmaxf(p[a], 0.0f), 1.0f) * Rf;  // exact: R is a power of two
    const float fl = fminf(floorf(u), Rf - 1.0f);
    ci[a] = (uint32_t)fl;
    f[a] = u - fl;
  }
  const uint64_t side = (uint64_t)R + 1;
  const bool dense = side * side * side <= (1ull << log2T);
  const uint32_t mask = (1u << log2T) - 1u;
  const uint32_t side32 = R + 1u;  // a dense level's corner index fits 32 bits (below 2^log2T)
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    const uint32_t x = ci[0] + dx, y = ci[1] + dy, z = ci[2] + dz;
    c.idx[k] = dense ? x + side32 * (y + side32 * z) : ((x * 1u) ^ (y * 2654435761u) ^ (z * 805459861u)) & mask;
    c.w[k] = (dx ? f[0] : 1.0f - f[0]) * (dy ? f[1] : 1.0f - f[1]) * (dz ? f[2] : 1.0f - f[2]);
  }
}

__device__ __forceinline__ void oneblob(float s, int bins, float* out) {
  s = fminf(fmaxf(s, 0.0f), 1.0f);
  for (int i = 0; i < bins; ++i) {
    const float d = (s - ((float)i + 0.5f) / (float)bins) * (float)bins;  // distance in bin widths (sigma)
    out[i] = expf(-0.5f * d * d);
  }
}

// The 32 StatNet inputs from raw = (p in [0,1]^3, w_o, remapped roughness).
__device__ __forceinline__ void statnet_encode(const float* __restrict__ table, uint32_t log2T, const float (&raw)[7],
                                               float (&enc)[32]) {
  const uint64_t T = 1ull << log2T;
#pragma unroll
  for (int l = 0; l < kHgLevels; ++l) {
    Corner8 c;
    hg_corners(raw[0], raw[1], raw[2], l, log2T, c);
    const float2* tl = reinterpret_cast<const float2*>(table + (uint64_t)l * T * kHgFeat);
    float e0 = 0.0f, e1 = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float2 v = tl[c.idx[k]];
      e0 = fmaf(c.w[k], v.x, e0);
      e1 = fmaf(c.w[k], v.y, e1);
    }
    enc[2 * l] = e0;
    enc[2 * l + 1] = e1;
    // at most two levels' 16 corner loads in flight: all 64 at once held 128 registers
    if (l & 1) asm volatile("" ::: "memory");
  }
  const float theta = acosf(fminf(fmaxf(raw[5], -1.0f), 1.0f));
  const float phi = atan2f(raw[4], raw[3]);
  float ob[16];
  oneblob(theta * 0.31830988618379067f, 4, ob);
  oneblob(phi * 0.15915494309189535f + 0.5f, 4, ob + 4);
  oneblob(raw[6], 8, ob + 8);
#pragma unroll
  for (int k = 0; k < 16; ++k) enc[16 + k] = ob[k];
}

// The 32 AID-NRRS RRSNet inputs: its own hash grid of p (16), one-blob w_o (8), Box-Cox of the
// throughput (3) and of the pixel value (1), one-blob of the remapped roughness with 4 bins (4).
__device__ __forceinline__ void aid_encode(const float* __restrict__ table, uint32_t log2T, const float (&raw)[7],
                                           float tx, float ty, float tz, float I, float (&enc)[32]) {
  const uint64_t T = 1ull << log2T;
#pragma unroll
  for (int l = 0; l < kHgLevels; ++l) {
    Corner8 c;
    hg_corners(raw[0], raw[1], raw[2], l, log2T, c);
    const float2* tl = reinterpret_cast<const float2*>(table + (uint64_t)l * T * kHgFeat);
    float e0 = 0.0f, e1 = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float2 v = tl[c.idx[k]];
      e0 = fmaf(c.w[k], v.x, e0);
      e1 = fmaf(c.w[k], v.y, e1);
    }
    enc[2 * l] = e0;
    enc[2 * l + 1] = e1;
    if (l & 1) asm volatile("" ::: "memory");  // as in statnet_encode
  }
  const float theta = acosf(fminf(fmaxf(raw[5], -1.0f), 1.0f));
  const float phi = atan2f(raw[4], raw[3]);
  float ob[12];
  oneblob(theta * 0.31830988618379067f, 4, ob);
  oneblob(phi * 0.15915494309189535f + 0.5f, 4, ob + 4);
  oneblob(raw[6], 4, ob + 8);
#pragma unroll
  for (int k = 0; k < 8; ++k) enc[16 + k] = ob[k];
  enc[24] = box_cox(tx);
  enc[25] = box_cox(ty);
  enc[26] = box_cox(tz);
  enc[27] = box_cox(I);
#pragma unroll
  for (int k = 0; k < 4; ++k) enc[28 + k] = ob[8 + k];
}

__device__ __forceinline__ void rrs_inputs(float m, float v, float tx, float ty, float tz, float I, float rho,
                                           float (&x)[7]) {
  const float mp = fmaxf(m, 0.0f), vp = fmaxf(v, 0.0f);
  x[0] = box_cox(mp);
  x[1] = box_cox(vp + mp * mp);
  x[2] = box_cox(tx);
  x[3] = box_cox(ty);
  x[4] = box_cox(tz);
  x[5] = box_cox(I);
  x[6] = rho;
}

// Raw StatNet inputs of a queue vertex: position scaled to the scene box, w_o, remapped
// roughness (1 - e^-alpha; alpha = 1 for Lambertian surfaces, as in the vertex features).
__device__ __forceinline__ void vertex_raw(const DevScene& sc, float4 vp, float4 dr, float4 m0, uint32_t type,
                                           float (&raw)[7]) {
  const float inv = 1.0f / sc.extent;
  raw[0] = (vp.x - sc.amin_x) * inv;
  raw[1] = (vp.y - sc.amin_y) * inv;
  raw[2] = (vp.z - sc.amin_z) * inv;
  raw[3] = -dr.x;
  raw[4] = -dr.y;
  raw[5] = -dr.z;
  raw[6] = 1.0f - expf(-(type == 1u ? m0.w : 1.0f));
}

__device__ __forceinline__ void load_lds(float* dst, const float* src, uint32_t n) {
  for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
}

// ------------------------------------------------------------------ inference
// The NRRS factor of every vertex of the depth that has a raw factor and a pixel history; a
// non-finite (or underflowed) factor keeps the heuristic one.  Persistent waves over groups of
// 64 vertices: each lane encodes its vertex (hash-grid gathers, one-blob, Box-Cox), then the
// wave runs the networks on the matrix cores (mlp_mfma), weights in LDS in operand order.  At
// most 96 VGPRs (5 waves per SIMD) to hide the gathers; a build per table size keeps the
// encodings' level layout constant, which that budget needs.
template <bool kAid, uint32_t kLog2T>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_nrrs_factor(RenderArgs a,
                                                                                                NrrsNet net) {
  constexpr uint32_t log2T = kLog2T;  // equal to net.log2T (the launch picks the build)
  using IS = Img<kAid ? kAidIn : kStatIn, kAid ? 1 : kStatOut>;
  using IR = Img<kRrsIn, 1>;
  __shared__ float ps[IS::N];
  __shared__ float pr[kAid ? 1 : IR::N];
  if constexpr (kAid) {
    load_img<kAidIn, 1>(ps, net.aid);
  } else {
    load_img<kStatIn, kStatOut>(ps, net.stat);
    load_img<kRrsIn, 1>(pr, net.rrs);
  }
  __syncthreads();
  const uint32_t n = a.ctl[a.depth].n;
  const uint32_t groups = (n + 63) / 64;
  const uint32_t waves = gridDim.x * (kT / 64);
  const uint32_t lane = __lane_id();
  // Entries that take the learned factor (q > 0 and a pixel with history) are gathered per wave
  // into full groups of 64 before the encodings and the matrix-core layers: a third to a half of
  // a bounce's queue is paths that just ended, and a group computes all 64 columns either way.
  // A column's result does not depend on the other columns of its tile.
  __shared__ uint32_t pick[kT / 64][128];
  uint32_t* const buf = pick[threadIdx.x / 64];
  uint32_t gi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kT / 64) + threadIdx.x / 64));
  uint32_t cnt = 0;  // gathered entries not yet computed (wave-uniform, below 128)
  for (;;) {
    while (cnt < 64 && gi < groups) {
      const uint32_t j = gi * 64 + lane;
      bool take = false;
      if (j < n && a.q[j] > 0.0f) take = a.guide[__float_as_uint(a.qin.dir[j].w)] >= 0.0f;
      const uint64_t m = __ballot(take);
      if (take) buf[cnt + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = j;
      cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)(cnt + (uint32_t)__popcll(m)));
      gi += waves;
    }
    if (cnt == 0) break;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const bool active = lane < cnt;
    const uint32_t i = active ? buf[lane] : 0u;
    const bool moves = lane + 64 < cnt;
    const uint32_t rest = moves ? buf[lane + 64] : 0u;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (moves) buf[lane] = rest;  // the entries past the first 64 move to the front
    cnt = cnt > 64 ? cnt - 64 : 0;
    asm volatile("" ::: "memory");  // weights re-read from LDS each group, not held in registers
    float g = 0.0f, rho = 0.0f;
    float4 th = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float enc[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) enc[k] = 0.0f;
    if (active) {
      const float4 dr = a.qin.dir[i];
      g = a.guide[__float_as_uint(dr.w)];
      if constexpr (kAid) th = a.qin.thr[i];
      const float4 vp = a.vpos[i], vn = a.vnrm[i];
      const uint32_t mid = __float_as_uint(vn.w);
      const float4 m0 = a.sc.mat[2 * mid], m1 = a.sc.mat[2 * mid + 1];
      float raw[7];
      vertex_raw(a.sc, vp, dr, m0, __float_as_uint(m1.w), raw);
      rho = raw[6];
      if constexpr (kAid) aid_encode(net.table_r, log2T, raw, th.x, th.y, th.z, g, enc);
      else statnet_encode(net.table, log2T, raw, enc);
    }
    float z[1];
    if constexpr (kAid) {
      mlp_mfma<kAidIn, 1>(ps, enc, z);
    } else {
      float mv[2], x[7];
      mlp_mfma<kStatIn, kStatOut>(ps, enc, mv);
      if (active) th = a.qin.thr[i];  // read after StatNet: not held through its layers
      rrs_inputs(mv[0], mv[1], th.x, th.y, th.z, g, rho, x);
      mlp_mfma<kRrsIn, 1>(pr, x, z);
    }
    const float q = softplus_mod(z[0]);
    if (active && q >= 1e-20f && q < 3.0e38f) a.q[i] = q;  // else the heuristic factor stays
  }
}

// Test entry points: the same networks on given rows, 64 rows per wave (the grid covers whole
// waves; rows past n compute on zeros and write nothing).
__global__ __launch_bounds__(kT) void k_nrrs_rows(const float* raw_in, const float* t, const float* I, uint32_t n,
                                                  NrrsNet net, float* mv_out, float* q_out, float* enc_out) {
  using IS = Img<kStatIn, kStatOut>;
  using IR = Img<kRrsIn, 1>;
  __shared__ float ps[IS::N];
  __shared__ float pr[IR::N];
  load_img<kStatIn, kStatOut>(ps, net.stat);
  load_img<kRrsIn, 1>(pr, net.rrs);
  __syncthreads();
  const uint32_t i = blockIdx.x * kT + threadIdx.x;
  const bool active = i < n;
  float raw[7], enc[32], tx = 0.0f, ty = 0.0f, tz = 0.0f, Iv = 0.0f;
#pragma unroll
  for (int k = 0; k < 7; ++k) raw[k] = active ? raw_in[7ull * i + k] : 0.0f;
#pragma unroll
  for (int k = 0; k < 32; ++k) enc[k] = 0.0f;
  if (active) {
    tx = t[3ull * i];
    ty = t[3ull * i + 1];
    tz = t[3ull * i + 2];
    Iv = I[i];
    statnet_encode(net.table, net.log2T, raw, enc);
  }
  float mv[2], x[7], z[1];
  mlp_mfma<kStatIn, kStatOut>(ps, enc, mv);
  rrs_inputs(mv[0], mv[1], tx, ty, tz, Iv, raw[6], x);
  mlp_mfma<kRrsIn, 1>(pr, x, z);
  if (!active) return;
  mv_out[2ull * i] = mv[0];
  mv_out[2ull * i + 1] = mv[1];
  q_out[i] = softplus_mod(z[0]);
  if (enc_out) {
#pragma unroll
    for (int k = 0; k < 32; ++k) enc_out[32ull * i + k] = enc[k];
  }
}

__global__ __launch_bounds__(kT) void k_aid_rows(const float* raw_in, const float* t, const float* I, uint32_t n,
                                                 NrrsNet net, float* q_out, float* enc_out) {
  using IA = Img<kAidIn, 1>;
  __shared__ float pa[IA::N];
  load_img<kAidIn, 1>(pa, net.aid);
  __syncthreads();
  const uint32_t i = blockIdx.x * kT + threadIdx.x;
  const bool active = i < n;
  float raw[7], enc[32];
#pragma unroll
  for (int k = 0; k < 7; ++k) raw[k] = active ? raw_in[7ull * i + k] : 0.0f;
#pragma unroll
  for (int k = 0; k < 32; ++k) enc[k] = 0.0f;
  if (active) aid_encode(net.table_r, net.log2T, raw, t[3ull * i], t[3ull * i + 1], t[3ull * i + 2], I[i], enc);
  float z[1];
  mlp_mfma<kAidIn, 1>(pa, enc, z);
  if (!active) return;
  q_out[i] = softplus_mod(z[0]);
  if (enc_out) {
#pragma unroll
    for (int k = 0; k < 32; ++k) enc_out[32ull * i + k] = enc[k];
  }
}

// Normalized factor and F of the records captured at this depth (after its roulette).
__global__ void k_record_qnorm(RenderArgs a) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t cnt = min(*a.rec.count, a.rec.cap);
  if (s >= cnt || a.rec.depth[s] != a.depth) return;
  const double F = a.ctl[a.depth].F;
  a.rec.nqf[s] = make_float2((float)(F * (double)a.q[a.rec.qidx[s]]), (float)F);
}

// ------------------------------------------------------------------ training
constexpr int kTG = 128;  // records per block of the gradient kernels

// dW[o][i] = sum over the block's rows of D[row][o] A[row][i] (o < NO, i < NI) and
// db[o] = sum of D[row][o], in row order, from the LDS tiles; written to the block's partial.
template <int NO, int NI>
__device__ __forceinline__ void tile_outer(const float* A, const float* D, float* outW, float* outB) {
  constexpr int NG = (NI + 3) / 4;
  for (int item = threadIdx.x; item < NO * NG; item += kTG) {
    const int o = item / NG, i0 = 4 * (item % NG);
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll 4
    for (int r = 0; r < kTG; ++r) {
      const float d = D[r * kPad + o];
      const float* ar = A + r * kPad + i0;
      s0 = fmaf(d, ar[0], s0);
      if (i0 + 1 < NI) s1 = fmaf(d, ar[1], s1);
      if (i0 + 2 < NI) s2 = fmaf(d, ar[2], s2);
      if (i0 + 3 < NI) s3 = fmaf(d, ar[3], s3);
    }
    outW[o * NI + i0] = s0;
    if (i0 + 1 < NI) outW[o * NI + i0 + 1] = s1;
    if (i0 + 2 < NI) outW[o * NI + i0 + 2] = s2;
    if (i0 + 3 < NI) outW[o * NI + i0 + 3] = s3;
  }
  for (int o = threadIdx.x; o < NO; o += kTG) {
    float s = 0.0f;
#pragma unroll 4
    for (int r = 0; r < kTG; ++r) s += D[r * kPad + o];
    outB[o] = s;
  }
}

template <int N>
__device__ __forceinline__ void put_row(float* tile, const float (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) tile[threadIdx.x * kPad + k] = v[k];
}

template <int N>
__device__ __forceinline__ void get_row(const float* tile, float (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = tile[threadIdx.x * kPad + k];
}

// g = W^T d for a 32-row layer (W row-major [32][K]): rows read in order, so that each weight
// row is one contiguous LDS read, accumulated into the K outputs.
template <int K>
__device__ __forceinline__ void tback(const float* __restrict__ W, const float (&d)[32], float (&g)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) g[i] = 0.0f;
#pragma unroll
  for (int o = 0; o < 32; ++o)
#pragma unroll
    for (int i = 0; i < K; ++i) g[i] = fmaf(W[o * K + i], d[o], g[i]);
}

// Per-record layer inputs of a block in LDS: H[0] = x, H[1..3] = hidden activations; D = deltas.
// LDS of a gradient block: one layer's inputs and that layer's deltas, a row per record (the
// hidden activations stay in the records' registers between the forward and the backward, so
// the two tiles serve every layer in turn and several blocks fit a CU).
struct GradTiles {
  float A[kTG * kPad];
  float D[kTG * kPad];  // also the block's loss scratch
};

// Backward of the block's rows from the output gradients dy, given each record's inputs x and
// hidden activations h1..h3 (as mlp32 leaves them): the block's weight gradients (layer-by-layer
// outer products of deltas and layer inputs) into `part`; dL/dx into dx.
template <int IN, int OUT>
__device__ __forceinline__ void backward_rows(const float* P, const float (&x)[IN], const float (&h1)[32],
                                              const float (&h2)[32], const float (&h3)[32], const float (&dy)[OUT],
                                              GradTiles& t, float* part, float (&dx)[IN]) {
  using Lo = L32<IN, OUT>;
  float d[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < OUT; ++k) s = fmaf(P[Lo::W4 + 32 * k + i], dy[k], s);
    d[i] = s * dleaky(h3[i]);
  }
  put_row(t.A, h3);
  put_row(t.D, dy);
  __syncthreads();
  tile_outer<OUT, 32>(t.A, t.D, part + Lo::W4, part + Lo::B4);
  __syncthreads();
  put_row(t.A, h2);
  put_row(t.D, d);  // delta of hidden layer 3
  __syncthreads();
  tile_outer<32, 32>(t.A, t.D, part + Lo::W3, part + Lo::B3);
  __syncthreads();
  {
    float g[32];
    tback<32>(P + Lo::W3, d, g);
#pragma unroll
    for (int i = 0; i < 32; ++i) d[i] = g[i] * dleaky(h2[i]);
  }
  put_row(t.A, h1);
  put_row(t.D, d);  // delta of hidden layer 2
  __syncthreads();
  tile_outer<32, 32>(t.A, t.D, part + Lo::W2, part + Lo::B2);
  __syncthreads();
  {
    float g[32];
    tback<32>(P + Lo::W2, d, g);
#pragma unroll
    for (int i = 0; i < 32; ++i) d[i] = g[i] * dleaky(h1[i]);
  }
  put_row(t.A, x);
  put_row(t.D, d);  // delta of hidden layer 1
  __syncthreads();
  tile_outer<32, IN>(t.A, t.D, part + Lo::W1, part + Lo::B1);
  __syncthreads();
  tback<IN>(P + Lo::W1, d, dx);
}

__device__ __forceinline__ void block_loss(float v, float* sh, float* out) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.0f;
#pragma unroll 4
    for (int k = 0; k < kTG; ++k) s += sh[k];
    *out = s;
  }
  __syncthreads();
}

__device__ __forceinline__ void load_raw(const NrrsRows& r, uint32_t row, float (&raw)[7], float& I) {
  const float* p = r.raw + 8ull * row;
#pragma unroll
  for (int k = 0; k < 7; ++k) raw[k] = p[k];
  I = p[7];
}

// Hash-grid gradient scatter of one level for the wave's records: (a, b) times each corner's
// weight added at the corner's two features.  The coarse levels are shared by many records (at
// level 0 every corner collects hundreds per step), so there the wave first adds the values of
// lanes with the same corner and issues one atomic per distinct corner; at the fine levels each
// lane adds its own.  (Per-lane atomics already add in no fixed order.)
constexpr int kAggLevels = 3;
__device__ __forceinline__ void scatter_level(float* gl, const Corner8& c, float a, float b, bool on, int l) {
  if (l >= kAggLevels) {
    if (on) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        atomicAdd(gl + 2ull * c.idx[k], c.w[k] * a);
        atomicAdd(gl + 2ull * c.idx[k] + 1, c.w[k] * b);
      }
    }
    return;
  }
  const uint32_t lane = __lane_id();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t idx = c.idx[k];
    const float va = c.w[k] * a, vb = c.w[k] * b;
    uint64_t pending = __ballot(on);
    while (pending) {  // wave-uniform: one round per distinct corner among the pending lanes
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const uint32_t key = (uint32_t)__shfl((int)idx, leader);
      const bool mine = ((pending >> lane) & 1ull) && idx == key;
      float sa = mine ? va : 0.0f, sb = mine ? vb : 0.0f;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        sa += __shfl_xor(sa, o);
        sb += __shfl_xor(sb, o);
      }
      if ((int)lane == leader) {
        atomicAdd(gl + 2ull * key, sa);
        atomicAdd(gl + 2ull * key + 1, sb);
      }
      pending &= ~__ballot(mine);
    }
  }
}

__global__ __launch_bounds__(kTG) void k_statnet_grad(NrrsRows r, const float* stat, const float* table, uint32_t log2T,
                                                      float eps, float* partial, float* loss_part, float* gtable) {
  __shared__ float ps[kStatParams];
  __shared__ GradTiles t;
  load_lds(ps, stat, kStatParams);
  __syncthreads();
  const uint32_t row = blockIdx.x * kTG + threadIdx.x;
  const bool valid = row < r.n;
  float raw[7] = {0, 0, 0, 0, 0, 0, 0}, I = 0.0f, L = 0.0f;
  if (valid) {
    load_raw(r, row, raw, I);
    if (r.acc) {
      const float lt = r.lum_t[row];
      L = lt > 0.0f ? fmaxf(r.acc[row], 0.0f) / lt : 0.0f;
    } else {
      L = r.target[row];
    }
  }
  float mv[2], enc[32], h1[32], h2[32], h3[32];
  statnet_encode(table, log2T, raw, enc);
  mlp32<kStatIn, kStatOut>(ps, enc, h1, h2, h3, mv);
  const float inv_n = 1.0f / (float)r.n;
  const float em = mv[0] - L;
  const float v1 = (L - mv[0]) * (L - mv[0]);  // one-sample variance about sg(m)
  const float ev = mv[1] - v1;
  float dy[2];
  dy[0] = valid ? 2.0f * em / (L * L + eps) * inv_n : 0.0f;
  dy[1] = valid ? 2.0f * ev / (v1 * v1 + eps) * inv_n : 0.0f;
  const float li = valid ? (em * em / (L * L + eps) + ev * ev / (v1 * v1 + eps)) * inv_n : 0.0f;
  float denc[32];
  backward_rows<kStatIn, kStatOut>(ps, enc, h1, h2, h3, dy, t, partial + (uint64_t)blockIdx.x * kStatParams, denc);
  block_loss(li, t.D, loss_part + blockIdx.x);
  {
    const uint64_t T = 1ull << log2T;
#pragma unroll
    for (int l = 0; l < kHgLevels; ++l) {
      Corner8 c;
      hg_corners(raw[0], raw[1], raw[2], l, log2T, c);
      scatter_level(gtable + (uint64_t)l * T * kHgFeat, c, denc[2 * l], denc[2 * l + 1], valid, l);
    }
  }
}

__global__ __launch_bounds__(kTG) void k_rrsnet_grad(NrrsRows r, const float* stat, const float* table, uint32_t log2T,
                                                     const float* rrs, int32_t step, const float* wpx,
                                                     const uint32_t* kpix, float g_rrs, float eps, float* partial,
                                                     float* loss_part) {
  __shared__ float ps[kStatParams];
  __shared__ float pr[kRrsParams];
  __shared__ GradTiles t;
  load_lds(ps, stat, kStatParams);
  load_lds(pr, rrs, kRrsParams);
  __syncthreads();
  const uint32_t row = blockIdx.x * kTG + threadIdx.x;
  const bool valid = row < r.n;
  float raw[7] = {0, 0, 0, 0, 0, 0, 0}, I = 0.0f;
  float4 tq = make_float4(0, 0, 0, 0);
  if (valid) {
    load_raw(r, row, raw, I);
    tq = r.tq[row];
  }
  // StatNet forward only (no gradient flows into it)
  float mv[2];
  {
    float enc[32], h1[32], h2[32], h3[32];
    statnet_encode(table, log2T, raw, enc);
    mlp32<kStatIn, kStatOut>(ps, enc, h1, h2, h3, mv);
  }
  float x[7], z[1], g1[32], g2[32], g3[32];
  rrs_inputs(mv[0], mv[1], tq.x, tq.y, tq.z, I, raw[6], x);
  mlp32<kRrsIn, 1>(pr, x, g1, g2, g3, z);
  const float q = softplus_mod(z[0]);
  float dq = 0.0f, li = 0.0f;
  if (valid) {
    if (step == 1) {
      const float inv_n = 1.0f / (float)r.n;
      dq = 2.0f * (q - 1.0f) / (1.0f + eps) * inv_n;
      li = (q - 1.0f) * (q - 1.0f) / (1.0f + eps) * inv_n;
    } else {
      const float2 qf = r.qf[row];
      if (qf.x > 0.0f) {
        const uint32_t p = r.pix[row];
        const uint32_t k = kpix[p];
        const float m = fmaxf(mv[0], 0.0f), v = fmaxf(mv[1], 0.0f);
        const float S = qf.x < 1.0f ? v + m * m : v;
        const float lt = r.lum_t[row];
        const float dvar = -(lt * lt) * S / (qf.x * qf.x);
        dq = (k ? wpx[p] / (float)k : 0.0f) * dvar * qf.y + 2.0f * g_rrs * (q - qf.x);
        li = g_rrs * (q - qf.x) * (q - qf.x);
      }
    }
  }
  float dy[1] = {dq * softplus_mod_grad(z[0])};
  float dx[7];
  backward_rows<kRrsIn, 1>(pr, x, g1, g2, g3, dy, t, partial + (uint64_t)blockIdx.x * kRrsParams, dx);
  block_loss(li, t.D, loss_part + blockIdx.x);
}

__global__ __launch_bounds__(kTG) void k_aid_grad(NrrsRows r, const float* stat, const float* table, uint32_t log2T,
                                                  const float* aid, const float* table_r, int32_t step,
                                                  const float* wpx, const uint32_t* kpix, float g_rrs, float eps,
                                                  float* partial, float* loss_part, float* gtable_r) {
  __shared__ float ps[kStatParams];
  __shared__ float pa[kAidParams];
  __shared__ GradTiles t;
  if (step != 1) load_lds(ps, stat, kStatParams);
  load_lds(pa, aid, kAidParams);
  __syncthreads();
  const uint32_t row = blockIdx.x * kTG + threadIdx.x;
  const bool valid = row < r.n;
  float raw[7] = {0, 0, 0, 0, 0, 0, 0}, I = 0.0f;
  float4 tq = make_float4(0, 0, 0, 0);
  if (valid) {
    load_raw(r, row, raw, I);
    tq = r.tq[row];
  }
  // StatNet supervises only: its statistics enter the transfer of step 2 (uniform branch)
  float mv[2] = {0.0f, 0.0f};
  if (step != 1) {
    float enc[32], h1[32], h2[32], h3[32];
    statnet_encode(table, log2T, raw, enc);
    mlp32<kStatIn, kStatOut>(ps, enc, h1, h2, h3, mv);
  }
  asm volatile("" ::: "memory");
  float z[1], enc[32], g1[32], g2[32], g3[32];
  aid_encode(table_r, log2T, raw, tq.x, tq.y, tq.z, I, enc);
  mlp32<kAidIn, 1>(pa, enc, g1, g2, g3, z);
  const float q = softplus_mod(z[0]);
  float dq = 0.0f, li = 0.0f;
  if (valid) {
    if (step == 1) {
      const float inv_n = 1.0f / (float)r.n;
      dq = 2.0f * (q - 1.0f) / (1.0f + eps) * inv_n;
      li = (q - 1.0f) * (q - 1.0f) / (1.0f + eps) * inv_n;
    } else {
      const float2 qf = r.qf[row];
      if (qf.x > 0.0f) {
        const uint32_t p = r.pix[row];
        const uint32_t k = kpix[p];
        const float m = fmaxf(mv[0], 0.0f), v = fmaxf(mv[1], 0.0f);
        const float S = qf.x < 1.0f ? v + m * m : v;
        const float lt = r.lum_t[row];
        const float dvar = -(lt * lt) * S / (qf.x * qf.x);
        dq = (k ? wpx[p] / (float)k : 0.0f) * dvar * qf.y + 2.0f * g_rrs * (q - qf.x);
        li = g_rrs * (q - qf.x) * (q - qf.x);
      }
    }
  }
  float dy[1] = {dq * softplus_mod_grad(z[0])};
  float dx[32];
  backward_rows<kAidIn, 1>(pa, enc, g1, g2, g3, dy, t, partial + (uint64_t)blockIdx.x * kAidParams, dx);
  block_loss(li, t.D, loss_part + blockIdx.x);
  {
    const uint64_t T = 1ull << log2T;
    const bool on = valid && dy[0] != 0.0f;
#pragma unroll
    for (int l = 0; l < kHgLevels; ++l) {
      Corner8 c;
      hg_corners(raw[0], raw[1], raw[2], l, log2T, c);
      scatter_level(gtable_r + (uint64_t)l * T * kHgFeat, c, dx[2 * l], dx[2 * l + 1], on, l);
    }
  }
}

// Fixed-order sum of the block partials: group g (of kSumGroups) adds blocks g, g + G, ... in
// order, then the groups are added in order — a fixed tree, with G times the parallelism of a
// plain loop over the blocks (one thread per parameter alone left most of the chip idle).
constexpr uint32_t kSumGroups = 32;
__global__ __launch_bounds__(256) void k_partial_sum_groups(const float* partial, uint32_t nb, uint32_t np,
                                                            float* group_sums) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y;
  if (p >= np) return;
  float s = 0.0f;
  for (uint32_t b = g; b < nb; b += kSumGroups) s += partial[(uint64_t)b * np + p];
  group_sums[(uint64_t)g * np + p] = s;
}

__global__ void k_partial_sum(const float* group_sums, uint32_t nb, uint32_t np, float* grad, const float* loss_part,
                              float* loss) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) {
    float s = 0.0f;
    for (uint32_t g = 0; g < kSumGroups; ++g) s += group_sums[(uint64_t)g * np + p];
    grad[p] = s;
  }
  if (p == 0 && loss) {
    float s = 0.0f;
    for (uint32_t b = 0; b < nb; ++b) s += loss_part[b];
    *loss = s;
  }
}

__global__ void k_adam(float* w, float* m, float* v, float* grad, uint64_t np, float c1, float c2, float lr,
                       float* infer, float decay, int zero_grad) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const float g = grad[k];
  const float mk = 0.9f * m[k] + 0.1f * g;
  const float vk = 0.999f * v[k] + 0.001f * g * g;
  m[k] = mk;
  v[k] = vk;
  const float wn = w[k] - lr * (mk / c1) / (sqrtf(vk / c2) + 1e-8f);
  w[k] = wn;
  infer[k] = decay > 0.0f ? fmaf(decay, infer[k] - wn, wn) : wn;
  if (zero_grad) grad[k] = 0.0f;
}

// ------------------------------------------------------------------ pixel error
__global__ void k_pixel_prep(PixelErrArgs p) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.w * p.h) return;
  const float ref = p.ref[i], cur = p.cur[i];
  const float acc = p.first ? cur : fmaf(p.a_mix, cur - p.acc[i], p.acc[i]);
  p.acc[i] = acc;
  p.Ep[i] = ref < 0.0f ? 0.0f : p.var_scale * (acc - ref) * (acc - ref) / (ref * ref + p.eps);
}

__global__ __launch_bounds__(256) void k_pixel_filter(PixelErrArgs p) {
  __shared__ double sh[2][256];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0, c = 0.0;
  if (i < p.w * p.h) {
    float E = 0.0f;
    if (p.ref[i] >= 0.0f) {
      const int x = (int)(i % p.w), y = (int)(i / p.w);
      float s = 0.0f;
      int n = 0;
      for (int dy = -p.radius; dy <= p.radius; ++dy)
        for (int dx = -p.radius; dx <= p.radius; ++dx) {
          const int xx = x + dx, yy = y + dy;
          if (xx < 0 || yy < 0 || xx >= (int)p.w || yy >= (int)p.h) continue;
          const uint32_t j = (uint32_t)yy * p.w + (uint32_t)xx;
          if (p.ref[j] < 0.0f) continue;
          s += p.Ep[j];
          ++n;
        }
      E = s / (float)n;
      e = E;
      c = 1.0;
    }
    p.E[i] = E;
  }
  sh[0][threadIdx.x] = e;
  sh[1][threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    p.part[2 * blockIdx.x] = sh[0][0];
    p.part[2 * blockIdx.x + 1] = sh[1][0];
  }
}

__global__ void k_pixel_eavg(PixelErrArgs p, uint32_t nb) {
  double s = 0.0, c = 0.0;
  for (uint32_t b = 0; b < nb; ++b) {
    s += p.part[2 * b];
    c += p.part[2 * b + 1];
  }
  *p.eavg = c > 0.0 ? s / c : 0.0;
}

__global__ void k_pixel_wpx(PixelErrArgs p) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.w * p.h) return;
  const float ref = p.ref[i];
  const float eavg = (float)*p.eavg;
  p.wpx[i] = ref < 0.0f ? 0.0f : (p.g_min + 2.0f * p.g_avg * (p.E[i] - eavg)) / (ref * ref + p.eps);
}

__global__ void k_frame_lum(const double* image, double* lum_start, uint32_t npx, double spp_frame, double spp_start,
                            float* cur, float* ref) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npx) return;
  const double l = (double)kLumR * image[3ull * i] + (double)kLumG * image[3ull * i + 1] +
                   (double)kLumB * image[3ull * i + 2];
  const double l0 = lum_start[i];
  cur[i] = (float)((l - l0) / spp_frame);
  ref[i] = spp_start > 0.0 ? (float)(l0 / spp_start) : -1.0f;
  lum_start[i] = l;
}

__global__ void k_count_pix(const uint32_t* pix, uint32_t n, uint32_t* kpix, uint32_t npx) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t p = pix[k];
  if (p < npx) atomicAdd(kpix + p, 1u);
}

__global__ void k_zero_u32_n(uint32_t* p, uint32_t n) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0u;
}

inline uint32_t blocks_of(uint64_t n, uint32_t t) { return (uint32_t)((n + t - 1) / t); }

}  // namespace

template <uint32_t L>
void launch_factor_t(const RenderArgs& a, const NrrsNet& n, dim3 g, bool aid, hipStream_t s) {
  if (aid) hipLaunchKernelGGL((k_nrrs_factor<true, L>), g, dim3(kT), 0, s, a, n);
  else hipLaunchKernelGGL((k_nrrs_factor<false, L>), g, dim3(kT), 0, s, a, n);
}

void launch_nrrs_factor(const RenderArgs& a, const NrrsNet& n, uint32_t blocks, bool aid, hipStream_t s) {
  // one build per table size (2^14 .. 2^22 entries per level, the sizes a context accepts):
  // with the level layout known, the dense / hashed choice and the level offsets are constants
  // and the kernel fits 5 waves per SIMD without spilling
  const dim3 g(std::max(blocks, 1u));
  switch (n.log2T) {
    case 14: launch_factor_t<14>(a, n, g, aid, s); break;
    case 15: launch_factor_t<15>(a, n, g, aid, s); break;
    case 16: launch_factor_t<16>(a, n, g, aid, s); break;
    case 17: launch_factor_t<17>(a, n, g, aid, s); break;
    case 18: launch_factor_t<18>(a, n, g, aid, s); break;
    case 19: launch_factor_t<19>(a, n, g, aid, s); break;
    case 20: launch_factor_t<20>(a, n, g, aid, s); break;
    case 21: launch_factor_t<21>(a, n, g, aid, s); break;
    default: launch_factor_t<22>(a, n, g, aid, s); break;
  }
}

void launch_aid_rows(const float* raw, const float* t, const float* I, uint32_t n, const NrrsNet& net, float* q,
                     float* enc, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_aid_rows, dim3(blocks_of(n, kT)), dim3(kT), 0, s, raw, t, I, n, net, q, enc);
}

void launch_aid_grad(const NrrsRows& r, const float* stat, const float* table, uint32_t log2T, const float* aid,
                     const float* table_r, int32_t step, const float* wpx, const uint32_t* kpix, float g_rrs,
                     float eps, float* partial, float* loss_part, float* gtable_r, hipStream_t s) {
  if (!r.n) return;
  hipLaunchKernelGGL(k_aid_grad, dim3(blocks_of(r.n, kTG)), dim3(kTG), 0, s, r, stat, table, log2T, aid, table_r,
                     step, wpx, kpix, g_rrs, eps, partial, loss_part, gtable_r);
}

void launch_record_qnorm(const RenderArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_record_qnorm, dim3(blocks_of(a.rec.cap, 256)), dim3(256), 0, s, a);
}

void launch_nrrs_rows(const float* raw, const float* t, const float* I, uint32_t n, const NrrsNet& net, float* mv,
                      float* q, float* enc, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_nrrs_rows, dim3(blocks_of(n, kT)), dim3(kT), 0, s, raw, t, I, n, net, mv, q, enc);
}

uint32_t nrrs_grad_blocks(uint32_t n) { return blocks_of(n, kTG); }

void launch_statnet_grad(const NrrsRows& r, const float* stat, const float* table, uint32_t log2T, float eps,
                         float* partial, float* loss_part, float* gtable, hipStream_t s) {
  if (!r.n) return;
  hipLaunchKernelGGL(k_statnet_grad, dim3(blocks_of(r.n, kTG)), dim3(kTG), 0, s, r, stat, table, log2T, eps, partial,
                     loss_part, gtable);
}

void launch_rrsnet_grad(const NrrsRows& r, const float* stat, const float* table, uint32_t log2T, const float* rrs,
                        int32_t step, const float* wpx, const uint32_t* kpix, float g_rrs, float eps, float* partial,
                        float* loss_part, hipStream_t s) {
  if (!r.n) return;
  hipLaunchKernelGGL(k_rrsnet_grad, dim3(blocks_of(r.n, kTG)), dim3(kTG), 0, s, r, stat, table, log2T, rrs, step, wpx,
                     kpix, g_rrs, eps, partial, loss_part);
}

void launch_partial_sum(const float* partial, uint32_t nblocks, uint32_t np, float* grad, const float* loss_part,
                        float* loss, float* group_sums, hipStream_t s) {
  hipLaunchKernelGGL(k_partial_sum_groups, dim3(blocks_of(np, 256), kSumGroups), dim3(256), 0, s, partial, nblocks,
                     np, group_sums);
  hipLaunchKernelGGL(k_partial_sum, dim3(blocks_of(np, 256)), dim3(256), 0, s, group_sums, nblocks, np, grad,
                     loss_part, loss);
}

uint32_t nrrs_sum_groups() { return kSumGroups; }

void launch_adam(float* w, float* m, float* v, float* grad, uint64_t np, uint64_t step, float lr, float* infer,
                 float decay, bool zero_grad, hipStream_t s) {
  const double t = (double)step;
  const float c1 = (float)(1.0 - std::pow(0.9, t)), c2 = (float)(1.0 - std::pow(0.999, t));
  hipLaunchKernelGGL(k_adam, dim3(blocks_of(np, 256)), dim3(256), 0, s, w, m, v, grad, np, c1, c2, lr, infer, decay,
                     zero_grad ? 1 : 0);
}

void launch_pixel_error(const PixelErrArgs& p, hipStream_t s) {
  const uint32_t npx = p.w * p.h, nb = blocks_of(npx, 256);
  hipLaunchKernelGGL(k_pixel_prep, dim3(nb), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_pixel_filter, dim3(nb), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_pixel_eavg, dim3(1), dim3(1), 0, s, p, nb);
  hipLaunchKernelGGL(k_pixel_wpx, dim3(nb), dim3(256), 0, s, p);
}

void launch_frame_lum(const double* image, double* lum_start, uint32_t npx, double spp_frame, double spp_start,
                      float* cur, float* ref, hipStream_t s) {
  hipLaunchKernelGGL(k_frame_lum, dim3(blocks_of(npx, 256)), dim3(256), 0, s, image, lum_start, npx, spp_frame,
                     spp_start, cur, ref);
}

void launch_count_pix(const uint32_t* pix, uint32_t n, uint32_t* kpix, uint32_t npx, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32_n, dim3(blocks_of(npx, 256)), dim3(256), 0, s, kpix, npx);
  if (n) hipLaunchKernelGGL(k_count_pix, dim3(blocks_of(n, 256)), dim3(256), 0, s, pix, n, kpix, npx);
}

}  // namespace nrrs
