// Matrix-core inference of the RRS network on gfx950 (BF16 and FP8-E4M3, FP32 accumulate).
//
// Each wave evaluates path vertices in tiles of 32 as C[unit][vertex] = W[unit][k] * X[k][vertex]
// with v_mfma_f32_32x32x16_bf16 (BF16) or v_mfma_scale_f32_32x32x64_f8f6f4 (FP8).  The weights
// are the A operand, packed once per block into LDS in operand order.  BF16: every lane owns one
// vertex (64 per wave step, two tiles); its own features feed the input layer of its tile
// through weight tiles that are zero in the other lane half's K range, so no lane computes or
// exchanges another lane's features.  FP8: the lane pair (l, l+32) owns vertex l % 32.  The hidden units of every layer are consumed in the order in which the
// previous layer's accumulator registers hold them, so the accumulators of one layer become
// the B operand of the next with no data exchange: the packing kernel permutes the weight
// columns accordingly.  The 64 -> 1 output layer and the modified softplus (Sec. 5, Eq. 22)
// run on the vector ALUs.
//
// FP8: weights carry one FP32 scale per layer (amax / 448), applied to the accumulator;
// activations carry one power-of-two scale per vertex, given to the MFMA as its E8M0
// block-scale operand.
#include <algorithm>

#include "features.hpp"
#include "launch.hpp"

namespace nrrs {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8;
typedef short i16x2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
constexpr int kBfTiles = 28;   // layer 1: 2 vertex tiles x 2 unit tiles x 3 k-steps; layers 2, 3: 2 x 4
constexpr int kBfL1 = 12;      // first tile of layer 2
constexpr int kF8Tiles = 6;    // 2 unit tiles x 1 k-step (K = 64) per layer
constexpr float kE4M3Max = 448.0f;

// Row (unit) of accumulator register v held by lane half h in a 32x32 tile.
__host__ __device__ constexpr int acc_row(int v, int h) { return 8 * (v / 4) + 4 * h + (v % 4); }

// Hidden unit read by element i of lane half h of the BF16 B operand at k-step ks
// (k-step ks takes registers 8 (ks % 2) .. +7 of accumulator tile ks / 2).
__device__ __forceinline__ int bf16_unit(int ks, int h, int i) { return 32 * (ks / 2) + acc_row(8 * (ks % 2) + i, h); }
// Hidden unit read by byte i of lane half h of the FP8 B operand (registers of tile i / 16).
__device__ __forceinline__ int fp8_unit(int h, int i) { return 32 * (i / 16) + acc_row(i % 16, h); }

// float -> OCP E4M3 (bias 7, max 448, no infinities), round to nearest even, saturating.
__device__ __forceinline__ uint32_t to_e4m3(float x) {
  const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  if (!(a == a)) return 0x7Fu;
  if (a >= kE4M3Max) return sign | 0x7Eu;
  const uint32_t u = __float_as_uint(a);
  const int e = (int)(u >> 23) - 127;
  if (e < -6) {  // subnormal: multiples of 2^-9
    const uint32_t m = (uint32_t)rintf(a * 512.0f);
    return sign | m;  // m == 8 is the smallest normal, same bits
  }
  const uint32_t r = u & 0x7FFFFFu;
  uint32_t m = r >> 20;
  const uint32_t rest = r & 0xFFFFFu;
  if (rest > 0x80000u || (rest == 0x80000u && (m & 1u))) ++m;
  int ee = e + 7;
  if (m == 8u) {
    m = 0;
    ++ee;
  }
  uint32_t code = ((uint32_t)ee << 3) | m;
  if (code > 0x7Eu) code = 0x7Eu;
  return sign | code;
}

__device__ __forceinline__ uint16_t to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float softplus_mod(float z) { return z < 0.0f ? log1pf(expf(z)) : 0.5f * z + 0.69314718055994531f; }

// ------------------------------------------------------------------------- packing
// Per-layer FP8 weight scales: amax / 448 of W1, W2, W3.
__global__ void k_fp8_scales(const float* W, float* scale) {
  __shared__ float sh[256];
  const int offs[3] = {kW1, kW2, kW3}, cnt[3] = {1280, 4096, 4096};
  for (int L = 0; L < 3; ++L) {
    float m = 0.0f;
    for (int k = threadIdx.x; k < cnt[L]; k += 256) m = fmaxf(m, fabsf(W[offs[L] + k]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
      __syncthreads();
    }
    if (threadIdx.x == 0) scale[L] = sh[0] > 0.0f ? sh[0] / kE4M3Max : 1.0f;
    __syncthreads();
  }
}

// One thread per packed element: BF16 tiles [tile][lane][8], FP8 tiles [tile][lane][32].
__global__ void k_pack(const float* W, const float* f8scale, uint16_t* bf, uint8_t* f8) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < (uint32_t)kBfTiles * 64 * 8) {
    const int t = g / 512, l = (g / 8) % 64, i = g % 8, h = l / 32;
    float w = 0.0f;
    if (t < kBfL1) {
      // input layer, vertex tile vt: only lane half vt carries feature 8 j + i, the other half's
      // K range is zero
      const int vt = t / 6, mt = (t / 3) % 2, j = t % 3, m = 32 * mt + l % 32, k = 8 * j + i;
      w = (h == vt && k < 20) ? W[kW1 + 20 * m + k] : 0.0f;
    } else {
      const int base = t < kBfL1 + 8 ? kW2 : kW3, tt = (t - kBfL1) % 8, mt = tt / 4, ks = tt % 4, m = 32 * mt + l % 32;
      w = W[base + 64 * m + bf16_unit(ks, h, i)];
    }
    bf[g] = to_bf16_bits(w);
  }
  if (g < (uint32_t)kF8Tiles * 64 * 32) {
    const int t = g / 2048, l = (g / 32) % 64, i = g % 32, h = l / 32, L = t / 2, mt = t % 2, m = 32 * mt + l % 32;
    float w;
    if (L == 0) {
      const int k = 32 * h + i;
      w = k < 20 ? W[kW1 + 20 * m + k] : 0.0f;
    } else {
      w = W[(L == 1 ? kW2 : kW3) + 64 * m + fp8_unit(h, i)];
    }
    f8[g] = (uint8_t)to_e4m3(w / f8scale[L]);
  }
}

// ------------------------------------------------------------------------- inference
struct Smem {
  float b[3][64];  // biases
  float w4[64];
  float b4;
  float s[3];      // FP8 per-layer weight scales
};

__device__ __forceinline__ void load_smem(Smem& sm, const float* W, const float* f8scale, bool fp8) {
  for (int k = threadIdx.x; k < 64; k += blockDim.x) {
    sm.b[0][k] = W[kB1 + k];
    sm.b[1][k] = W[kB2 + k];
    sm.b[2][k] = W[kB3 + k];
    sm.w4[k] = W[kW4 + k];
  }
  if (threadIdx.x == 0) {
    sm.b4 = W[kB4];
    for (int L = 0; L < 3; ++L) sm.s[L] = fp8 ? f8scale[L] : 1.0f;
  }
  __syncthreads();
}

__device__ __forceinline__ f32x16 bias_tile(const float* b, int mt, int h) {
  f32x16 c;
#pragma unroll
  for (int v = 0; v < 16; ++v) c[v] = b[32 * mt + acc_row(v, h)];
  return c;
}

// max(x, 0) as a signed-integer maximum of the bits: the same value for every non-NaN x
// (negative values and -0 give +0), without the NaN-quieting canonicalization an IEEE fmaxf
// needs on each operand.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// ReLU after the BF16 rounding, as a packed 16-bit integer maximum of each value pair with 0:
// a BF16 value with the sign bit set reads as a negative integer, so every negative value (and
// -0) becomes +0 and every other value is kept; rounding to nearest commutes with max(x, 0),
// so the bits equal those of rounding the ReLU output, at half the vector instructions.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef short i16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16x8 relu_bf16(const f32x16& c, int first) {
  int r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // one packed round-to-nearest-even conversion per pair, then the packed ReLU
    const bf16x2v b = __builtin_convertvector((f32x2){c[first + 2 * k], c[first + 2 * k + 1]}, bf16x2v);
    r[k] = __builtin_bit_cast(int, __builtin_elementwise_max(__builtin_bit_cast(i16x2v, b), (i16x2v)0));
  }
  return __builtin_bit_cast(bf16x8, r);
}

__device__ __forceinline__ float output_layer(const Smem& sm, const f32x16& c0, const f32x16& c1, int h) {
  float z = 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    z = fmaf(sm.w4[acc_row(v, h)], relu(c0[v]), z);
    z = fmaf(sm.w4[32 + acc_row(v, h)], relu(c1[v]), z);
  }
  z += __shfl_xor(z, 32);
  return z + sm.b4;
}

// Hidden layers 2, 3 and the output layer of one 32-vertex tile from its input-layer
// accumulators; returns z of vertex l % 32 (in both lane halves).
// Test entry point only: the BF16 bit patterns of this lane's 32 activations of hidden layer L
// (row crow of the vertex whose column the lane holds), in unit order.
// The whole vector is reinterpreted at once: with this compiler, a bit cast of one subscripted
// element of these vectors returned the first element for every index.
typedef __attribute__((__vector_size__(8 * sizeof(uint16_t)))) uint16_t u16x8;
__device__ __forceinline__ void store_codes_bf16(uint16_t* crow, int L, int h, bf16x8 b0, bf16x8 b1, bf16x8 b2,
                                                 bf16x8 b3) {
  const u16x8 u0 = __builtin_bit_cast(u16x8, b0), u1 = __builtin_bit_cast(u16x8, b1);
  const u16x8 u2 = __builtin_bit_cast(u16x8, b2), u3 = __builtin_bit_cast(u16x8, b3);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    crow[64 * L + acc_row(i, h)] = u0[i];
    crow[64 * L + acc_row(8 + i, h)] = u1[i];
    crow[64 * L + 32 + acc_row(i, h)] = u2[i];
    crow[64 * L + 32 + acc_row(8 + i, h)] = u3[i];
  }
}

template <bool kCodes = false>
__device__ __forceinline__ float bf16_hidden(const bf16x8* __restrict__ w, const Smem& sm, f32x16 c0, f32x16 c1,
                                             int h, uint16_t* crow = nullptr) {
#pragma unroll
  for (int L = 1; L < 3; ++L) {
    const bf16x8 b0 = relu_bf16(c0, 0), b1 = relu_bf16(c0, 8), b2 = relu_bf16(c1, 0), b3 = relu_bf16(c1, 8);
    if constexpr (kCodes)
      if (crow) store_codes_bf16(crow, L, h, b0, b1, b2, b3);
    const int t = kBfL1 + 8 * (L - 1);
    c0 = bias_tile(sm.b[L], 0, h);
    c1 = bias_tile(sm.b[L], 1, h);
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (t + 0)], b0, c0, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (t + 1)], b1, c0, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (t + 2)], b2, c0, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (t + 3)], b3, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (t + 4)], b0, c1, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (t + 5)], b1, c1, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (t + 6)], b2, c1, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (t + 7)], b3, c1, 0, 0, 0);
  }
  return output_layer(sm, c0, c1, h);
}

// BF16: every lane passes its own vertex's features and gets that vertex's output
// pre-activation z.  Lanes 0-31 form vertex tile 0, lanes 32-63 tile 1.
// cstep (test entry point only): code rows of the step's 64 vertices, of which nleft exist.
template <bool kCodes = false>
__device__ __forceinline__ float mlp_bf16(const bf16x8* __restrict__ wl, const Smem& sm, const float f[20],
                                          uint16_t* cstep = nullptr, uint32_t nleft = 0) {
  const bf16x8* w = wl + __lane_id();  // this lane's part of tile t is w[64 t]
  const int h = (int)(__lane_id() >> 5);
  bf16x8 x[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 8; ++i) x[j][i] = (__bf16)(8 * j + i < 20 ? f[(8 * j + i) % 20] : 0.0f);
  if constexpr (kCodes) {
    if (__lane_id() < nleft)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const u16x8 u = __builtin_bit_cast(u16x8, x[j]);
#pragma unroll
        for (int i = 0; i < 8; ++i) cstep[192 * __lane_id() + 8 * j + i] = u[i];
      }
  }
  float z[2];
#pragma unroll
  for (int vt = 0; vt < 2; ++vt) {
    // re-read the weights from LDS for the second tile rather than keep them in registers
    asm volatile("" ::: "memory");
    f32x16 c0 = bias_tile(sm.b[0], 0, h), c1 = bias_tile(sm.b[0], 1, h);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (6 * vt + j)], x[j], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[64 * (6 * vt + 3 + j)], x[j], c1, 0, 0, 0);
    }
    uint16_t* crow = nullptr;
    if constexpr (kCodes) {
      const uint32_t v = 32u * vt + (__lane_id() & 31u);  // the vertex whose column this lane holds
      if (v < nleft) crow = cstep + 192ull * v;
    }
    z[vt] = bf16_hidden<kCodes>(w, sm, c0, c1, h, crow);
  }
  return h ? z[1] : z[0];
}

// Power-of-two scale (E8M0 code) shared by the two lanes of a vertex, so that the vertex's
// largest activation fits E4M3, and this lane's 32 packed bytes.  One scale per vertex keeps
// the result independent of how the hardware groups K into scale blocks.
__device__ __forceinline__ i32x8 quant_block(const float (&x)[32], int& scale_code) {
  float amax = 0.0f;
#pragma unroll
  for (int i = 0; i < 32; ++i) amax = fmaxf(amax, fabsf(x[i]));
  amax = fmaxf(amax, __shfl_xor(amax, 32));
  // smallest e with 2^e >= amax / 448 (exact: from the binary exponent of the quotient)
  int e = 0;
  const float ratio = amax / kE4M3Max;
  if (ratio > 0.0f) {
    int ex;
    const float m = frexpf(ratio, &ex);  // ratio = m 2^ex, m in [0.5, 1)
    e = (m == 0.5f) ? ex - 1 : ex;
  }
  e = max(-120, min(120, e));
  scale_code = 127 + e;
  // hardware conversion of x / 2^e (OCP E4M3, round to nearest even; the scale keeps every
  // value within +-448, so saturation never applies): same bytes as to_e4m3(ldexpf(x, -e))
  const float sc = ldexpf(1.0f, e);
  i32x8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const i16x2 lo = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(i16x2{0, 0}, x[4 * j], x[4 * j + 1], sc, false);
    const i16x2 hi = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(lo, x[4 * j + 2], x[4 * j + 3], sc, true);
    r[j] = __builtin_bit_cast(int, hi);
  }
  return r;
}

// Test entry point only: this lane's 32 E4M3 codes of layer L (0 = inputs) and the layer's
// block-scale exponent, into row crow of the lane pair's vertex.
__device__ __forceinline__ void store_codes_fp8(uint16_t* crow, int8_t* serow, int L, int h, const i32x8& xb, int sx) {
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const uint16_t b = (uint16_t)(((uint32_t)xb[i / 4] >> (8 * (i % 4))) & 0xFFu);
    crow[64 * L + (L == 0 ? 32 * h + i : fp8_unit(h, i))] = b;
  }
  if (h == 0) serow[L] = (int8_t)(sx - 127);
}

template <bool kCodes = false>
__device__ __forceinline__ float mlp_fp8(const i32x8* __restrict__ wl, const Smem& sm, const float f[20],
                                         uint16_t* crow = nullptr, int8_t* serow = nullptr) {
  const i32x8* w = wl + __lane_id();  // this lane's part of tile t is w[64 t]
  const int h = (int)(__lane_id() >> 5);
  float x[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) x[i] = (h == 0 && i < 20) ? f[i % 20] : 0.0f;
  int sx;
  i32x8 xb = quant_block(x, sx);
  if constexpr (kCodes)
    if (crow) store_codes_fp8(crow, serow, 0, h, xb, sx);
  f32x16 c0 = {}, c1 = {};
  c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(w[64 * (0)], xb, c0, 0, 0, 0, 127, 0, sx);
  c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(w[64 * (1)], xb, c1, 0, 0, 0, 127, 0, sx);
#pragma unroll
  for (int L = 1; L < 3; ++L) {
    // previous layer: scale, bias, ReLU -> this layer's B operand (registers in unit order)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      x[v] = fmaxf(fmaf(c0[v], sm.s[L - 1], sm.b[L - 1][acc_row(v, h)]), 0.0f);
      x[16 + v] = fmaxf(fmaf(c1[v], sm.s[L - 1], sm.b[L - 1][32 + acc_row(v, h)]), 0.0f);
    }
    xb = quant_block(x, sx);
    if constexpr (kCodes)
      if (crow) store_codes_fp8(crow, serow, L, h, xb, sx);
    c0 = f32x16{};
    c1 = f32x16{};
    c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(w[64 * (2 * L)], xb, c0, 0, 0, 0, 127, 0, sx);
    c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(w[64 * (2 * L + 1)], xb, c1, 0, 0, 0, 127, 0, sx);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    c0[v] = fmaf(c0[v], sm.s[2], sm.b[2][acc_row(v, h)]);
    c1[v] = fmaf(c1[v], sm.s[2], sm.b[2][32 + acc_row(v, h)]);
  }
  return output_layer(sm, c0, c1, h);
}

// Packed weights live in LDS (one copy per block); each MFMA reads its lane's 16 or 32 bytes.
template <int P>
struct Weights;
template <>
struct Weights<1> {
  static constexpr int kVerts = 64;  // vertices per wave step: one per lane
  static constexpr int kBytes = kBfTiles * 64 * 16;
  const bf16x8* lds;
  __device__ void load(const NetArgs& n, void* smem) {
    const uint4* src = reinterpret_cast<const uint4*>(n.bf16);
    uint4* dst = reinterpret_cast<uint4*>(smem);
    for (int k = threadIdx.x; k < kBytes / 16; k += blockDim.x) dst[k] = src[k];
    lds = reinterpret_cast<const bf16x8*>(smem);
  }
  __device__ float eval(const Smem& sm, const float f[20]) const { return mlp_bf16(lds, sm, f); }
  // test entry point: also the codes of the step's vertices (rows cstep, nleft of them)
  __device__ float eval_codes(const Smem& sm, const float f[20], uint16_t* cstep, int8_t*, uint32_t nleft) const {
    return mlp_bf16<true>(lds, sm, f, cstep, nleft);
  }
};
template <>
struct Weights<2> {
  static constexpr int kVerts = 32;  // vertices per wave step: one per lane pair
  static constexpr int kBytes = kF8Tiles * 64 * 32;
  const i32x8* lds;
  __device__ void load(const NetArgs& n, void* smem) {
    const uint4* src = reinterpret_cast<const uint4*>(n.fp8);
    uint4* dst = reinterpret_cast<uint4*>(smem);
    for (int k = threadIdx.x; k < kBytes / 16; k += blockDim.x) dst[k] = src[k];
    lds = reinterpret_cast<const i32x8*>(smem);
  }
  __device__ float eval(const Smem& sm, const float f[20]) const { return mlp_fp8(lds, sm, f); }
  __device__ float eval_codes(const Smem& sm, const float f[20], uint16_t* cstep, int8_t* sestep,
                              uint32_t nleft) const {
    // every lane runs the same code (matrix-core and cross-lane operations need the whole
    // wave); only the stores of lanes past the last vertex are skipped
    const uint32_t v = __lane_id() & 31u;  // the lane pair's vertex
    uint16_t* crow = v < nleft ? cstep + 192ull * v : nullptr;
    int8_t* serow = v < nleft ? sestep + 3ull * v : nullptr;
    return mlp_fp8<true>(lds, sm, f, crow, serow);
  }
};

// Network factors for the vertices of one depth: persistent waves over tiles of 32 entries.
// At most 128 VGPRs (4 waves per SIMD), so that one wave's vector epilogue overlaps other
// waves' matrix-core work.
template <int P>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_rrsnet_mfma(RenderArgs a,
                                                                                                 NetArgs net) {
  __shared__ Smem sm;
  __shared__ __attribute__((aligned(16))) uint8_t wsm[Weights<P>::kBytes];
  Weights<P> W;
  W.load(net, wsm);
  load_smem(sm, net.master, net.fp8_scale, P == 2);
  constexpr uint32_t kV = Weights<P>::kVerts;
  const uint32_t n = a.ctl[a.depth].n;
  const uint32_t tiles = (n + kV - 1) / kV;
  const uint32_t wave = blockIdx.x * (kThreads / 64) + threadIdx.x / 64;
  const uint32_t waves = gridDim.x * (kThreads / 64);
  const uint32_t lane = __lane_id();
  for (uint32_t tile = wave; tile < tiles; tile += waves) {
    // keep the weights in LDS: re-read them every tile instead of pinning ~80 registers
    asm volatile("" ::: "memory");
    const uint32_t i = tile * kV + (lane & (kV - 1));
    bool active = false;
    float f[20];
    float g = 0.0f, lt = 0.0f, qh = 0.0f;
#pragma unroll
    for (int k = 0; k < 20; ++k) f[k] = 0.0f;
    if (i < n) qh = a.q[i];
    if (i < n && qh > 0.0f) {
      const float4 dr = a.qin.dir[i];
      g = a.guide[__float_as_uint(dr.w)];
      if (g >= 0.0f) {
        active = true;
        const float4 th = a.qin.thr[i], vp = a.vpos[i], vn = a.vnrm[i];
        const uint32_t mid = __float_as_uint(vn.w);
        const float4 m0 = a.sc.mat[2 * mid], m1 = a.sc.mat[2 * mid + 1];
        vertex_features(a.sc, xyz(vp), xyz(vn), v3(-dr.x, -dr.y, -dr.z), xyz(th), m0, __float_as_uint(m1.w),
                        a.depth, a.max_depth, f);
        lt = lum(xyz(th));
      }
    }
    const float z = W.eval(sm, f);
    if (active && lane < kV) a.q[i] = network_factor(lt, softplus_mod(z), g, qh);
  }
}

template <int P, bool kCodes = false>
__global__ __launch_bounds__(kThreads) void k_rows_mfma(const float* x, uint32_t n, NetArgs net, float* y, float* zout,
                                                      uint16_t* codes = nullptr, int8_t* scale_exp = nullptr) {
  __shared__ Smem sm;
  __shared__ __attribute__((aligned(16))) uint8_t wsm[Weights<P>::kBytes];
  Weights<P> W;
  W.load(net, wsm);
  load_smem(sm, net.master, net.fp8_scale, P == 2);
  constexpr uint32_t kV = Weights<P>::kVerts;
  const uint32_t tiles = (n + kV - 1) / kV;
  const uint32_t wave = blockIdx.x * (kThreads / 64) + threadIdx.x / 64;
  const uint32_t waves = gridDim.x * (kThreads / 64);
  const uint32_t lane = __lane_id();
  for (uint32_t tile = wave; tile < tiles; tile += waves) {
    asm volatile("" ::: "memory");
    const uint32_t i = tile * kV + (lane & (kV - 1));
    float f[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) f[k] = i < n ? x[20ull * i + k] : 0.0f;
    float z;
    if constexpr (kCodes)
      z = W.eval_codes(sm, f, codes + 192ull * tile * kV, scale_exp + 3ull * tile * kV, n - tile * kV);
    else
      z = W.eval(sm, f);
    if (i < n && lane < kV) {
      y[i] = softplus_mod(z);
      if (zout) zout[i] = z;
    }
  }
}

// Persistent grid: CUs x resident blocks, one cached value per kernel variant.
template <typename K>
uint32_t grid_for(K kernel, int slot) {
  static uint32_t blocks[4] = {0, 0, 0, 0};
  if (blocks[slot] == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kThreads, 0) != hipSuccess || per < 1) per = 1;
    blocks[slot] = (uint32_t)(std::max(cus, 1) * per);
  }
  return blocks[slot];
}

}  // namespace

uint32_t packed_bf16_elems() { return kBfTiles * 64 * 8; }
uint32_t packed_fp8_bytes() { return kF8Tiles * 64 * 32; }

void warm_mfma_launch_cache() {
  grid_for(k_rrsnet_mfma<1>, 0);
  grid_for(k_rrsnet_mfma<2>, 1);
  grid_for(k_rows_mfma<1>, 2);
  grid_for(k_rows_mfma<2>, 3);
}

void launch_pack_weights(const float* master, uint16_t* bf16, uint8_t* fp8, float* fp8_scale, hipStream_t s) {
  hipLaunchKernelGGL(k_fp8_scales, dim3(1), dim3(256), 0, s, master, fp8_scale);
  const uint32_t n = std::max(packed_bf16_elems(), packed_fp8_bytes());
  hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, s, master, fp8_scale, bf16, fp8);
}

void launch_rrsnet_mfma(const RenderArgs& a, const NetArgs& n, hipStream_t s) {
  if (n.precision == 2)
    hipLaunchKernelGGL(k_rrsnet_mfma<2>, dim3(grid_for(k_rrsnet_mfma<2>, 1)), dim3(kThreads), 0, s, a, n);
  else
    hipLaunchKernelGGL(k_rrsnet_mfma<1>, dim3(grid_for(k_rrsnet_mfma<1>, 0)), dim3(kThreads), 0, s, a, n);
}

void launch_codes_mfma(const float* x, uint32_t n, const NetArgs& net, float* y, uint16_t* codes, int8_t* scale_exp,
                       hipStream_t s) {
  if (!n) return;
  const uint32_t blocks = (n + 4 * 32 - 1) / (4 * 32);
  if (net.precision == 2)
    hipLaunchKernelGGL((k_rows_mfma<2, true>), dim3(blocks), dim3(kThreads), 0, s, x, n, net, y, nullptr, codes,
                       scale_exp);
  else
    hipLaunchKernelGGL((k_rows_mfma<1, true>), dim3(blocks), dim3(kThreads), 0, s, x, n, net, y, nullptr, codes,
                       scale_exp);
}

void launch_rows_mfma(const float* x, uint32_t n, const NetArgs& net, float* y, float* z, hipStream_t s) {
  if (!n) return;
  if (net.precision == 2)
    hipLaunchKernelGGL(k_rows_mfma<2>, dim3(grid_for(k_rows_mfma<2>, 3)), dim3(kThreads), 0, s, x, n, net, y, z);
  else
    hipLaunchKernelGGL(k_rows_mfma<1>, dim3(grid_for(k_rows_mfma<1>, 2)), dim3(kThreads), 0, s, x, n, net, y, z);
}

}  // namespace nrrs
