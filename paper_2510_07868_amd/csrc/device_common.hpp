// Device-side building blocks shared by the gfx950 kernels: Philox4x32-10,
// float3 helpers, the BSDFs and the data layouts of the wavefront queues.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nrrs {

constexpr uint32_t kMiss = 0xffffffffu;
constexpr int kMaxRec = 4;           // training records carried per path (depths 1..4)
constexpr int kNParam = 9729;        // 20-64-64-64-1 network
constexpr int kGuardSteps = 32;      // alpha reductions counted in parallel by the overflow guard
constexpr double kAlphaMin = 1e-3;   // the guard reports an overflow once alpha falls below this
constexpr int kScanBlocks = 2048;    // blocks of the chunked reductions / scans
constexpr int kScanThreads = 256;
constexpr uint32_t kFlagDead = 1u;   // entry was emitted below the horizon: traced as nothing
constexpr uint32_t kFlagTrain = 2u;  // entry belongs to a training path
constexpr uint32_t kPurposeCamera = 0u, kPurposeRoulette = 1u, kPurposeChild = 2u, kPurposeTrain = 3u,
                   kPurposeNee = 4u;
constexpr float kLumR = 0.2126f, kLumG = 0.7152f, kLumB = 0.0722f;  // Rec. 709

// Parameter vector offsets: W1[64][20], b1, W2[64][64], b2, W3[64][64], b3, W4[64], b4.
constexpr int kW1 = 0, kB1 = 1280, kW2 = 1344, kB2 = 5440, kW3 = 5504, kB3 = 9600, kW4 = 9664, kB4 = 9728;

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplies with the Weyl-sequence key schedule.
__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r != 0) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const uint32_t a = c.x, b = c.z;
    const uint32_t hi_a = __umulhi(0xD2511F53u, a), lo_a = 0xD2511F53u * a;
    const uint32_t hi_b = __umulhi(0xCD9E8D57u, b), lo_b = 0xCD9E8D57u * b;
    c = make_uint4(hi_b ^ c.y ^ k.x, lo_b, hi_a ^ c.w ^ k.y, lo_a);
  }
  return c;
}

// Counter layout of every draw: (lineage id lo, lineage id hi, purpose | depth << 8, index).
__device__ __forceinline__ uint4 draw(uint2 key, uint2 lineage, uint32_t purpose, uint32_t depth, uint32_t j) {
  return philox(make_uint4(lineage.x, lineage.y, purpose | (depth << 8), j), key);
}

// 24 random bits -> [0, 1) on the 2^-24 grid (exact in float).
__device__ __forceinline__ float unit(uint32_t x) { return (float)(x >> 8) * 0x1.0p-24f; }

// ---------------------------------------------------------------------------------------
struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ V3 mul(V3 a, V3 b) { return v3(a.x * b.x, a.y * b.y, a.z * b.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 normalized(V3 a) { return rsqrtf(dot(a, a)) * a; }
__device__ __forceinline__ float lum(V3 c) { return kLumR * c.x + kLumG * c.y + kLumB * c.z; }
__device__ __forceinline__ V3 xyz(float4 f) { return v3(f.x, f.y, f.z); }
__device__ __forceinline__ float4 pack(V3 a, uint32_t w) { return make_float4(a.x, a.y, a.z, __uint_as_float(w)); }
__device__ __forceinline__ float4 pack(V3 a, float w) { return make_float4(a.x, a.y, a.z, w); }

// Frisvad-style branchless basis of Duff et al. (JCGT 2017) around unit n.
__device__ __forceinline__ void basis(V3 n, V3& t, V3& b) {
  const float s = n.z >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (s + n.z);
  const float c = n.x * n.y * a;
  t = v3(1.0f + s * n.x * n.x * a, s * c, -s * n.x);
  b = v3(c, s + n.y * n.y * a, -n.y);
}

// ---------------------------------------------------------------------------------------
// BSDFs (local frame, normal = +z).
// Lambertian: cosine-weighted direction, weight f cos / pdf = albedo.
__device__ __forceinline__ V3 sample_cosine(float u1, float u2) {
  const float r = sqrtf(u1);
  float s, c;
  sincosf(6.2831853071795864f * u2, &s, &c);
  return v3(r * c, r * s, sqrtf(fmaxf(0.0f, 1.0f - u1)));
}

__device__ __forceinline__ float ggx_lambda(float a, V3 w) {
  const float c2 = w.z * w.z;
  const float s2 = fmaxf(0.0f, 1.0f - c2);
  if (s2 <= 0.0f) return 0.0f;
  return 0.5f * (-1.0f + sqrtf(1.0f + a * a * s2 / c2));
}

// GGX visible-normal sample (Heitz, JCGT 2018): returns the reflected direction and the
// weight F * G2 / G1(wo) per channel (Cook-Torrance, height-correlated Smith, Schlick).
__device__ __forceinline__ bool sample_ggx(float a, V3 f0, V3 wo, float u1, float u2, V3& wi, V3& w) {
  const V3 s = normalized(v3(a * wo.x, a * wo.y, wo.z));
  const float l2 = s.x * s.x + s.y * s.y;
  V3 t1 = l2 > 0.0f ? rsqrtf(l2) * v3(-s.y, s.x, 0.0f) : v3(1.0f, 0.0f, 0.0f);
  V3 t2 = cross(s, t1);
  const float r = sqrtf(u1);
  float sn, cs;
  sincosf(6.2831853071795864f * u2, &sn, &cs);
  const float p1 = r * cs;
  const float mix = 0.5f * (1.0f + s.z);
  const float p2 = (1.0f - mix) * sqrtf(fmaxf(0.0f, 1.0f - p1 * p1)) + mix * (r * sn);
  const float p3 = sqrtf(fmaxf(0.0f, 1.0f - p1 * p1 - p2 * p2));
  const V3 nh = p1 * t1 + p2 * t2 + p3 * s;
  const V3 h = normalized(v3(a * nh.x, a * nh.y, fmaxf(0.0f, nh.z)));
  const float c = dot(wo, h);
  wi = (2.0f * c) * h - wo;
  if (wi.z <= 0.0f) {
    w = v3(0.0f, 0.0f, 0.0f);
    return false;
  }
  const float lo = ggx_lambda(a, wo);
  const float g_ratio = (1.0f + lo) / (1.0f + lo + ggx_lambda(a, wi));
  const float m = 1.0f - c;
  const float m5 = (m * m) * (m * m) * m;
  w = v3(f0.x + (1.0f - f0.x) * m5, f0.y + (1.0f - f0.y) * m5, f0.z + (1.0f - f0.z) * m5);
  w = g_ratio * w;
  return true;
}

// GGX normal distribution, the visible-normal sampling pdf of a reflected direction (solid
// angle: G1(wo) D(h) / (4 wo.z)) and f cos per channel (D G2 F / (4 wo.z)) — what light
// sampling needs to weigh a direction the BSDF could also have sampled.
__device__ __forceinline__ float ggx_D(float a, V3 h) {
  const float a2 = a * a;
  const float d = h.z * h.z * (a2 - 1.0f) + 1.0f;
  return a2 / (3.14159265358979323846f * d * d);
}

__device__ __forceinline__ float ggx_pdf(float a, V3 wo, V3 wi) {
  if (wo.z <= 0.0f || wi.z <= 0.0f) return 0.0f;
  const V3 h = normalized(wo + wi);
  return ggx_D(a, h) / ((1.0f + ggx_lambda(a, wo)) * 4.0f * wo.z);
}

__device__ __forceinline__ V3 ggx_eval_cos(float a, V3 f0, V3 wo, V3 wi) {
  if (wo.z <= 0.0f || wi.z <= 0.0f) return v3(0.0f, 0.0f, 0.0f);
  const V3 h = normalized(wo + wi);
  const float g2 = 1.0f / (1.0f + ggx_lambda(a, wo) + ggx_lambda(a, wi));
  const float m = 1.0f - dot(wo, h);
  const float m5 = (m * m) * (m * m) * m;
  const float k = ggx_D(a, h) * g2 / (4.0f * wo.z);
  return v3(k * (f0.x + (1.0f - f0.x) * m5), k * (f0.y + (1.0f - f0.y) * m5), k * (f0.z + (1.0f - f0.z) * m5));
}

// ---------------------------------------------------------------------------------------
// Device views of the scene and the queues.
struct DevScene {
  const float4* tri;    // 3 float4 per triangle in BVH order: (v0, orig id), (e1, material), (e2, 0)
  const float4* node;   // 4 float4 per BVH2 node (two child boxes + child links)
  const float4* node4;  // 8 float4 per 4-wide node: lo.x, hi.x, lo.y, hi.y, lo.z, hi.z, links, unused
  const float4* mat;    // 2 float4 per material: (rho rgb, ggx alpha), (Le rgb, type)
  uint32_t nt, nn, nm, nn4;
  float amin_x, amin_y, amin_z, extent, tmin, offset;
  float env_r, env_g, env_b;
  float eye_x, eye_y, eye_z, fwd_x, fwd_y, fwd_z, rx, ry, rz, ux, uy, uz;  // R, U pre-scaled
  // lights for next-event estimation: the emitting triangles in world space (3 float4 each, the
  // layout of tri), chosen with probability lum(L_e) x area through the CDF; that probability
  // per unit area is lum(L_e) x light_scale (light_scale = 1 / sum of lum(L_e) x area)
  const float4* light_geo;
  const float* light_cdf;  // nl + 1 entries, 0 .. 1
  float light_scale;
  uint32_t nl;
  // Two-level scenes (n_inst > 0): the traversal starts at node `root` of a tree over
  // instances, whose leaves (kInstLeaf set) list up to four instances; each instance is 7
  // float4: the rows of A^-1 with the translation t's components in w (a world point p maps to
  // A^-1 (p - t)), the rows of the object-to-world map (A | t), and (object tree's root link,
  // uid offset, material or kNoMat, first uid) as bits.
  // A hit's primitive id (uid) is the tri index k below nt_base (the non-instanced triangles),
  // else k + uid offset of its instance; inst_uid holds (first uid, record) pairs ascending by uid.
  const float4* inst;
  const uint32_t* inst_uid;
  uint32_t n_inst, root, nt_base;
};

constexpr uint32_t kInstLeaf = 4u;        // in a leaf link of the instance tree
constexpr uint32_t kExitInst = 0xFFFFFFFEu;  // stack entry: leave the instance, back to world space
constexpr uint32_t kNoMat = 0xFFFFFFFFu;     // instance keeps its triangles' own materials

struct Queue {
  float4* orig;  // origin xyz, excluded triangle (BVH index) bits
  float4* dir;   // unit direction xyz, pixel index bits
  float4* thr;   // throughput rgb, flag bits
  uint2* id;     // lineage id
  int4* rec;     // training-record ids of the depths 1..4 ancestors (-1 = none)
  uint32_t* path;  // primary path (index within the pass) the entry descends from; only when
                   // per-path radiance is traced
  float* pdf;      // solid-angle pdf with which the BSDF sampled the entry's direction (0 for a
                   // camera ray); only with next-event estimation
};

struct Records {
  float* feat;     // [cap][20]
  float* lum_t;    // [cap]
  float* acc;      // [cap] descendant emission luminance
  uint32_t* depth;
  uint32_t* pix;
  uint2* lineage;
  uint32_t* qidx;  // [cap] queue slot of the record's vertex at capture (features filled later)
  uint32_t* count;
  uint32_t cap;
  // NRRS training (reserved only with a hash grid): StatNet / RRSNet inputs of the vertex and
  // the factor the renderer applied
  float* nraw;     // [cap][8] position in the scene box scaled to [0,1]^3, w_o, remapped roughness, I_px
  float4* ntq;     // [cap] throughput (rgb), unused
  float2* nqf;     // [cap] normalized factor q_norm = F q and the normalization factor F
};

// Per-depth control block on the device (one per depth of a pass).
struct DepthCtl {
  uint32_t n;          // entries entering this depth
  uint32_t S;          // children emitted
  uint32_t guard;      // 1: the first roulette count overflowed the capacity
  uint32_t retries;    // alpha reductions applied
  double sumq;         // FP64 sum of the raw factors
  double F;            // normalization factor finally used
  uint32_t pad[2];
};

// The persistent traversal hands out the queue of one depth in kWorkSlices contiguous slices,
// each with its own claim counter (counters kWorkStride words apart), so that claims are
// spread over several addresses instead of serializing on one.
constexpr uint32_t kWorkSlices = 8;
constexpr uint32_t kWorkStride = 64;

// ---------------------------------------------------------------------------------------
// Wave64 helpers.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// One atomic per wave: lanes with `pred` receive consecutive slots from *counter.
__device__ __forceinline__ uint32_t wave_alloc(uint32_t* counter, bool pred) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return 0;
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if ((int)__lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = __shfl(base, leader);
  return base + lanes_below(m);
}

}  // namespace nrrs
