// gfx950 kernels of one wavefront bounce: camera spawn, BVH closest hit (extend), shading,
// FP64 sum of the RRS factors, normalization + stochastic rounding + overflow guard +
// exclusive scan, and the split/compaction expansion into the next queue.
//
// Method (NRRS, arXiv 2510.07868): per-depth normalization q_norm = F q, F = N / sum q
// (Sec. 4.1.2, Eqs. 9-11) with rate control and adaptive alpha (Sec. 4.1.4, Eqs. 12-14),
// child counts by stochastic rounding (Sec. 3, Eq. 8), lights and misses end paths
// (Sec. 3 "Wavefront Architecture").  The entry counts of every depth live on the device,
// so a whole pass is launched without a host round trip.
#include <algorithm>

#include "features.hpp"
#include "claim.hpp"
#include "launch.hpp"

namespace nrrs {

namespace {

constexpr int kEntryThreads = 256;
constexpr int kShadeThreads = 1024;
constexpr int kTraceThreads = 128;
constexpr int kLdsStack = 16;     // stack entries per lane kept in LDS
constexpr int kStackMax = 96;     // total stack entries per lane
// Modes 0 and 1 push at most one entry per tree level (depth <= kMaxBvhDepth).  Mode 2 also
// parks extra leaf links, but only while fewer than kLeafPushLimit entries are stacked, so
// the stack never exceeds kLeafPushLimit + 3 + kMaxBvhDepth <= kStackMax entries.
constexpr int kLeafPushLimit = kStackMax - 3 - kMaxBvhDepth;
static_assert(kLeafPushLimit > 0, "traversal stack too small");
static_assert(3 * kMaxBvh4Depth + 1 <= kStackMax, "traversal stack too small for the 4-wide tree");
constexpr uint32_t kLeafBit = 0x80000000u;

__device__ __forceinline__ uint32_t bits(float f) { return __float_as_uint(f); }

// ------------------------------------------------------------------------------ camera
__global__ __launch_bounds__(kEntryThreads) void k_camera(RenderArgs a) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) {
    a.ctl[1].n = a.nprim;
    a.ctl[a.max_depth].S = 0;
  }
  if (k < (a.max_depth + 1) * kWorkSlices) {
    a.work[(uint64_t)k * kWorkStride] = 0;
    if (a.nee) a.work_nee[(uint64_t)k * kWorkStride] = 0;
  }
  if (k >= a.nprim) return;
  // primary path k is sample k mod s_batch of pixel k / s_batch: a pixel's paths stay adjacent
  const uint32_t s_batch = a.nprim / (a.width * a.height);
  const uint32_t pix = k / s_batch;
  const uint32_t px = pix % a.width, py = pix / a.width;
  const uint2 lin = make_uint2(k, a.pass_state->pass);
  const uint4 r = draw(a.key, lin, kPurposeCamera, 0, 0);
  const float sx = 2.0f * ((float)px + unit(r.x)) / (float)a.width - 1.0f;
  const float sy = 1.0f - 2.0f * ((float)py + unit(r.y)) / (float)a.height;
  const DevScene& c = a.sc;
  const V3 d = normalized(v3(c.fwd_x + sx * c.rx + sy * c.ux, c.fwd_y + sx * c.ry + sy * c.uy,
                             c.fwd_z + sx * c.rz + sy * c.uz));
  uint32_t flags = 0;
  if (a.records_on) {
    const uint4 rt = draw(a.key, lin, kPurposeTrain, 0, 0);
    if (unit(rt.x) < a.p_train) flags |= kFlagTrain;
  }
  a.qin.orig[k] = make_float4(c.eye_x, c.eye_y, c.eye_z, __uint_as_float(kMiss));
  a.qin.dir[k] = pack(d, pix);
  a.qin.thr[k] = make_float4(1.0f, 1.0f, 1.0f, __uint_as_float(flags));
  a.qin.id[k] = lin;
  if (a.trace) a.qin.path[k] = k;
  if (a.nee) a.qin.pdf[k] = 0.0f;
  // record slots travel only with training paths (every reader checks kFlagTrain first)
  if (flags & kFlagTrain) a.qin.rec[k] = make_int4(-1, -1, -1, -1);
}

// ------------------------------------------------------------------------------ extend
// Conservative slab test.  A plane distance is computed as fma(l, inv, oi) with oi = -o * inv
// rounded once, so it errs by at most 2u |t| + u |oi| (u = 2^-24): relative to t, plus an
// absolute part from the rounding of oi that does not shrink with t (a box near an origin far
// from the coordinate origin).  The far distance is therefore widened by 2^-20 relative and by
// a per-ray eps = 2^-22 max|oi| absolute, which covers both errors on both ends, so rounding
// does not cull a box that the exact ray touches.  eps takes |oi| only over the axes the ray is
// not nearly parallel to (|d| >= 2^-10, bounding eps by 2^-12 |o|): on a nearly parallel axis
// |oi| is huge and would open every box.  The one case left uncovered is a box whose entry or
// exit is decided by a face the ray runs within 2^-10 of parallel to, with the exact overlap
// below u |o| / |d| on that axis: a grazing pass along a box face.
__device__ __forceinline__ bool slab(float lx, float ly, float lz, float hx, float hy, float hz, V3 inv, V3 oi,
                                     float eps, float tmax, float& tnear) {
  const float t0x = fmaf(lx, inv.x, oi.x), t1x = fmaf(hx, inv.x, oi.x);
  const float t0y = fmaf(ly, inv.y, oi.y), t1y = fmaf(hy, inv.y, oi.y);
  const float t0z = fmaf(lz, inv.z, oi.z), t1z = fmaf(hz, inv.z, oi.z);
  const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
  const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
  tnear = tn;
  return tn <= fmaf(tf, 1.00000095367431640625f, eps);
}

constexpr float kInf = __builtin_huge_valf();

// (ka, la) <= (kb, lb) after the call, ordered by key
__device__ __forceinline__ void sort2(float& ka, uint32_t& la, float& kb, uint32_t& lb) {
  const bool sw = kb < ka;
  const float k = sw ? kb : ka;
  const uint32_t l = sw ? lb : la;
  kb = sw ? ka : kb;
  lb = sw ? la : lb;
  ka = k;
  la = l;
}

struct HitState {
  float t, b1, b2;
  uint32_t prim, orig;
};

// Moller-Trumbore with inclusive edges of triangle k (BVH order) for a ray with current
// closest distance ht.  A division-free test with a relative margin of 1e-5 first rejects
// triangles that the exact test (barycentrics and t from the reciprocal of the determinant)
// would reject too, or that lie beyond ht; only the rest pay for the division, so results are
// those of the exact test alone.  Returns true with t, b1, b2 and the original index when the
// ray hits the triangle at t > tmin.
__device__ __forceinline__ bool test_tri_data(const DevScene& sc, float4 a0, float4 a1, float4 a2, V3 o, V3 d,
                                              float ht, float& t, float& b1, float& b2, uint32_t& og) {
  constexpr float kMargin = 1e-5f;
  const V3 e1 = xyz(a1), e2 = xyz(a2);
  const V3 p = cross(d, e2);
  const float det = dot(e1, p);
  const V3 s = o - xyz(a0);
  const V3 qv = cross(s, e1);
  // sign-normalized numerators: b1 = u / |det|, b2 = v / |det|, t = w / |det|
  const float ad = fabsf(det);
  const float u = copysignf(1.0f, det) * dot(s, p);
  const float v = copysignf(1.0f, det) * dot(d, qv);
  const float w = copysignf(1.0f, det) * dot(e2, qv);
  const float lim = ad * (1.0f + kMargin), neg = -kMargin * ad;
  if (ad == 0.0f || u < neg || u > lim || v < neg || u + v > lim || (w <= 0.0f && sc.tmin >= 0.0f) || w > lim * ht)
    return false;
  const float inv = 1.0f / det;
  b1 = dot(s, p) * inv;
  if (b1 < 0.0f || b1 > 1.0f) return false;
  b2 = dot(d, qv) * inv;
  if (b2 < 0.0f || b1 + b2 > 1.0f) return false;
  t = dot(e2, qv) * inv;
  og = bits(a0.w);
  return t > sc.tmin;
}

__device__ __forceinline__ bool test_tri(const DevScene& sc, uint32_t k, V3 o, V3 d, float ht, float& t, float& b1,
                                         float& b2, uint32_t& og) {
  return test_tri_data(sc, sc.tri[3 * k], sc.tri[3 * k + 1], sc.tri[3 * k + 2], o, d, ht, t, b1, b2, og);
}

// All triangles of a leaf for one ray: closest t wins, equal t goes to the smaller original
// triangle index.
// In an instance, uoff turns the triangle's index k into its primitive id k + uoff and its
// stored index (k itself) into the tie-break key; outside instances uoff is 0.
__device__ __forceinline__ void test_leaf(const DevScene& sc, uint32_t link, V3 o, V3 d, uint32_t excl,
                                          HitState& h, uint32_t& tris, uint32_t uoff = 0u) {
  const uint32_t first = (link >> 3) & 0x0fffffffu;
  const uint32_t count = (link & 7u) + 1u;
  tris += count;
  for (uint32_t k = first; k < first + count; ++k) {
    if (k + uoff == excl) continue;
    float t, b1, b2;
    uint32_t og;
    if (test_tri(sc, k, o, d, h.t, t, b1, b2, og) && (t < h.t || (t == h.t && og + uoff < h.orig))) {
      h.t = t;
      h.b1 = b1;
      h.b2 = b2;
      h.prim = k + uoff;
      h.orig = og + uoff;
    }
  }
}

// Closest-hit order as one 64-bit key: t (positive float bits, order-preserving) then the
// original triangle index.
__device__ __forceinline__ unsigned long long hit_key(float t, uint32_t orig) {
  return ((unsigned long long)__float_as_uint(t) << 32) | orig;
}

// The parked leaves of a wave, intersected triangle-parallel: the parked lane of rank r among
// the wave's parked lanes owns the group of lanes 4 (r mod 16) .. +3 in round r / 16, and lane
// 4 (r mod 16) + k tests triangle k of its leaf (leaves hold at most kLeafMaxTris = 4
// triangles).  The owners' lane numbers go through an LDS table indexed by rank; a lane reads
// its owner's leaf link, starts loading its triangle, and only then fetches the owner's ray
// through cross-lane shuffles, so the loads' latency overlaps the shuffles.  Each owner's
// closest hit is an LDS atomic minimum of hit keys; after each round the lane holding the
// current minimum publishes triangle and barycentrics.  Same result as test_leaf on every owner.
static_assert(kLeafMaxTris == 4, "the leaf phase deals four lanes to each parked leaf");
template <bool kCount, bool kInst>
__device__ __forceinline__ void leaf_phase_shared(const DevScene& sc, bool mine, uint32_t link, V3 o, V3 d,
                                                  uint32_t excl, HitState& h, uint32_t& tris,
                                                  unsigned long long* key, float4* slot, uint8_t* owner,
                                                  uint32_t uoff) {
  const uint32_t lane = __lane_id();
  const uint64_t parked = __ballot(mine);
  const uint32_t n_parked = (uint32_t)__popcll(parked);
  if constexpr (kCount) {
    const uint32_t cnt = mine ? (link & 7u) + 1u : 0u;
    uint32_t total = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) total += (uint32_t)__popcll(__ballot((cnt >> b) & 1u)) << b;
    tris += total;  // wave-uniform count of the (ray, triangle) pairs
  }
  const unsigned long long start = hit_key(h.t, h.orig);
  if (mine) {
    key[lane] = start;
    owner[lanes_below(parked)] = (uint8_t)lane;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (uint32_t r0 = 0; r0 < n_parked; r0 += 16) {
    const uint32_t q = r0 + (lane >> 2);
    const bool qv = q < n_parked;
    const int own = qv ? (int)owner[q] : 0;
    const uint32_t link_o = (uint32_t)__shfl((int)link, own);
    const uint32_t kk = lane & 3u;
    const bool pair = qv && kk <= (link_o & 7u);
    // the triangle: for a lane without a pair the owner's first one, or triangle 0 for a lane
    // past the last owner (in bounds either way, result unused)
    const uint32_t k = qv ? ((link_o >> 3) & 0x0fffffffu) + (pair ? kk : 0u) : 0u;
    const float4 a0 = sc.tri[3 * k], a1 = sc.tri[3 * k + 1], a2 = sc.tri[3 * k + 2];
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the shuffles below
    const uint32_t ex_o = (uint32_t)__shfl((int)excl, own);
    const V3 o_o = v3(__shfl(o.x, own), __shfl(o.y, own), __shfl(o.z, own));
    const V3 d_o = v3(__shfl(d.x, own), __shfl(d.y, own), __shfl(d.z, own));
    const float ht_o = __shfl(h.t, own);
    const uint32_t uo = kInst ? (uint32_t)__shfl((int)uoff, own) : 0u;
    float t = 0.0f, b1 = 0.0f, b2 = 0.0f;
    uint32_t og = 0;
    const bool hit = pair && k + uo != ex_o && test_tri_data(sc, a0, a1, a2, o_o, d_o, ht_o, t, b1, b2, og);
    const unsigned long long ck = hit ? hit_key(t, og + uo) : ~0ull;
    if (hit) atomicMin(&key[own], ck);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (hit && key[own] == ck) slot[own] = make_float4(__uint_as_float(k + uo), b1, b2, 0.0f);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  if (mine) {
    const unsigned long long best = key[lane];
    if (best != start) {
      const float4 sl = slot[lane];
      h.t = __uint_as_float((uint32_t)(best >> 32));
      h.orig = (uint32_t)best;
      h.prim = __float_as_uint(sl.x);
      h.b1 = sl.y;
      h.b2 = sl.z;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Traversal stack of one lane: the top kLdsStack entries in LDS ([depth][lane] layout: no bank
// conflicts), deeper entries in a global spill area (entry k at spill[k * gthreads]).
struct LaneStack {
  uint32_t (*lds)[kTraceThreads];
  uint32_t* spill;
  uint32_t gthreads;
  int tid, sp;
  __device__ void push(uint32_t v) {
    if (sp < kLdsStack) lds[sp][tid] = v;
    else if (sp < kStackMax) spill[(uint64_t)(sp - kLdsStack) * gthreads] = v;
    sp = min(sp + 1, kStackMax);
  }
  __device__ uint32_t pop() {
    --sp;
    // the LDS entry is read unconditionally (clamped index) and the spill area only past it,
    // so the common case is a plain LDS read rather than a generic-address load
    typedef __attribute__((address_space(1))) const uint32_t GlobalU32;
    uint32_t v = lds[sp < kLdsStack ? sp : kLdsStack - 1][tid];
    if (sp >= kLdsStack) v = ((GlobalU32*)spill)[(uint64_t)(sp - kLdsStack) * gthreads];
    return v;
  }
};

constexpr uint32_t kNoNode = 0xFFFFFFFFu;

// Persistent BVH2 traversal.  Each lane holds one ray; when a.ext_refill lanes of a wave are
// idle the wave takes a new batch of queue entries with one atomic on the counter of its
// current queue slice, so long rays do not hold a whole wave idle.
//   kMode 0: a lane intersects the triangles of a hit leaf child at once.
//   kMode 1: a lane that reaches a leaf parks it and waits; the wave intersects the parked
//     leaves together once a.ext_leaf_batch lanes hold one or no lane still looks for one, so
//     the triangle loop runs with most lanes busy (leaf links share the stack).
//   kMode 2: as 1, but a lane with a parked leaf keeps descending (further leaves go on the
//     stack) while others still look for theirs.
//   kMode 3: as 1, but the wave intersects the parked leaves triangle-parallel
//     (leaf_phase_shared): all 64 lanes share the (ray, triangle) pairs.
//   kMode 4: as 3 over the 4-wide tree: a visit tests four child boxes, pushes the hit
//     children farthest first and pops the nearest (a leaf is parked).  At most 3 entries
//     per level stay on the stack, so the tree must be at most kMaxBvh4Depth levels deep.
// kInst (modes 0, 1, 3): a two-level scene.  The walk starts in the tree over instances; a
// lane that reaches one of its leaves enters the leaf's first instance: it pushes the leaf's
// other instances and a kExitInst mark, moves its ray into the instance's object space (the
// direction is not renormalized, so distances t stay those of the world ray) and walks the
// instance's own tree from its root.  Popping the mark restores the world ray.  Parked leaves
// are tested with the lane's ray of the moment, which is the object-space ray of the leaf's
// instance: a lane does not step while it holds a parked leaf.
template <int kMode, bool kCount, bool kInst>
__device__ __forceinline__ void extend_body(const RenderArgs& a) {
  static_assert(!kInst || kMode == 0 || kMode == 1 || kMode == 3, "instances in modes 0, 1 and 3 only");
  __shared__ uint32_t stack_lds[kLdsStack][kTraceThreads];
  __shared__ unsigned long long cnt[3];  // rays traced, nodes visited, triangles tested
  __shared__ unsigned long long hit_keys[kMode >= 3 ? kTraceThreads : 1];
  __shared__ float4 hit_slots[kMode >= 3 ? kTraceThreads : 1];
  __shared__ uint8_t leaf_owner[kMode >= 3 ? kTraceThreads : 1];
  const int tid = threadIdx.x;
  if (tid < 3) cnt[tid] = 0;
  __syncthreads();
  const DevScene& sc = a.sc;
  const uint32_t n = a.ctl[a.depth].n;
  uint32_t* const work = a.work + (uint64_t)a.depth * kWorkSlices * kWorkStride;
  LaneStack st{stack_lds, a.spill + blockIdx.x * kTraceThreads + tid, gridDim.x * kTraceThreads, tid, 0};
  const int refill = (int)a.ext_refill;
  const int leaf_batch = (int)a.ext_leaf_batch;
  const uint32_t chunk = a.ext_chunk;
  bool active = false, exhausted = false;
  uint32_t ray = 0, excl = 0, ni = 0, pend = 0;
  // wave-uniform pool of claimed queue entries not yet handed to a lane (claim.hpp); claims
  // start in slice blockIdx % kWorkSlices and move on to the next slice once one is used up
  ClaimState cs = claim_start(n, blockIdx.x, kWorkSlices);
  V3 o = v3(0, 0, 0), d = o, inv = o, oi = o;
  float eps = 0.0f;
  // the world ray while the lane walks an instance (kInst), kept in LDS rather than registers
  __shared__ float world_lds[kInst ? 6 : 1][kInst ? kTraceThreads : 1];
  uint32_t uoff = 0u;  // primitive id offset of the instance being walked (kInst)
  HitState h;
  // reciprocal direction, -o/d and the slab test's absolute widening of the lane's ray
  auto prep_ray = [&]() {
    const V3 dd = v3(fabsf(d.x) > 1e-20f ? d.x : copysignf(1e-20f, d.x),
                     fabsf(d.y) > 1e-20f ? d.y : copysignf(1e-20f, d.y),
                     fabsf(d.z) > 1e-20f ? d.z : copysignf(1e-20f, d.z));
    inv = v3(1.0f / dd.x, 1.0f / dd.y, 1.0f / dd.z);
    oi = v3(-o.x * inv.x, -o.y * inv.y, -o.z * inv.z);
    // |oi| of axes the ray is not nearly parallel to (|d| >= 2^-10); see slab()
    eps = fmaxf(fmaxf(fabsf(o.x) * fminf(fabsf(inv.x), 1024.0f), fabsf(o.y) * fminf(fabsf(inv.y), 1024.0f)),
                fabsf(o.z) * fminf(fabsf(inv.z), 1024.0f)) *
          0x1p-22f;
  };
  // a leaf of the lane's current tree holding triangles (not instances)
  auto tri_leaf = [](uint32_t l) { return (l & kLeafBit) && (!kInst || !(l & kInstLeaf)); };
  // enter the first instance of the instance leaf ni (kInst)
  auto enter_instance = [&]() {
    const uint32_t first = (ni >> 3) & 0x0fffffffu, cnt = (ni & 3u) + 1u;
    if (cnt > 1u) st.push(kLeafBit | ((first + 1u) << 3) | kInstLeaf | (cnt - 2u));
    st.push(kExitInst);
    const float4* rec = sc.inst + 7ull * first;
    const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2], info = rec[6];
    if constexpr (kInst) {
      world_lds[0][tid] = o.x;
      world_lds[1][tid] = o.y;
      world_lds[2][tid] = o.z;
      world_lds[3][tid] = d.x;
      world_lds[4][tid] = d.y;
      world_lds[5][tid] = d.z;
    }
    const V3 oc = v3(o.x - r0.w, o.y - r1.w, o.z - r2.w);  // origin minus the translation, first
    const V3 wd = d;
    o = v3(fmaf(r0.x, oc.x, fmaf(r0.y, oc.y, r0.z * oc.z)), fmaf(r1.x, oc.x, fmaf(r1.y, oc.y, r1.z * oc.z)),
           fmaf(r2.x, oc.x, fmaf(r2.y, oc.y, r2.z * oc.z)));
    d = v3(fmaf(r0.x, wd.x, fmaf(r0.y, wd.y, r0.z * wd.z)), fmaf(r1.x, wd.x, fmaf(r1.y, wd.y, r1.z * wd.z)),
           fmaf(r2.x, wd.x, fmaf(r2.y, wd.y, r2.z * wd.z)));
    prep_ray();
    uoff = bits(info.y);
    ni = bits(info.x);
  };
  auto leave_instance = [&]() {
    if constexpr (kInst) {
      o = v3(world_lds[0][tid], world_lds[1][tid], world_lds[2][tid]);
      d = v3(world_lds[3][tid], world_lds[4][tid], world_lds[5][tid]);
    }
    prep_ray();
    uoff = 0u;
  };
  // statistics: rays and nodes counted per wave (wave-uniform, no per-lane registers);
  // triangles per wave in the shared leaf phase, per lane where a lane tests its own leaves
  uint32_t w_rays = 0, w_nodes = 0, w_tris = 0, c_tris = 0;
  for (;;) {
    if (!exhausted) {
      const uint64_t idle = __ballot(!active);
      if (idle != 0 && (__popcll(idle) >= refill || idle == __ballot(true))) {
        const uint32_t want = (uint32_t)__popcll(idle);
        const uint32_t rank = lanes_below(idle);  // this lane's rank among the idle lanes
        // claim what the idle lanes still need, or a whole chunk of entries, from the current
        // slice with one atomic; the returned range is clamped to the slice
        const bool claim = claim_needed(cs, want);
        uint32_t off = 0, take = 0;
        if (claim) {
          take = claim_amount(cs, want, chunk);
          const int leader = __ffsll((unsigned long long)idle) - 1;
          uint32_t b = 0;
          if ((int)__lane_id() == leader) b = atomicAdd(work + cs.slice * kWorkStride, take);
          off = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl(b, leader));
        }
        const uint32_t my = claim_hand_out(cs, n, kWorkSlices, want, rank, claim, off, take);
        exhausted = claim_exhausted(cs);
        if (!active && my < n) {
          // ray data loaded together (one round trip), dead entries only write a miss
          const float4 th = a.qin.thr[my], og = a.qin.orig[my], dr = a.qin.dir[my];
          if (bits(th.w) & kFlagDead) {
            a.hit[my] = make_float4(__builtin_inff(), 0.0f, 0.0f, __uint_as_float(kMiss));
          } else {
            o = xyz(og);
            d = xyz(dr);
            excl = bits(og.w);
            prep_ray();
            uoff = 0u;
            h.t = __builtin_inff();
            h.b1 = h.b2 = 0.0f;
            h.prim = kMiss;
            h.orig = kMiss;
            ni = kInst ? sc.root : 0u;
            pend = 0;
            st.sp = 0;
            ray = my;
            active = true;
          }
        }
        w_rays += (uint32_t)__popcll(__ballot(active) & idle);
      }
    }
    if (__ballot(active) == 0) {
      if (exhausted) break;
      continue;
    }
    if constexpr (kMode == 0) {
      if constexpr (kCount) w_nodes += (uint32_t)__popcll(__ballot(active));
      if (!active) continue;
      if constexpr (kInst) {
        if (ni & kLeafBit) {  // an instance leaf: one step to enter its first instance
          enter_instance();
          continue;
        }
      }
      // one node: test both child boxes, intersect leaf children, descend or pop
      const float4 n0 = sc.node[4 * ni], n1 = sc.node[4 * ni + 1], n2 = sc.node[4 * ni + 2], n3 = sc.node[4 * ni + 3];
      float tn0, tn1;
      bool h0 = slab(n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, inv, oi, eps, h.t, tn0);
      bool h1 = slab(n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, inv, oi, eps, h.t, tn1);
      const uint32_t l0 = bits(n3.x), l1 = bits(n3.y);
      if (h0 && tri_leaf(l0)) {
        test_leaf(sc, l0, o, d, excl, h, c_tris, uoff);
        h0 = false;
      }
      if (h1 && tri_leaf(l1)) {
        test_leaf(sc, l1, o, d, excl, h, c_tris, uoff);
        h1 = false;
      }
      if (h0 && h1) {
        const bool first0 = tn0 <= tn1;
        st.push(first0 ? l1 : l0);
        ni = first0 ? l0 : l1;
      } else if (h0) {
        ni = l0;
      } else if (h1) {
        ni = l1;
      } else {
        for (;;) {
          if (st.sp == 0) {
            a.hit[ray] = make_float4(h.t, h.b1, h.b2, __uint_as_float(h.prim));
            active = false;
            break;
          }
          const uint32_t e = st.pop();
          if (kInst && e == kExitInst) {
            leave_instance();
            continue;
          }
          ni = e;
          break;
        }
      }
    } else {
      // Node phase: lanes without a parked leaf take one step each per round (visit a node, or
      // pop the stack) until enough leaves are parked, no lane is still looking for one, or
      // enough lanes have finished to make a refill worthwhile.
      uint64_t parked, seeking;
      // one step of every lane without a parked leaf: visit a node, or pop the stack
      auto node_step = [&]() {
        if constexpr (kCount)
          w_nodes += (uint32_t)__popcll(__ballot(active && ni != kNoNode && (kMode == 2 || pend == 0)));
        if (active) {
          if constexpr (kMode == 4) {
            if (ni != kNoNode && pend == 0) {
              const float4* nd = sc.node4 + 8ull * ni;
              const float4 lx = nd[0], hx = nd[1], ly = nd[2], hy = nd[3], lz = nd[4], hz = nd[5], lk = nd[6];
              float k0, k1, k2, k3;
              uint32_t c0 = bits(lk.x), c1 = bits(lk.y), c2 = bits(lk.z), c3 = bits(lk.w);
              if (!(c0 != kEmptyChild4 && slab(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, inv, oi, eps, h.t, k0))) k0 = kInf;
              if (!(c1 != kEmptyChild4 && slab(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, inv, oi, eps, h.t, k1))) k1 = kInf;
              if (!(c2 != kEmptyChild4 && slab(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, inv, oi, eps, h.t, k2))) k2 = kInf;
              if (!(c3 != kEmptyChild4 && slab(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, inv, oi, eps, h.t, k3))) k3 = kInf;
              // ascending by entry distance (misses last): five compare-exchanges
              sort2(k0, c0, k1, c1);
              sort2(k2, c2, k3, c3);
              sort2(k0, c0, k2, c2);
              sort2(k1, c1, k3, c3);
              sort2(k1, c1, k2, c2);
              if (k3 != kInf) st.push(c3);
              if (k2 != kInf) st.push(c2);
              if (k1 != kInf) st.push(c1);
              if (k0 != kInf) st.push(c0);
              ni = kNoNode;
            }
          } else if (kInst && ni != kNoNode && pend == 0 && (ni & kLeafBit)) {
            enter_instance();
          } else if (ni != kNoNode && (kMode == 2 || pend == 0)) {
            const float4 n0 = sc.node[4 * ni], n1 = sc.node[4 * ni + 1], n2 = sc.node[4 * ni + 2],
                         n3 = sc.node[4 * ni + 3];
            float tn0, tn1;
            const bool h0 = slab(n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, inv, oi, eps, h.t, tn0);
            const bool h1 = slab(n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, inv, oi, eps, h.t, tn1);
            const uint32_t l0 = bits(n3.x), l1 = bits(n3.y);
            const bool first0 = tn0 <= tn1;
            const bool f0 = h0 && tri_leaf(l0), f1 = h1 && tri_leaf(l1);
            const bool i0 = h0 && !tri_leaf(l0), i1 = h1 && !tri_leaf(l1);
            // leaves: the nearer one is parked if the lane has none, the others wait on the
            // stack; a nearly full stack (possible only in mode 2) intersects them at once
            if (f0 || f1) {
              const uint32_t lnear = (f0 && (first0 || !f1)) ? l0 : l1;
              const uint32_t lfar = (f0 && f1) ? (first0 ? l1 : l0) : 0u;
              if (kMode == 2 && st.sp > kLeafPushLimit) {
                if (lfar) test_leaf(sc, lfar, o, d, excl, h, c_tris, uoff);
                test_leaf(sc, lnear, o, d, excl, h, c_tris, uoff);
              } else {
                if (lfar) st.push(lfar);
                if (pend == 0) pend = lnear;
                else st.push(lnear);
              }
            }
            if (i0 && i1) {
              ni = first0 ? l0 : l1;
              st.push(first0 ? l1 : l0);
            } else {
              ni = i0 ? l0 : (i1 ? l1 : kNoNode);
            }
          }
          if (ni == kNoNode && pend == 0) {
            if (st.sp > 0) {
              const uint32_t e = st.pop();
              if (kInst && e == kExitInst) leave_instance();
              else if (tri_leaf(e)) pend = e;
              else ni = e;
            } else {
              a.hit[ray] = make_float4(h.t, h.b1, h.b2, __uint_as_float(h.prim));
              active = false;
            }
          }
        }
      };
      // two steps per check of the wave-wide exit conditions: a lane that parks a leaf or
      // finishes in the first step only idles through the second, and the ballots, counts and
      // branches of the check are paid once per two node visits
      for (;;) {
        node_step();
        node_step();
        parked = __ballot(active && pend != 0);
        seeking = __ballot(active && pend == 0);
        if (seeking == 0 || __popcll(parked) >= leaf_batch) break;
        if (!exhausted && __popcll(~(parked | seeking)) >= refill) break;
      }
      if (parked != 0 && (seeking == 0 || __popcll(parked) >= leaf_batch)) {
        if constexpr (kMode >= 3) {
          const int wbase = tid & ~63;
          leaf_phase_shared<kCount, kInst>(sc, active && pend != 0, pend, o, d, excl, h, w_tris,
                                           hit_keys + wbase, hit_slots + wbase, leaf_owner + wbase, uoff);
          if (active) pend = 0;
        } else if (active && pend != 0) {
          test_leaf(sc, pend, o, d, excl, h, c_tris, uoff);
          pend = 0;
        }
      }
    }
  }
  if (__lane_id() == 0) {
    atomicAdd(&cnt[0], (unsigned long long)w_rays);
    atomicAdd(&cnt[1], (unsigned long long)w_nodes);
  }
  if (kMode >= 3) {
    if (__lane_id() == 0) atomicAdd(&cnt[2], (unsigned long long)w_tris);
  } else {
    atomicAdd(&cnt[2], (unsigned long long)c_tris);
  }
  __syncthreads();
  if (tid < 3 && cnt[tid]) atomicAdd(a.rays + tid, cnt[tid]);
}

// Variants that park leaves fit 72 VGPRs without spilling: 7 waves per SIMD.  kCount: BVH
// nodes visited and triangles tested are counted too (per-stage timing runs only).
template <int kMode, bool kCount>
__global__ __launch_bounds__(kTraceThreads) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_extend(RenderArgs a) {
  extend_body<kMode, kCount, false>(a);
}
template <bool kCount>
__global__ __launch_bounds__(kTraceThreads) void k_extend_immediate(RenderArgs a) { extend_body<0, kCount, false>(a); }
// Two-level scenes: the saved world ray sits in LDS, the instance state in registers (89-94,
// 5 waves per SIMD, no spills; with the world ray in registers the kernel needed 105).
template <int kMode, bool kCount>
__global__ __launch_bounds__(kTraceThreads) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_extend_inst(RenderArgs a) {
  extend_body<kMode, kCount, true>(a);
}

// ------------------------------------------------------------------------------- shade
constexpr uint32_t kNoPix = 0xFFFFFFFFu;

// FP64 image accumulation of one wave's emissions: lanes with the same pixel in consecutive
// lanes (queue entries of one pixel are adjacent: primary paths are pixel-major and
// compaction keeps parent order) are summed by a segmented scan, and the last lane of each
// run adds the run's total with one atomic per channel.  Lanes without a pixel pass kNoPix.
// Every lane of the wave must call it.
__device__ __forceinline__ void image_add_wave(const RenderArgs& a, uint32_t pix, double cx, double cy, double cz) {
  const int lane = (int)__lane_id();
  const uint32_t prev = (uint32_t)__shfl_up((int)pix, 1);
  const uint64_t heads = __ballot(lane == 0 || prev != pix);
  const int start = 63 - __clzll(heads & ((2ull << lane) - 1ull));  // first lane of this run
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double tx = __shfl_up(cx, off), ty = __shfl_up(cy, off), tz = __shfl_up(cz, off);
    if (lane - off >= start) {
      cx += tx;
      cy += ty;
      cz += tz;
    }
  }
  const uint32_t next = (uint32_t)__shfl_down((int)pix, 1);
  if ((lane == 63 || next != pix) && pix != kNoPix && (cx != 0.0 || cy != 0.0 || cz != 0.0)) {
    double* px = a.image + 3ull * pix;
    atomicAdd(px + 0, cx);
    atomicAdd(px + 1, cy);
    atomicAdd(px + 2, cz);
  }
}

// Emission credited to the training records of the path's recorded vertices.
__device__ __forceinline__ void record_emission(const RenderArgs& a, V3 c, int4 rec) {
  const float l = lum(c);
  if (rec.x >= 0) atomicAdd(a.rec.acc + rec.x, l);
  if (rec.y >= 0) atomicAdd(a.rec.acc + rec.y, l);
  if (rec.z >= 0) atomicAdd(a.rec.acc + rec.z, l);
  if (rec.w >= 0) atomicAdd(a.rec.acc + rec.w, l);
}

// Record slots for a whole block with one counter atomic: per-wave counts in LDS, a block
// prefix by the first thread.  Every thread of the block must call it.
__device__ __forceinline__ uint32_t block_alloc(uint32_t* counter, bool pred, uint32_t* sh) {
  constexpr int kWaves = kShadeThreads / 64;
  const uint64_t m = __ballot(pred);
  const int wave = threadIdx.x >> 6;
  if (__lane_id() == 0) sh[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = sh[w];
      sh[w] = tot;
      tot += c;
    }
    sh[kWaves] = tot ? atomicAdd(counter, tot) : 0u;
  }
  __syncthreads();
  return sh[kWaves] + sh[wave] + lanes_below(m);
}

// The world-space triangle of primitive id `prim` (v0, e1, e2 in a0..a2, material in a1.w): the
// stored one, or for a triangle of an instance (two-level scenes, prim >= nt_base) its object-
// space copy moved by the instance's transform (the instance's material, unless it keeps the
// triangle's own).  Barycentrics are those of the object-space hit.
__device__ __forceinline__ void world_tri(const DevScene& sc, uint32_t prim, float4& a0, float4& a1, float4& a2) {
  if (sc.n_inst == 0u || prim < sc.nt_base) {
    a0 = sc.tri[3 * prim];
    a1 = sc.tri[3 * prim + 1];
    a2 = sc.tri[3 * prim + 2];
    return;
  }
  uint32_t lo = 0, hi = sc.n_inst - 1u;  // the last instance whose first uid is <= prim
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1u) >> 1;
    if (sc.inst_uid[2 * mid] <= prim) lo = mid;
    else hi = mid - 1u;
  }
  const float4* rec = sc.inst + 7ull * sc.inst_uid[2 * lo + 1];
  const float4 f0 = rec[3], f1 = rec[4], f2 = rec[5], info = rec[6];
  const uint32_t k = prim - bits(info.y);
  const float4 b0 = sc.tri[3 * k], b1 = sc.tri[3 * k + 1], b2 = sc.tri[3 * k + 2];
  const uint32_t mat = bits(info.z) != kNoMat ? bits(info.z) : bits(b1.w);
  a0 = make_float4(fmaf(f0.x, b0.x, fmaf(f0.y, b0.y, fmaf(f0.z, b0.z, f0.w))),
                   fmaf(f1.x, b0.x, fmaf(f1.y, b0.y, fmaf(f1.z, b0.z, f1.w))),
                   fmaf(f2.x, b0.x, fmaf(f2.y, b0.y, fmaf(f2.z, b0.z, f2.w))), b0.w);
  a1 = make_float4(fmaf(f0.x, b1.x, fmaf(f0.y, b1.y, f0.z * b1.z)), fmaf(f1.x, b1.x, fmaf(f1.y, b1.y, f1.z * b1.z)),
                   fmaf(f2.x, b1.x, fmaf(f2.y, b1.y, f2.z * b1.z)), __uint_as_float(mat));
  a2 = make_float4(fmaf(f0.x, b2.x, fmaf(f0.y, b2.y, f0.z * b2.z)), fmaf(f1.x, b2.x, fmaf(f1.y, b2.y, f1.z * b2.z)),
                   fmaf(f2.x, b2.x, fmaf(f2.y, b2.y, f2.z * b2.z)), 0.0f);
}

// Next-event estimation at a vertex that may continue: one light (probability lum(L_e) x area
// through the CDF), a point uniform on it, the BSDF's f cos toward it and the power-heuristic
// weight against the BSDF's own sampling of that direction.  The shadow ray goes to the
// out-queue slot i (origin offset along the face-forwarded normal, excluded triangle in the
// origin's w; direction and pixel; contribution t f cos L_e w / pdf_light and flags; the light
// distance shortened by 1e-4 as float bits in id.x), to be traced by the traversal kernel.
__device__ __forceinline__ void nee_shadow_ray(const RenderArgs& a, uint32_t i, V3 p, V3 nrm, V3 wo, V3 t, float4 m0,
                                               uint32_t type, uint32_t pix, uint32_t prim) {
  const uint32_t dead = kFlagDead;
  if (a.sc.nl == 0u) {
    a.qout.thr[i] = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float(dead));
    return;
  }
  const uint4 r = draw(a.key, a.qin.id[i], kPurposeNee, a.depth, 0);
  const float u0 = unit(r.x), u1 = unit(r.y), u2 = unit(r.z);
  uint32_t lo = 0, hi = a.sc.nl - 1u;  // smallest k with cdf[k + 1] > u0
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a.sc.light_cdf[mid + 1] > u0) hi = mid;
    else lo = mid + 1;
  }
  const float4 l0 = a.sc.light_geo[3 * lo], l1 = a.sc.light_geo[3 * lo + 1], l2 = a.sc.light_geo[3 * lo + 2];
  const V3 e1 = xyz(l1), e2 = xyz(l2);
  const V3 ngl = normalized(cross(e1, e2));
  const float su = sqrtf(u1);
  const float b1 = su * (1.0f - u2), b2 = su * u2;
  const V3 y = xyz(l0) + b1 * e1 + b2 * e2;
  const float eps = a.sc.offset;
  const V3 o = v3(fmaf(eps, nrm.x, p.x), fmaf(eps, nrm.y, p.y), fmaf(eps, nrm.z, p.z));
  V3 d = y - o;
  const float dist = sqrtf(dot(d, d));
  const float cos_x = dot(nrm, d) / dist, cos_l = -dot(ngl, d) / dist;
  if (!(dist > 0.0f) || cos_x <= 0.0f || cos_l <= 0.0f) {
    a.qout.thr[i] = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float(dead));
    return;
  }
  d = (1.0f / dist) * d;
  V3 fc;
  float pb;
  V3 tb, bb;
  basis(nrm, tb, bb);
  const V3 wol = v3(dot(wo, tb), dot(wo, bb), dot(wo, nrm));
  const V3 wil = v3(dot(d, tb), dot(d, bb), cos_x);
  if (type == 1u) {
    fc = ggx_eval_cos(m0.w, xyz(m0), wol, wil);
    pb = ggx_pdf(m0.w, wol, wil);
  } else {
    fc = (cos_x * 0.31830988618379067f) * xyz(m0);
    pb = cos_x * 0.31830988618379067f;
  }
  const float4 lm = a.sc.mat[2 * bits(l1.w) + 1];
  const float pl = lum(xyz(lm)) * a.sc.light_scale * dist * dist / cos_l;
  const float w = pl * pl / (pl * pl + pb * pb);
  const float k = w / pl;
  const V3 c = v3(t.x * fc.x * lm.x * k, t.y * fc.y * lm.y * k, t.z * fc.z * lm.z * k);
  a.qout.orig[i] = make_float4(o.x, o.y, o.z, __uint_as_float(prim));
  a.qout.dir[i] = pack(d, pix);
  a.qout.thr[i] = pack(c, 0u);
  a.qout.id[i] = make_uint2(__float_as_uint(dist * (1.0f - 1e-4f)), 0u);
}

// The unoccluded light samples of the depth: the shadow ray's closest hit (written over the
// out-queue's record slots) lies beyond the shortened light distance.  Their contributions go
// to the image, to the vertex's ancestors' records (the vertex's own record does not see its
// own light sample) and to the per-path radiance.
__global__ __launch_bounds__(kShadeThreads) void k_nee_resolve(RenderArgs a) {
  const uint32_t n = a.ctl[a.depth].n;
  const uint32_t i0 = blockIdx.x * kShadeThreads + threadIdx.x;
  if (blockIdx.x * kShadeThreads >= n) return;  // uniform over the block
  const bool in_range = i0 < n;
  const uint32_t i = in_range ? i0 : n - 1;
  const float4 th = a.qout.thr[i];
  bool lit = false;
  uint32_t pix = kNoPix;
  if (in_range && !(bits(th.w) & kFlagDead)) {
    const float4 hh = reinterpret_cast<const float4*>(a.qout.rec)[i];
    const float tmax = __uint_as_float(a.qout.id[i].x);
    lit = bits(hh.w) == kMiss || hh.x >= tmax;
    if (lit) pix = bits(a.qout.dir[i].w);
  }
  const V3 c = lit ? xyz(th) : v3(0.0f, 0.0f, 0.0f);
  image_add_wave(a, pix, (double)c.x, (double)c.y, (double)c.z);
  if (lit && a.records_on && (bits(a.qin.thr[i].w) & kFlagTrain)) {
    int4 rec = a.qin.rec[i];
    if (a.depth == 1u) rec.x = -1;
    else if (a.depth == 2u) rec.y = -1;
    else if (a.depth == 3u) rec.z = -1;
    else if (a.depth == 4u) rec.w = -1;
    record_emission(a, c, rec);
  }
  if (lit && a.trace) {
    double* tp = a.trace + 3ull * ((uint64_t)a.qin.path[i] * a.trace_depth + (a.depth - 1));
    atomicAdd(tp + 0, (double)c.x);
    atomicAdd(tp + 1, (double)c.y);
    atomicAdd(tp + 2, (double)c.z);
  }
}

constexpr uint32_t kShadeStripes = 64;

// kNee: next-event estimation on (a.nee); kInst: a two-level scene (a.sc.n_inst > 0).  The
// variants keep the code of the options a context does not use out of the kernel.
template <bool kNee, bool kInst>
__global__ __launch_bounds__(kShadeThreads) void k_shade(RenderArgs a) {
  __shared__ uint32_t alloc_sh[kShadeThreads / 64 + 1];
  const uint32_t n = a.ctl[a.depth].n;
  const uint32_t tiles = (n + kShadeThreads - 1) / kShadeThreads;
  if (blockIdx.x >= tiles) return;  // uniform over the block
  // Blocks take the queue's tiles interleaved over kShadeStripes stripes, so that the blocks
  // that run first (and take the first record slots) cover the whole image: with a pixel's
  // paths adjacent in the queue, tiles in plain order would give the record buffer the top
  // rows of the image first whenever it fills up.
  const uint32_t per = tiles / kShadeStripes;
  const uint32_t b = blockIdx.x;
  const uint32_t tile = b < per * kShadeStripes ? (b % kShadeStripes) * per + b / kShadeStripes : b;
  const uint32_t i0 = tile * kShadeThreads + threadIdx.x;
  const bool in_range = i0 < n;
  const uint32_t i = in_range ? i0 : n - 1;
  // the entry's queue data in one round trip (dead entries are rare)
  const float4 th = a.qin.thr[i], dr = a.qin.dir[i], hh = a.hit[i];
  const uint32_t flags = bits(th.w);
  int4 rec = a.records_on && (flags & kFlagTrain) ? a.qin.rec[i] : make_int4(-1, -1, -1, -1);
  float q = 0.0f;
  bool want_rec = false;
  V3 t = xyz(th), p = v3(0, 0, 0), nrm = p, wo = p, em = p;
  float4 m0 = make_float4(0, 0, 0, 0);
  uint32_t type = 0, pix = 0;
  bool emits = false, nee_written = false;
  if (in_range && !(flags & kFlagDead)) {
    pix = bits(dr.w);
    const uint32_t prim = bits(hh.w);
    if (prim == kMiss) {
      em = mul(t, v3(a.sc.env_r, a.sc.env_g, a.sc.env_b));
      emits = true;
    } else {
      float4 a0, a1, a2;
      if constexpr (kInst) {
        world_tri(a.sc, prim, a0, a1, a2);
      } else {
        a0 = a.sc.tri[3 * prim];
        a1 = a.sc.tri[3 * prim + 1];
        a2 = a.sc.tri[3 * prim + 2];
      }
      const V3 e1 = xyz(a1), e2 = xyz(a2);
      const uint32_t mid = bits(a1.w);
      const V3 ng = normalized(cross(e1, e2));
      p = xyz(a0) + hh.y * e1 + hh.z * e2;
      wo = v3(-dr.x, -dr.y, -dr.z);
      const bool front = dot(ng, wo) > 0.0f;
      nrm = front ? ng : v3(-ng.x, -ng.y, -ng.z);
      m0 = a.sc.mat[2 * mid];
      const float4 m1 = a.sc.mat[2 * mid + 1];
      type = bits(m1.w);
      if (front && (m1.x != 0.0f || m1.y != 0.0f || m1.z != 0.0f)) {
        em = mul(t, xyz(m1));
        emits = true;
        if (kNee && a.depth > 1u) {
          // a BSDF-sampled hit on a light: power-heuristic weight against light sampling
          const float pb = a.qin.pdf[i];
          if (pb > 0.0f) {
            const float pl = lum(xyz(m1)) * a.sc.light_scale * hh.x * hh.x / dot(ng, wo);
            em = (pb * pb / (pb * pb + pl * pl)) * em;
          }
        }
      }
      if (a.depth < a.max_depth && type != 2u) {
        q = a.mode == 0u ? 1.0f : lum(mul(t, xyz(m0)));
        want_rec = a.records_on && (flags & kFlagTrain) && a.depth <= a.net_max_depth && a.depth <= (uint32_t)kMaxRec;
        if constexpr (kNee) {
          nee_shadow_ray(a, i, p, nrm, wo, t, m0, type, pix, prim);
          nee_written = true;
        }
      }
      a.vpos[i] = pack(p, prim);
      a.vnrm[i] = pack(nrm, mid);
    }
  }
  // slots without a light sample carry a dead shadow ray (the traversal skips them)
  if (kNee && in_range && !nee_written) a.qout.thr[i] = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float(kFlagDead));
  if (in_range) a.q[i] = q;
  image_add_wave(a, in_range && !(flags & kFlagDead) ? pix : kNoPix, (double)em.x, (double)em.y, (double)em.z);
  if (emits && a.records_on) record_emission(a, em, rec);
  if (emits && a.trace) {
    double* tp = a.trace + 3ull * ((uint64_t)a.qin.path[i] * a.trace_depth + (a.depth - 1));
    atomicAdd(tp + 0, (double)em.x);
    atomicAdd(tp + 1, (double)em.y);
    atomicAdd(tp + 2, (double)em.z);
  }
  // training record: one counter atomic per block (converged code)
  if (a.records_on) {
    const uint32_t slot = block_alloc(a.rec.count, want_rec, alloc_sh);
    if (want_rec && slot < a.rec.cap) {
      // the 20 features are filled by k_record_features over the dense record slots
      a.rec.qidx[slot] = i;
      a.rec.lum_t[slot] = lum(t);
      a.rec.acc[slot] = 0.0f;
      a.rec.depth[slot] = a.depth;
      a.rec.pix[slot] = pix;
      a.rec.lineage[slot] = a.qin.id[i];
      if (a.depth == 1) rec.x = (int)slot;
      else if (a.depth == 2) rec.y = (int)slot;
      else if (a.depth == 3) rec.z = (int)slot;
      else rec.w = (int)slot;
      a.qin.rec[i] = rec;
    }
  }
}

// Features of the records captured at this depth, one thread per record slot (the shading
// kernel only reserved the slots and noted the queue entries).
__global__ __launch_bounds__(kEntryThreads) void k_record_features(RenderArgs a) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t cnt = min(*a.rec.count, a.rec.cap);
  if (s >= cnt || a.rec.depth[s] != a.depth) return;
  const uint32_t i = a.rec.qidx[s];
  const float4 vp = a.vpos[i], vn = a.vnrm[i], dr = a.qin.dir[i], th = a.qin.thr[i];
  const uint32_t mid = bits(vn.w);
  const float4 m0 = a.sc.mat[2 * mid], m1 = a.sc.mat[2 * mid + 1];
  float f[20];
  vertex_features(a.sc, xyz(vp), xyz(vn), v3(-dr.x, -dr.y, -dr.z), xyz(th), m0, bits(m1.w), a.depth, a.max_depth, f);
  float* dst = a.rec.feat + 20ull * s;
#pragma unroll
  for (int k = 0; k < 20; ++k) dst[k] = f[k];
  if (a.rec.nraw) {
    // StatNet / RRSNet inputs of the vertex (NRRS training): position in the scene box, w_o,
    // remapped roughness and the pixel value the factor was computed with
    const float inv = 1.0f / a.sc.extent;
    float* nr = a.rec.nraw + 8ull * s;
    nr[0] = (vp.x - a.sc.amin_x) * inv;
    nr[1] = (vp.y - a.sc.amin_y) * inv;
    nr[2] = (vp.z - a.sc.amin_z) * inv;
    nr[3] = -dr.x;
    nr[4] = -dr.y;
    nr[5] = -dr.z;
    nr[6] = 1.0f - expf(-(bits(m1.w) == 1u ? m0.w : 1.0f));
    nr[7] = a.guide[bits(dr.w)];
    a.rec.ntq[s] = make_float4(th.x, th.y, th.z, 0.0f);
  }
}

// -------------------------------------------------------------------- FP64 sum of q
// Chunked: block b owns entries [b*chunk, (b+1)*chunk); a fixed grid and fixed reduction
// tree make the FP64 sum the same on every run.
__device__ __forceinline__ uint32_t chunk_of(uint32_t n) {
  uint32_t c = (n + kScanBlocks - 1) / kScanBlocks;
  return (c + kScanThreads - 1) / kScanThreads * kScanThreads;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = kScanThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  T r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanThreads) void k_sum_q_partial(RenderArgs a) {
  __shared__ double sh[kScanThreads];
  const uint32_t n = a.ctl[a.depth].n;
  const uint32_t chunk = chunk_of(n);
  const uint32_t beg = blockIdx.x * chunk;
  double acc = 0.0;
  for (uint32_t base = beg; base < beg + chunk && base < n; base += kScanThreads) {
    const uint32_t i = base + threadIdx.x;
    if (i < n && i < beg + chunk) acc += (double)a.q[i];
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
}

// The partial sums added in a fixed tree by one block.  (A single launch in which the last
// block to finish adds the partials needs every block to publish its partial with a
// device-wide release, which on the eight-XCD MI355X writes back each XCD's L2: measured four
// times slower than this second launch.)
__global__ __launch_bounds__(kScanThreads) void k_sum_q_final(RenderArgs a) {
  __shared__ double sh[kScanThreads];
  double acc = 0.0;
  for (int b = threadIdx.x; b < kScanBlocks; b += kScanThreads) acc += a.partial[b];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) a.ctl[a.depth].sumq = s;
}

// ------------------------------------------------------------ roulette and scan
// Normalization factor for a given alpha (Eqs. 10, 12-14; Sec. 5 downscale variant).
__device__ __forceinline__ double norm_factor(const RenderArgs& a, double sumq, double alpha) {
  if (a.mode == 0u) return 1.0;
  if (a.F_fixed) return a.F_fixed[a.depth];
  if (!(sumq > 0.0)) return 0.0;
  double F = (a.f_rate * alpha) * a.budget_base / sumq;
  if (a.norm_mode == 1u && F > 1.0) F = 1.0;
  return F;
}

// Eq. (8): X = floor(q_norm) + [u < q_norm - floor(q_norm)] with q_norm rounded to float.
__device__ __forceinline__ uint32_t child_count(float q, double F, float u) {
  const float qn = (float)(F * (double)q);
  const float k = floorf(qn);
  return (uint32_t)k + (u < qn - k ? 1u : 0u);
}

__device__ __forceinline__ float roulette_u(const RenderArgs& a, uint32_t i) {
  return unit(draw(a.key, a.qin.id[i], kPurposeRoulette, a.depth, 0).x);
}

// Exclusive scan of kScanBlocks values by one block of kScanThreads threads (4 per thread).
__device__ __forceinline__ uint64_t scan_blocks(const uint32_t* in, uint32_t* out, uint64_t* sh) {
  const int tid = threadIdx.x;
  constexpr int per = kScanBlocks / kScanThreads;
  uint64_t local[per];
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    local[k] = in[tid * per + k];
    s += local[k];
  }
  sh[tid] = s;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    uint64_t v = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += v;
    __syncthreads();
  }
  const uint64_t total = sh[kScanThreads - 1];
  uint64_t run = sh[tid] - s;
  if (out) {
#pragma unroll
    for (int k = 0; k < per; ++k) {
      out[tid * per + k] = (uint32_t)run;
      run += local[k];
    }
  }
  __syncthreads();
  return total;
}

// Offsets of the blocks' children, the total S, and whether the overflow guard runs.
__global__ __launch_bounds__(kScanThreads) void k_roulette_scan(RenderArgs a) {
  __shared__ uint64_t sh[kScanThreads];
  const uint64_t S = scan_blocks(a.bsum, a.boff, sh);
  if (threadIdx.x == 0) {
    DepthCtl& c = a.ctl[a.depth];
    c.retries = 0;
    c.F = norm_factor(a, c.sumq, *a.alpha);
    if (S > a.cap) {
      c.guard = 1;
    } else {
      c.guard = 0;
      c.S = (uint32_t)S;
      a.ctl[a.depth + 1].n = (uint32_t)S;
    }
  }
}

__global__ __launch_bounds__(kScanThreads) void k_roulette_count(RenderArgs a) {
  __shared__ uint32_t sh[kScanThreads];
  const uint32_t n = a.ctl[a.depth].n;
  const uint32_t chunk = chunk_of(n);
  const uint32_t beg = blockIdx.x * chunk;
  const double F = norm_factor(a, a.ctl[a.depth].sumq, *a.alpha);
  uint32_t acc = 0;
#pragma unroll 4
  for (uint32_t base = beg; base < beg + chunk && base < n; base += kScanThreads) {
    const uint32_t i = base + threadIdx.x;
    if (i < n && i < beg + chunk) {
      const float q = a.q[i];
      const uint32_t x = q > 0.0f ? child_count(q, F, roulette_u(a, i)) : 0u;
      a.offs[i] = x;  // kept for k_offsets unless the overflow guard changes the factor
      acc += x;
    }
  }
  const uint32_t s = block_sum(acc, sh);
  if (threadIdx.x == 0) a.bsum[blockIdx.x] = s;
}

// alpha after k reductions by the factor 0.99 (Eq. 14), applied one at a time as in a loop
// that retries the roulette.
__device__ __forceinline__ double alpha_after(double alpha, int k) {
  for (int j = 0; j < k; ++j) alpha *= 0.99;
  return alpha;
}

// Children emitted for the k-th alpha reduction, counted by one block over all n entries.
__device__ __forceinline__ uint64_t block_count_all(const RenderArgs& a, uint32_t n, double F, uint64_t* sh) {
  uint64_t acc = 0;
  for (uint32_t i = threadIdx.x; i < n; i += kScanThreads) {
    const float q = a.q[i];
    if (q > 0.0f) acc += child_count(q, F, roulette_u(a, i));
  }
  return block_sum(acc, sh);
}

// Picks the first alpha reduction whose children fit the capacity, as a loop that retries
// the roulette with alpha * 0.99 until S <= C would, and gives up (overflow) once alpha falls
// below 1e-3.  The counts of reductions 1..kGuardSteps come from k_guard_count; when none of
// them fits, this block searches the later reductions itself by bisection (the children count
// does not grow as alpha shrinks: every rounding on the way from alpha to X is monotone).
__global__ __launch_bounds__(kScanThreads) void k_guard_select(RenderArgs a) {
  if (a.ctl[a.depth].guard == 0) return;
  __shared__ uint64_t sh[kScanThreads];
  __shared__ int chosen;   // reduction count that fits, or -(count at which alpha < 1e-3)
  __shared__ uint64_t chosen_S;
  DepthCtl& c = a.ctl[a.depth];
  const uint32_t n = c.n;
  const double alpha0 = *a.alpha;
  if (threadIdx.x == 0) chosen = 0;
  __syncthreads();
  for (int k = 1; k <= kGuardSteps; ++k) {
    const uint64_t S = scan_blocks(a.gsum + kScanBlocks * (k - 1), nullptr, sh);
    if (alpha_after(alpha0, k) < kAlphaMin) {
      if (threadIdx.x == 0) chosen = -k;
      break;
    }
    if (S <= a.cap) {
      scan_blocks(a.gsum + kScanBlocks * (k - 1), a.boff, sh);
      if (threadIdx.x == 0) {
        chosen = k;
        chosen_S = S;
      }
      break;
    }
  }
  __syncthreads();
  const int first = chosen;
  __syncthreads();  // every wave holds the first loop's result before thread 0 may change it
  bool need_block_sums = false;
  if (first == 0) {
    // rare path: bisection over the reductions kGuardSteps+1 .. K, K the last with alpha >= 1e-3
    int K = kGuardSteps;
    double aK = alpha_after(alpha0, K);
    while (aK * 0.99 >= kAlphaMin) {
      aK *= 0.99;
      ++K;
    }
    int lo = kGuardSteps + 1, hi = K;
    uint64_t S_hi = ~0ull;
    if (hi >= lo) S_hi = block_count_all(a, n, norm_factor(a, c.sumq, aK), sh);
    if (hi < lo || S_hi > a.cap) {
      if (threadIdx.x == 0) chosen = -(K + 1);
    } else {
      while (lo < hi) {  // invariant: S(hi) <= cap; every k < lo has S(k) > cap
        const int mid = (lo + hi) / 2;
        const uint64_t Sm = block_count_all(a, n, norm_factor(a, c.sumq, alpha_after(alpha0, mid)), sh);
        if (Sm <= a.cap) {
          hi = mid;
          S_hi = Sm;
        } else {
          lo = mid + 1;
        }
      }
      if (threadIdx.x == 0) {
        chosen = hi;
        chosen_S = S_hi;
      }
      need_block_sums = true;
    }
    __syncthreads();
  }
  const int k = chosen;
  if (need_block_sums) {
    // children per chunk of k_offsets for the chosen reduction, then their exclusive scan
    const double F = norm_factor(a, c.sumq, alpha_after(alpha0, k));
    const uint32_t chunk = chunk_of(n);
    for (int b = 0; b < kScanBlocks; ++b) {
      const uint32_t beg = (uint32_t)b * chunk;
      uint64_t acc = 0;
      for (uint32_t i = beg + threadIdx.x; i < beg + chunk && i < n; i += kScanThreads) {
        const float q = a.q[i];
        if (q > 0.0f) acc += child_count(q, F, roulette_u(a, i));
      }
      const uint64_t s = block_sum(acc, sh);
      if (threadIdx.x == 0) a.gsum[b] = (uint32_t)s;
    }
    __syncthreads();
    scan_blocks(a.gsum, a.boff, sh);
  }
  if (threadIdx.x == 0) {
    if (k > 0) {
      const double alpha = alpha_after(alpha0, k);
      *a.alpha = alpha;
      c.F = norm_factor(a, c.sumq, alpha);
      c.S = (uint32_t)chosen_S;
      c.retries = (uint32_t)k;
      a.ctl[a.depth + 1].n = (uint32_t)chosen_S;
    } else {
      // alpha fell below 1e-3 before any reduction fit: end this pass at this depth, report it
      *a.alpha = alpha_after(alpha0, -k);
      c.F = 0.0;
      c.S = 0;
      c.retries = (uint32_t)(-k);
      a.ctl[a.depth + 1].n = 0;
      *a.overflow = 1;
    }
  }
  if (k < 0)
    for (int b = threadIdx.x; b < kScanBlocks; b += kScanThreads) a.boff[b] = 0;
}

// Overflow guard, only active when the first count overflowed: counts for the next
// kGuardSteps values alpha * 0.99^k, k = 1..kGuardSteps (Eq. 14 applied repeatedly).
__global__ __launch_bounds__(kScanThreads) void k_guard_count(RenderArgs a) {
  if (a.ctl[a.depth].guard == 0) return;
  __shared__ uint32_t sh[kScanThreads];
  const uint32_t n = a.ctl[a.depth].n;
  const uint32_t chunk = chunk_of(n);
  const uint32_t beg = blockIdx.x * chunk;
  const double sumq = a.ctl[a.depth].sumq;
  double alpha = *a.alpha;
  for (int k = 0; k < kGuardSteps; ++k) {
    alpha *= 0.99;
    const double F = norm_factor(a, sumq, alpha);
    uint32_t acc = 0;
    for (uint32_t base = beg; base < beg + chunk && base < n; base += kScanThreads) {
      const uint32_t i = base + threadIdx.x;
      if (i < n && i < beg + chunk) {
        const float q = a.q[i];
        if (q > 0.0f) acc += child_count(q, F, roulette_u(a, i));
      }
    }
    const uint32_t s = block_sum(acc, sh);
    if (threadIdx.x == 0) a.gsum[kScanBlocks * k + blockIdx.x] = s;
  }
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = (int)__lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = (uint32_t)__shfl_up((int)v, off);
    if (lane >= off) v += t;
  }
  return v;
}

// First child slot of every entry: per-tile exclusive scan (wave scans, then the waves'
// totals) plus the block's offset.
__global__ __launch_bounds__(kScanThreads) void k_offsets(RenderArgs a) {
  constexpr int kWaves = kScanThreads / 64;
  __shared__ uint32_t wsum[2][kWaves];
  const uint32_t n = a.ctl[a.depth].n;
  const uint32_t chunk = chunk_of(n);
  const uint32_t beg = blockIdx.x * chunk;
  const double F = a.ctl[a.depth].F;
  // the counts k_roulette_count stored are final unless the guard chose a smaller alpha
  const bool stored = a.ctl[a.depth].guard == 0;
  uint32_t run = a.boff[blockIdx.x];
  const int tid = threadIdx.x, wave = tid >> 6;
  int buf = 0;
  for (uint32_t base = beg; base < beg + chunk && base < n; base += kScanThreads) {
    const uint32_t i = base + tid;
    uint32_t x = 0;
    if (i < n && i < beg + chunk) {
      if (stored) {
        x = a.offs[i];
      } else {
        const float q = a.q[i];
        if (q > 0.0f) x = child_count(q, F, roulette_u(a, i));
      }
    }
    const uint32_t incl = wave_incl_scan(x);
    if ((tid & 63) == 63) wsum[buf][wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t t = wsum[buf][w];
      before += w < wave ? t : 0u;
      total += t;
    }
    if (i < n && i < beg + chunk) a.offs[i] = run + before + incl - x;
    run += total;
    buf ^= 1;  // the next tile writes the other buffer: one barrier per tile suffices
  }
}

// ------------------------------------------------------------------------------ expand
// One thread per child slot: find the parent by binary search over the offsets, sample
// the BSDF with the child's own random numbers and write the child densely.
// Largest i with offs[i] <= s: the parent of child slot s under parent-major compaction.
__device__ __forceinline__ uint32_t find_parent(const uint32_t* offs, uint32_t n, uint32_t s) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (offs[mid] <= s) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kEntryThreads) void k_parents(RenderArgs a) {
  const uint32_t S = a.ctl[a.depth].S;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) a.dbg_parent[s] = find_parent(a.offs, a.ctl[a.depth].n, s);
}

// Child s = child j of parent i: BSDF sample, throughput divided by the parent's normalized
// factor, origin offset along the face-forwarded normal.
__device__ __forceinline__ void expand_child(const RenderArgs& a, uint32_t i, uint32_t s, uint32_t j) {
  const float qn = (float)(a.ctl[a.depth].F * (double)a.q[i]);
  const float4 vp = a.vpos[i], vn = a.vnrm[i], dr = a.qin.dir[i], th = a.qin.thr[i];
  const uint2 lin = a.qin.id[i];
  const uint32_t mid = bits(vn.w);
  const float4 m0 = a.sc.mat[2 * mid], m1 = a.sc.mat[2 * mid + 1];
  const V3 nrm = xyz(vn);
  V3 tb, bb;
  basis(nrm, tb, bb);
  const V3 wo = v3(-dr.x, -dr.y, -dr.z);
  const V3 wol = v3(dot(wo, tb), dot(wo, bb), dot(wo, nrm));
  const uint4 r = draw(a.key, lin, kPurposeChild, a.depth, j);
  const float u2 = unit(r.x), u3 = unit(r.y);
  V3 wil, w;
  bool alive = true;
  if (bits(m1.w) == 1u) {
    alive = sample_ggx(m0.w, xyz(m0), wol, u2, u3, wil, w);
  } else {
    wil = sample_cosine(u2, u3);
    w = xyz(m0);
  }
  const V3 wi = normalized(wil.x * tb + wil.y * bb + wil.z * nrm);
  const float inv_q = 1.0f / qn;
  const V3 tc = alive ? v3(th.x * w.x * inv_q, th.y * w.y * inv_q, th.z * w.z * inv_q) : v3(0.0f, 0.0f, 0.0f);
  const uint32_t flags = (bits(th.w) & kFlagTrain) | (alive ? 0u : kFlagDead);
  // the child leaves the surface from a point offset along the face-forwarded normal
  const float eps = a.sc.offset;
  a.qout.orig[s] = make_float4(fmaf(eps, nrm.x, vp.x), fmaf(eps, nrm.y, vp.y), fmaf(eps, nrm.z, vp.z), vp.w);
  a.qout.dir[s] = pack(wi, bits(dr.w));
  a.qout.thr[s] = pack(tc, flags);
  a.qout.id[s] = make_uint2(r.z, r.w);
  if (a.records_on && (flags & kFlagTrain)) a.qout.rec[s] = a.qin.rec[i];
  if (a.trace) a.qout.path[s] = a.qin.path[i];
  if (a.nee) a.qout.pdf[s] = bits(m1.w) == 1u ? ggx_pdf(m0.w, wol, wil) : wil.z * 0.31830988618379067f;
}

// Children of a block of kEntryThreads consecutive parents: the block's offsets go to LDS and
// each child finds its parent (the last one whose first child is <= s) by a binary search
// there; children are written in slot order, so stores coalesce.
__global__ __launch_bounds__(kEntryThreads) void k_expand(RenderArgs a) {
  __shared__ uint32_t so[kEntryThreads + 1];
  const uint32_t n = a.ctl[a.depth].n, S = a.ctl[a.depth].S;
  const uint32_t p0 = blockIdx.x * kEntryThreads;
  if (p0 >= n) return;  // uniform over the block
  const uint32_t np = min((uint32_t)kEntryThreads, n - p0);
  const uint32_t tid = threadIdx.x;
  if (tid < np) so[tid] = a.offs[p0 + tid];
  if (tid == 0) so[np] = p0 + np < n ? a.offs[p0 + np] : S;
  __syncthreads();
  const uint32_t c1 = so[np];
  for (uint32_t s = so[0] + tid; s < c1; s += kEntryThreads) {
    uint32_t lo = 0, hi = np;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (so[mid] <= s) lo = mid;
      else hi = mid;
    }
    expand_child(a, p0 + lo, s, s - so[lo]);
  }
}

// ------------------------------------------------------------------------------ misc
__global__ void k_guide(const double* image, uint32_t npx, const PassState* ps, float* guide) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npx) return;
  const double spp = ps->spp;
  const double* c = image + 3ull * p;
  guide[p] = (float)((0.2126 * c[0] + 0.7152 * c[1] + 0.0722 * c[2]) / spp);
}

__global__ void k_begin_pass(PassState* ps, double spp_per_pass) {
  ps->pass += 1u;
  ps->spp += spp_per_pass;
}
__global__ void k_set_pass_state(PassState* ps, uint32_t pass, double spp) {
  ps->pass = pass;
  ps->spp = spp;
}

__global__ void k_zero_u32(uint32_t* p, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}
__global__ void k_zero_f64(double* p, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}
__global__ void k_fill_f32(float* p, uint64_t n, float v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_set_f64(double* p, double v) { *p = v; }

__global__ void k_accumulate_stats(const DepthCtl* ctl, uint32_t D, unsigned long long* n_sum,
                                   unsigned long long* s_sum, unsigned long long* r_sum, double* sumq_last,
                                   double* f_last) {
  const uint32_t d = threadIdx.x + 1;
  if (d > D) return;
  n_sum[d] += ctl[d].n;
  if (d < D) {
    s_sum[d] += ctl[d].S;
    r_sum[d] += ctl[d].retries;
    sumq_last[d] = ctl[d].sumq;
    f_last[d] = ctl[d].F;
  }
}

__global__ void k_philox(const uint4* ctr, uint2 key, uint4* out, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = philox(ctr[i], key);
}

inline uint32_t blocks_for(uint64_t n, int threads) { return (uint32_t)((n + threads - 1) / threads); }

}  // namespace

void launch_camera(const RenderArgs& a, hipStream_t s) {
  // enough threads for the primary rays and for clearing every depth's claim counters
  const uint32_t nthreads = std::max(a.nprim, (a.max_depth + 1) * kWorkSlices);
  hipLaunchKernelGGL(k_camera, dim3(blocks_for(nthreads, kEntryThreads)), dim3(kEntryThreads), 0, s, a);
}
template <bool kCount>
void launch_extend_t(const RenderArgs& a, hipStream_t s) {
  const dim3 g(a.trace_blocks), b(kTraceThreads);
  if (a.sc.n_inst) {  // two-level scene: modes 0, 1 and 3 (the tuning keeps to these)
    if (a.ext_variant == 0) hipLaunchKernelGGL((k_extend_inst<0, kCount>), g, b, 0, s, a);
    else if (a.ext_variant == 1) hipLaunchKernelGGL((k_extend_inst<1, kCount>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_extend_inst<3, kCount>), g, b, 0, s, a);
    return;
  }
  if (a.ext_variant == 4) hipLaunchKernelGGL((k_extend<4, kCount>), g, b, 0, s, a);
  else if (a.ext_variant == 3) hipLaunchKernelGGL((k_extend<3, kCount>), g, b, 0, s, a);
  else if (a.ext_variant == 2) hipLaunchKernelGGL((k_extend<2, kCount>), g, b, 0, s, a);
  else if (a.ext_variant == 1) hipLaunchKernelGGL((k_extend<1, kCount>), g, b, 0, s, a);
  else hipLaunchKernelGGL(k_extend_immediate<kCount>, g, b, 0, s, a);
}
void launch_extend(const RenderArgs& a, hipStream_t s) {
  if (a.count_work) launch_extend_t<true>(a, s);
  else launch_extend_t<false>(a, s);
}
uint32_t extend_blocks_per_cu(uint32_t variant, bool inst) {
  int nb = 0;
  hipError_t e;
  if (inst && variant == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_extend_inst<0, false>, kTraceThreads, 0);
  else if (inst && variant == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_extend_inst<1, false>, kTraceThreads, 0);
  else if (inst) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_extend_inst<3, false>, kTraceThreads, 0);
  else if (variant == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_extend<4, false>, kTraceThreads, 0);
  else if (variant == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_extend<3, false>, kTraceThreads, 0);
  else if (variant == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_extend<2, false>, kTraceThreads, 0);
  else if (variant == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_extend<1, false>, kTraceThreads, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_extend_immediate<false>, kTraceThreads, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return (uint32_t)nb;
}
uint32_t extend_threads_per_block() { return kTraceThreads; }
uint32_t extend_spill_depth() { return kStackMax - kLdsStack; }
void launch_record_features(const RenderArgs& a, uint64_t records_cap, hipStream_t s) {
  if (records_cap)
    hipLaunchKernelGGL(k_record_features, dim3(blocks_for(records_cap, kEntryThreads)), dim3(kEntryThreads), 0, s, a);
}
void launch_shade(const RenderArgs& a, hipStream_t s) {
  const dim3 g(blocks_for(a.cap, kShadeThreads)), b(kShadeThreads);
  if (a.nee && a.sc.n_inst) hipLaunchKernelGGL((k_shade<true, true>), g, b, 0, s, a);
  else if (a.nee) hipLaunchKernelGGL((k_shade<true, false>), g, b, 0, s, a);
  else if (a.sc.n_inst) hipLaunchKernelGGL((k_shade<false, true>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_shade<false, false>), g, b, 0, s, a);
}

void launch_nee(const RenderArgs& a, hipStream_t s) {
  // the shadow rays sit in the out-queue's origin / direction / throughput slots; the traversal
  // writes their closest hits over the out-queue's record slots, with claim counters and work
  // counters of their own
  RenderArgs b = a;
  b.qin.orig = a.qout.orig;
  b.qin.dir = a.qout.dir;
  b.qin.thr = a.qout.thr;
  b.qin.id = a.qout.id;
  b.qin.rec = a.qout.rec;
  b.qin.path = nullptr;
  b.qin.pdf = nullptr;
  b.hit = reinterpret_cast<float4*>(a.qout.rec);
  b.work = a.work_nee;
  b.rays = a.rays + 3;
  b.count_work = 0u;
  b.trace = nullptr;
  launch_extend(b, s);
  hipLaunchKernelGGL(k_nee_resolve, dim3(blocks_for(a.cap, kShadeThreads)), dim3(kShadeThreads), 0, s, a);
}
void launch_sum_q(const RenderArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_q_partial, dim3(kScanBlocks), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(k_sum_q_final, dim3(1), dim3(kScanThreads), 0, s, a);
}
void launch_roulette(const RenderArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_roulette_count, dim3(kScanBlocks), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(k_roulette_scan, dim3(1), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(k_guard_count, dim3(kScanBlocks), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(k_guard_select, dim3(1), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(k_offsets, dim3(kScanBlocks), dim3(kScanThreads), 0, s, a);
}
void launch_expand(const RenderArgs& a, hipStream_t s) {
  if (a.cap == 0) return;
  hipLaunchKernelGGL(k_expand, dim3(blocks_for(a.cap, kEntryThreads)), dim3(kEntryThreads), 0, s, a);
}
void launch_parents(const RenderArgs& a, hipStream_t s) {
  if (a.cap == 0) return;
  hipLaunchKernelGGL(k_parents, dim3(blocks_for(a.cap, kEntryThreads)), dim3(kEntryThreads), 0, s, a);
}
void launch_guide(const RenderArgs& a, float* guide, hipStream_t s) {
  const uint32_t npx = a.width * a.height;
  hipLaunchKernelGGL(k_guide, dim3(blocks_for(npx, 256)), dim3(256), 0, s, a.image, npx, a.pass_state, guide);
}
void launch_begin_pass(const RenderArgs& a, double spp_per_pass, hipStream_t s) {
  hipLaunchKernelGGL(k_begin_pass, dim3(1), dim3(1), 0, s, a.pass_state, spp_per_pass);
}
void launch_set_pass_state(PassState* ps, uint32_t pass, double spp, hipStream_t s) {
  hipLaunchKernelGGL(k_set_pass_state, dim3(1), dim3(1), 0, s, ps, pass, spp);
}
void launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_zero_u32, dim3(std::min<uint64_t>(blocks_for(n, 256), 4096)), dim3(256), 0, s, p, n);
}
void launch_zero_f64(double* p, uint64_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_zero_f64, dim3(std::min<uint64_t>(blocks_for(n, 256), 4096)), dim3(256), 0, s, p, n);
}
void launch_fill_f32(float* p, uint64_t n, float v, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_f32, dim3(std::min<uint64_t>(blocks_for(n, 256), 4096)), dim3(256), 0, s, p, n, v);
}
void launch_set_f64(double* p, double v, hipStream_t s) { hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, s, p, v); }
void launch_accumulate_stats(const DepthCtl* ctl, uint32_t max_depth, unsigned long long* n_sum,
                             unsigned long long* s_sum, unsigned long long* r_sum, double* sumq_last,
                             double* f_last, hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate_stats, dim3(1), dim3(64), 0, s, ctl, max_depth, n_sum, s_sum, r_sum, sumq_last,
                     f_last);
}
void launch_philox(const uint4* ctr, uint2 key, uint4* out, uint32_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_philox, dim3(blocks_for(n, 256)), dim3(256), 0, s, ctr, key, out, n);
}

}  // namespace nrrs
