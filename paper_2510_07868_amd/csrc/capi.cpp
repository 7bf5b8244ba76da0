// Host runtime of the C ABI declared in include/nrrs.h: workspace carving, scene upload
// (host BVH build), the per-pass launch sequence of the wavefront bounce loop, training
// steps and the test entry points.  No device memory is allocated here: every buffer is
// carved out of the caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/nrrs.h"
#include "bvh.hpp"
#include "launch.hpp"

using namespace nrrs;

namespace {

constexpr uint32_t kMaxMinibatch = 65536;

struct Carve {
  uint8_t* base;
  uint64_t off = 0;
  template <typename T>
  T* take(uint64_t count) {
    off = (off + 255) & ~uint64_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * count;
    return p;
  }
};

}  // namespace

struct nrrs_ctx {
  nrrs_config cfg{};
  hipStream_t stream = nullptr;
  uint64_t npx = 0, nprim = 0, cap = 0;
  uint32_t cus = 0;                 // compute units of the device
  uint32_t ext_occ[5] = {1, 1, 1, 1, 1};  // resident traversal blocks per CU of each variant (0: not
                                          // available for the current scene)
  uint32_t ext_occ_flat[5] = {1, 1, 1, 1, 1}, ext_occ_inst[5] = {1, 1, 0, 1, 0};  // one- / two-level scenes
  bool bvh4_ok = false;             // the 4-wide tree fits the traversal stack (variant 4)
  uint32_t* spill = nullptr;        // sized for cus * max(ext_occ) blocks
  uint32_t* work = nullptr;         // traversal claim counters per depth and queue slice
  nrrs_tuning tune{};               // launch parameters of the traversal kernel
  uint64_t net_depths = 0;          // Mix-Depth table: bit d-1 = network factor at depth d (NET mode)
  uint64_t fixed_depths = 0;        // Mix-Depth table: bit d-1 = fixed rate at depth d (wins over the network)
  // workspace
  uint8_t* ws = nullptr;
  uint64_t ws_bytes = 0, max_tris = 0;
  uint32_t max_mats = 0;
  float4 *tri = nullptr, *node = nullptr, *node4 = nullptr, *mat = nullptr;
  Queue qa{}, qb{};
  uint8_t* qb_pool = nullptr;  // queue B's bytes double as scratch for the test entry points
  uint64_t qb_pool_bytes = 0;
  float4 *hit = nullptr, *vpos = nullptr, *vnrm = nullptr;
  float* q = nullptr;
  uint32_t* offs = nullptr;
  double* partial = nullptr;
  uint32_t *bsum = nullptr, *boff = nullptr, *gsum = nullptr;
  DepthCtl* ctl = nullptr;
  double* alpha = nullptr;
  uint32_t* overflow = nullptr;
  unsigned long long* rays = nullptr;
  unsigned long long *st_n = nullptr, *st_s = nullptr, *st_r = nullptr;
  double *st_sumq = nullptr, *st_f = nullptr;
  uint32_t* work_nee = nullptr;  // shadow-ray claim counters (next-event estimation)
  float4* light_geo = nullptr;  // NEE light list (world-space triangles) and its CDF
  float* light_cdf = nullptr;
  double* f_fixed = nullptr;  // [NRRS_MAX_DEPTH + 1] normalization factors given by nrrs_debug_set_norm_factors
  uint32_t f_fixed_n = 0;     // depths 1..f_fixed_n use them (0: computed)
  double* image = nullptr;
  float* guide = nullptr;
  double* trace = nullptr;  // per-path radiance [nprim][trace_depth][3] (reserved when cfg.trace_depth > 0)
  bool trace_on = false;
  Records rec{};
  float* target = nullptr;
  float *master = nullptr, *adam_m = nullptr, *adam_v = nullptr, *grad = nullptr;
  float* infer = nullptr;  // inference weights: moving average of master (or master itself)
  uint16_t* bf16 = nullptr;
  uint8_t* fp8 = nullptr;
  float* fp8_scale = nullptr;
  float *grad_partial = nullptr, *loss_partial = nullptr, *loss_accum = nullptr;
  // NRRS proper (reserved when cfg.hash_log2 > 0): StatNet, RRSNet and the hash grid, each as
  // master, inference copy, Adam moments and gradient; gradient partials; per-pixel error state
  struct NetState {
    float *w = nullptr, *infer = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  };
  NetState nstat{}, nrrs_net{}, ntab{}, naid{}, ntab_r{};  // naid, ntab_r: the AID-NRRS RRSNet
  uint64_t ntab_n = 0;  // floats of the hash grid
  float *npartial = nullptr, *nloss_part = nullptr, *nloss = nullptr, *ngroups = nullptr;
  double *lum_start = nullptr, *pix_part = nullptr, *eavg = nullptr;
  float *pcur = nullptr, *pref = nullptr, *pacc = nullptr, *pEp = nullptr, *pE = nullptr, *pwpx = nullptr;
  uint32_t* kpix = nullptr;
  uint64_t nrrs_step = 0, nrrs_rstep = 0, nrrs_astep = 0, nrrs_frames = 0, nrrs_spp_start = 0;
  // scene
  bool bound = false, scene = false;
  DevScene sc{};
  std::vector<uint32_t> bvh_order, orig_to_bvh;
  // counters on the host
  uint64_t spp_total = 0, passes_done = 0, adam_step = 0;
  std::string err;
  PassState* pass_state = nullptr;
  // stage timing
  bool timing = false;
  std::vector<hipEvent_t> events;
  std::vector<int> event_stage;
  // launch mode: 1 = replay one captured hipGraph per pass (keyed by depth, mode, records)
  int32_t launch_mode = 1;
  std::map<std::tuple<uint32_t, int32_t, uint32_t>, hipGraphExec_t> graphs;
  void drop_graphs() {
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  ~nrrs_ctx() {
    drop_graphs();
    for (hipEvent_t e : events) hipEventDestroy(e);
  }
};

namespace {

int32_t fail(nrrs_ctx* c, int32_t code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPC(ctx, expr)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return fail(ctx, NRRS_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

uint64_t carve(nrrs_ctx* c, uint8_t* base, uint64_t max_tris, uint32_t max_mats) {
  Carve k{base};
  const uint64_t C = c->cap, npx = c->npx, rc = c->cfg.records_cap;
  c->tri = k.take<float4>(3 * max_tris);
  c->node = k.take<float4>(4 * (max_tris + 2));
  c->node4 = k.take<float4>(8 * (max_tris + 2));  // a 4-wide node per BVH2 inner node at most
  c->mat = k.take<float4>(2 * (uint64_t)max_mats);
  for (Queue* qq : {&c->qa, &c->qb}) {
    uint64_t start = (k.off + 255) & ~uint64_t(255);
    qq->orig = k.take<float4>(C);
    qq->dir = k.take<float4>(C);
    qq->thr = k.take<float4>(C);
    qq->id = k.take<uint2>(C);
    qq->rec = k.take<int4>(C);
    qq->path = c->cfg.trace_depth ? k.take<uint32_t>(C) : nullptr;
    qq->pdf = c->cfg.nee ? k.take<float>(C) : nullptr;
    if (qq == &c->qb) {
      c->qb_pool = base ? base + start : nullptr;
      c->qb_pool_bytes = k.off - start;
    }
  }
  const uint64_t max_blocks = (uint64_t)c->cus * std::max(*std::max_element(c->ext_occ_flat, c->ext_occ_flat + 5),
                                                          *std::max_element(c->ext_occ_inst, c->ext_occ_inst + 5));
  c->spill = k.take<uint32_t>((uint64_t)extend_spill_depth() * max_blocks * extend_threads_per_block());
  c->hit = k.take<float4>(C);
  c->vpos = k.take<float4>(C);
  c->vnrm = k.take<float4>(C);
  c->q = k.take<float>(C);
  c->offs = k.take<uint32_t>(C);
  c->partial = k.take<double>(kScanBlocks);
  c->bsum = k.take<uint32_t>(kScanBlocks);
  c->boff = k.take<uint32_t>(kScanBlocks);
  c->gsum = k.take<uint32_t>((uint64_t)kScanBlocks * kGuardSteps);
  c->ctl = k.take<DepthCtl>(NRRS_MAX_DEPTH + 2);
  c->work = k.take<uint32_t>((uint64_t)(NRRS_MAX_DEPTH + 2) * kWorkSlices * kWorkStride);
  c->work_nee = c->cfg.nee ? k.take<uint32_t>((uint64_t)(NRRS_MAX_DEPTH + 2) * kWorkSlices * kWorkStride) : nullptr;
  c->light_geo = c->cfg.nee ? k.take<float4>(3 * max_tris) : nullptr;
  c->light_cdf = c->cfg.nee ? k.take<float>(max_tris + 1) : nullptr;
  c->alpha = k.take<double>(1);
  c->overflow = k.take<uint32_t>(1);
  c->rays = k.take<unsigned long long>(6);  // rays, nodes, triangles; the same for shadow rays
  c->pass_state = k.take<PassState>(1);
  c->st_n = k.take<unsigned long long>(NRRS_MAX_DEPTH + 1);
  c->st_s = k.take<unsigned long long>(NRRS_MAX_DEPTH + 1);
  c->st_r = k.take<unsigned long long>(NRRS_MAX_DEPTH + 1);
  c->st_sumq = k.take<double>(NRRS_MAX_DEPTH + 1);
  c->st_f = k.take<double>(NRRS_MAX_DEPTH + 1);
  c->f_fixed = k.take<double>(NRRS_MAX_DEPTH + 1);
  c->image = k.take<double>(3 * npx);
  c->guide = k.take<float>(npx);
  c->trace = c->cfg.trace_depth ? k.take<double>(3ull * c->cfg.trace_depth * c->nprim) : nullptr;
  c->rec.feat = k.take<float>(20 * rc);
  c->rec.lum_t = k.take<float>(rc);
  c->rec.acc = k.take<float>(rc);
  c->rec.depth = k.take<uint32_t>(rc);
  c->rec.pix = k.take<uint32_t>(rc);
  c->rec.lineage = k.take<uint2>(rc);
  c->rec.qidx = k.take<uint32_t>(rc);
  c->rec.count = k.take<uint32_t>(1);
  c->rec.cap = (uint32_t)rc;
  c->target = k.take<float>(rc);
  c->master = k.take<float>(kNParam);
  c->infer = k.take<float>(kNParam);
  c->adam_m = k.take<float>(kNParam);
  c->adam_v = k.take<float>(kNParam);
  c->grad = k.take<float>(kNParam);
  c->bf16 = k.take<uint16_t>(packed_bf16_elems());
  c->fp8 = k.take<uint8_t>(packed_fp8_bytes());
  c->fp8_scale = k.take<float>(4);
  const uint64_t gb = mlp_grad_blocks(kMaxMinibatch);
  c->grad_partial = k.take<float>(mlp_grad_scratch_floats(kMaxMinibatch));
  c->loss_partial = k.take<float>(gb);
  c->loss_accum = k.take<float>(1);
  if (c->cfg.hash_log2) {
    c->rec.nraw = k.take<float>(8 * rc);
    c->rec.ntq = k.take<float4>(rc);
    c->rec.nqf = k.take<float2>(rc);
    c->ntab_n = (uint64_t)kHgLevels * kHgFeat << c->cfg.hash_log2;
    auto state = [&](nrrs_ctx::NetState& st, uint64_t n) {
      st.w = k.take<float>(n);
      st.infer = k.take<float>(n);
      st.m = k.take<float>(n);
      st.v = k.take<float>(n);
      st.g = k.take<float>(n);
    };
    state(c->nstat, kStatParams);
    state(c->nrrs_net, kRrsParams);
    state(c->ntab, c->ntab_n);
    state(c->naid, kAidParams);
    state(c->ntab_r, c->ntab_n);
    const uint64_t nb = nrrs_grad_blocks((uint32_t)std::max<uint64_t>(rc, 1));
    c->npartial = k.take<float>(nb * std::max(kStatParams, std::max(kRrsParams, kAidParams)));
    c->nloss_part = k.take<float>(nb);
    c->nloss = k.take<float>(2);
    c->ngroups = k.take<float>((uint64_t)nrrs_sum_groups() * std::max(kStatParams, std::max(kRrsParams, kAidParams)));
    c->lum_start = k.take<double>(npx);
    c->pix_part = k.take<double>(2 * ((npx + 255) / 256));
    c->eavg = k.take<double>(1);
    c->pcur = k.take<float>(npx);
    c->pref = k.take<float>(npx);
    c->pacc = k.take<float>(npx);
    c->pEp = k.take<float>(npx);
    c->pE = k.take<float>(npx);
    c->pwpx = k.take<float>(npx);
    c->kpix = k.take<uint32_t>(npx);
  } else {
    c->rec.nraw = nullptr;
    c->rec.ntq = nullptr;
    c->rec.nqf = nullptr;
  }
  return (k.off + 255) & ~uint64_t(255);
}

// Host Philox4x32-10 for the weight initialisation (counter = (index, 0, 5, 0)).
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t pa = (uint64_t)0xD2511F53u * c[0], pb = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t n0 = (uint32_t)(pb >> 32) ^ c[1] ^ k0, n2 = (uint32_t)(pa >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)pb;
    c[2] = n2;
    c[3] = (uint32_t)pa;
  }
}

// He-uniform weights, zero biases, output layer scaled by 0.1.
void init_params(uint64_t seed, std::vector<float>& w) {
  w.assign(kNParam, 0.0f);
  struct L {
    int off, n, fan_in;
    float extra;
  } layers[] = {{kW1, 1280, 20, 1.0f}, {kW2, 4096, 64, 1.0f}, {kW3, 4096, 64, 1.0f}, {kW4, 64, 64, 0.1f}};
  for (const L& l : layers) {
    const float lim = std::sqrt(6.0f / (float)l.fan_in) * l.extra;
    for (int k = 0; k < l.n; ++k) {
      uint32_t c[4] = {(uint32_t)(l.off + k), 0u, 5u, 0u};
      philox_host(c, (uint32_t)seed, (uint32_t)(seed >> 32));
      float u = (float)(c[0] >> 8) * 0x1.0p-24f;
      w[l.off + k] = (2.0f * u - 1.0f) * lim;
    }
  }
}

// NRRS networks: He-uniform hidden layers (leaky ReLU), output layers scaled by 0.1, zero
// biases except RRSNet's output bias 2 (1 - ln 2), which starts the factor at 1 (Eq. 22 at
// z >= 0: z / 2 + ln 2); hash-grid features uniform in [-1e-4, 1e-4].  Philox counters
// (index, stream, 7, 0) keep the three vectors independent of the NET weights.
void init_nrrs_params(uint64_t seed, std::vector<float>& stat, std::vector<float>& rrs, std::vector<float>& table,
                      uint64_t table_n, std::vector<float>& aid, std::vector<float>& table_r) {
  auto uni = [&](uint32_t stream, uint64_t i) {
    uint32_t c[4] = {(uint32_t)i, stream, 7u, (uint32_t)(i >> 32)};
    philox_host(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return (float)(c[0] >> 8) * 0x1.0p-24f;
  };
  auto mlp = [&](std::vector<float>& w, int in, int out, uint32_t stream) {
    w.assign(mlp32_params(in, out), 0.0f);
    const int fan_in[4] = {in, 32, 32, 32}, fan_out[4] = {32, 32, 32, out};
    uint64_t o = 0;
    for (int L = 0; L < 4; ++L) {
      const float lim = std::sqrt(6.0f / (float)fan_in[L]) * (L == 3 ? 0.1f : 1.0f);
      for (int k = 0; k < fan_in[L] * fan_out[L]; ++k) w[o + k] = (2.0f * uni(stream, o + k) - 1.0f) * lim;
      o += (uint64_t)fan_in[L] * fan_out[L] + fan_out[L];
    }
  };
  mlp(stat, kStatIn, kStatOut, 1u);
  mlp(rrs, kRrsIn, 1, 2u);
  rrs[kRrsParams - 1] = 2.0f * (1.0f - 0.69314718055994531f);
  mlp(aid, kAidIn, 1, 4u);
  aid[kAidParams - 1] = 2.0f * (1.0f - 0.69314718055994531f);
  table.resize(table_n);
  table_r.resize(table_n);
  for (uint64_t k = 0; k < table_n; ++k) table[k] = (2.0f * uni(3u, k) - 1.0f) * 1e-4f;
  for (uint64_t k = 0; k < table_n; ++k) table_r[k] = (2.0f * uni(5u, k) - 1.0f) * 1e-4f;
}

int32_t upload_nrrs_state(nrrs_ctx* c, const float* stat, const float* rrs, const float* table,
                          const float* aid = nullptr, const float* table_r = nullptr) {
  hipStream_t s = c->stream;
  auto put = [&](nrrs_ctx::NetState& st, const float* src, uint64_t n) -> int32_t {
    if (!src) return NRRS_OK;
    HIPC(c, hipMemcpyAsync(st.w, src, sizeof(float) * n, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(st.infer, src, sizeof(float) * n, hipMemcpyHostToDevice, s));
    launch_zero_u32((uint32_t*)st.m, n, s);
    launch_zero_u32((uint32_t*)st.v, n, s);
    launch_zero_u32((uint32_t*)st.g, n, s);
    return NRRS_OK;
  };
  int32_t r = put(c->nstat, stat, kStatParams);
  if (r == NRRS_OK) r = put(c->nrrs_net, rrs, kRrsParams);
  if (r == NRRS_OK) r = put(c->ntab, table, c->ntab_n);
  if (r == NRRS_OK) r = put(c->naid, aid, kAidParams);
  if (r == NRRS_OK) r = put(c->ntab_r, table_r, c->ntab_n);
  if (r != NRRS_OK) return r;
  HIPC(c, hipStreamSynchronize(s));
  if (stat || table) c->nrrs_step = 0;
  if (rrs) c->nrrs_rstep = 0;
  if (aid || table_r) c->nrrs_astep = 0;
  return NRRS_OK;
}

NrrsNet nrrs_net_args(nrrs_ctx* c, bool inference) {
  NrrsNet n{};
  n.stat = inference ? c->nstat.infer : c->nstat.w;
  n.rrs = inference ? c->nrrs_net.infer : c->nrrs_net.w;
  n.table = inference ? c->ntab.infer : c->ntab.w;
  n.aid = inference ? c->naid.infer : c->naid.w;
  n.table_r = inference ? c->ntab_r.infer : c->ntab_r.w;
  n.log2T = c->cfg.hash_log2;
  return n;
}

RenderArgs base_args(nrrs_ctx* c) {
  RenderArgs a{};
  a.sc = c->sc;
  a.qin = c->qa;
  a.qout = c->qb;
  a.hit = c->hit;
  a.vpos = c->vpos;
  a.vnrm = c->vnrm;
  a.q = c->q;
  a.offs = c->offs;
  a.partial = c->partial;
  a.bsum = c->bsum;
  a.boff = c->boff;
  a.gsum = c->gsum;
  a.ctl = c->ctl;
  a.alpha = c->alpha;
  a.overflow = c->overflow;
  a.rays = c->rays;
  a.image = c->image;
  a.guide = c->guide;
  a.trace = c->trace_on ? c->trace : nullptr;
  a.trace_depth = c->cfg.trace_depth;
  a.rec = c->rec;
  a.key = make_uint2((uint32_t)c->cfg.seed, (uint32_t)(c->cfg.seed >> 32));
  a.width = c->cfg.width;
  a.height = c->cfg.height;
  a.nprim = (uint32_t)c->nprim;
  a.cap = (uint32_t)c->cap;
  a.norm_mode = (uint32_t)c->cfg.norm_mode;
  a.net_max_depth = (uint32_t)c->cfg.net_max_depth;
  a.p_train = (float)c->cfg.p_train;
  a.f_rate = c->cfg.f_rate;
  a.budget_base = (double)c->nprim;
  a.F_fixed = c->f_fixed_n ? c->f_fixed : nullptr;
  a.dbg_parent = nullptr;
  a.spill = c->spill;
  a.work = c->work;
  a.trace_blocks = c->cus * c->tune.extend_blocks_per_cu;
  a.ext_variant = c->tune.extend_variant;
  a.ext_refill = c->tune.extend_refill;
  a.ext_leaf_batch = c->tune.extend_leaf_batch;
  a.ext_chunk = c->tune.extend_chunk;
  a.count_work = c->timing ? 1u : 0u;
  a.nee = c->cfg.nee;
  a.work_nee = c->work_nee;
  a.pass_state = c->pass_state;
  return a;
}

NetArgs net_args(nrrs_ctx* c, int32_t precision) {
  NetArgs n{};
  n.master = c->infer;
  n.bf16 = c->bf16;
  n.fp8 = c->fp8;
  n.fp8_scale = c->fp8_scale;
  n.precision = precision;
  return n;
}

bool finite_all(const float* p, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

extern "C" {

const char* nrrs_status_string(int32_t s) {
  switch (s) {
    case NRRS_OK: return "ok";
    case NRRS_EINVAL: return "invalid argument";
    case NRRS_ESTATE: return "call out of order";
    case NRRS_ENOMEM: return "workspace too small";
    case NRRS_EHIP: return "HIP runtime error";
    case NRRS_EOVERFLOW: return "queue overflow guard exhausted";
    case NRRS_EUNSUPPORTED: return "unsupported device or feature";
    default: return "unknown status";
  }
}

const char* nrrs_last_error(const nrrs_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t nrrs_create(const nrrs_config* cfg, void* hip_stream, nrrs_ctx** out) {
  if (!cfg || !out) return NRRS_EINVAL;
  *out = nullptr;
  if (cfg->width == 0 || cfg->height == 0 || cfg->s_batch == 0 || !(cfg->cap_factor >= 1.0) ||
      !(cfg->f_rate > 0.0) || cfg->net_max_depth < 0 || cfg->net_max_depth > kMaxRec ||
      (cfg->norm_mode != NRRS_NORM_TWO_SIDED && cfg->norm_mode != NRRS_NORM_DOWNSCALE) ||
      cfg->precision < NRRS_PREC_FP32 || cfg->precision > NRRS_PREC_FP8 || !(cfg->p_train >= 0.0) ||
      cfg->p_train > 1.0 || (cfg->loss != NRRS_LOSS_REL_L2 && cfg->loss != NRRS_LOSS_LOG_MSE) ||
      !(cfg->ema_decay >= 0.0) || cfg->ema_decay >= 1.0 || cfg->trace_depth > NRRS_MAX_DEPTH ||
      (cfg->hash_log2 != 0 && (cfg->hash_log2 < 14 || cfg->hash_log2 > 22)) || cfg->nee > 1)
    return NRRS_EINVAL;
  const uint64_t npx = (uint64_t)cfg->width * cfg->height;
  const uint64_t nprim = npx * cfg->s_batch;
  const uint64_t cap = (uint64_t)std::floor(cfg->cap_factor * (double)nprim);
  if (nprim > 0x40000000ull || cap > 0x7fffffffull) return NRRS_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return NRRS_EHIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return NRRS_EHIP;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return NRRS_EUNSUPPORTED;
  nrrs_ctx* c = new (std::nothrow) nrrs_ctx();
  if (!c) return NRRS_EINVAL;
  c->cfg = *cfg;
  c->net_depths = (uint64_t(1) << cfg->net_max_depth) - 1;
  c->stream = (hipStream_t)hip_stream;
  c->npx = npx;
  c->nprim = nprim;
  c->cap = cap;
  c->cus = (uint32_t)prop.multiProcessorCount;
  for (uint32_t v = 0; v < 5; ++v) {
    c->ext_occ_flat[v] = c->ext_occ[v] = extend_blocks_per_cu(v, false);
    c->ext_occ_inst[v] = (v == 0 || v == 1 || v == 3) ? extend_blocks_per_cu(v, true) : 0u;
  }
  c->tune.extend_variant = 3;
  c->tune.extend_blocks_per_cu = c->ext_occ[3];
  c->tune.extend_refill = 16;
  c->tune.extend_leaf_batch = 12;
  c->tune.extend_chunk = 64;
  warm_mfma_launch_cache();
  *out = c;
  return NRRS_OK;
}

void nrrs_destroy(nrrs_ctx* ctx) {
  if (!ctx) return;
  if (ctx->bound) hipStreamSynchronize(ctx->stream);
  delete ctx;
}

int32_t nrrs_workspace_size(const nrrs_ctx* ctx, uint64_t max_tris, uint32_t max_materials, uint64_t* bytes) {
  if (!ctx || !bytes || max_tris == 0 || max_materials == 0 || max_tris > (1ull << 28)) return NRRS_EINVAL;
  nrrs_ctx tmp = *ctx;
  *bytes = carve(&tmp, nullptr, max_tris, max_materials);
  return NRRS_OK;
}

int32_t nrrs_bind_workspace(nrrs_ctx* c, void* device_ptr, uint64_t bytes, uint64_t max_tris, uint32_t max_materials) {
  if (!c || !device_ptr || max_tris == 0 || max_materials == 0 || max_tris > (1ull << 28)) return NRRS_EINVAL;
  if (((uintptr_t)device_ptr & 255u) != 0) return fail(c, NRRS_EINVAL, "workspace must be 256-byte aligned");
  nrrs_ctx tmp = *c;
  const uint64_t need = carve(&tmp, nullptr, max_tris, max_materials);
  if (bytes < need) return fail(c, NRRS_ENOMEM, "workspace smaller than nrrs_workspace_size");
  carve(c, (uint8_t*)device_ptr, max_tris, max_materials);
  c->ws = (uint8_t*)device_ptr;
  c->ws_bytes = bytes;
  c->drop_graphs();
  c->max_tris = max_tris;
  c->max_mats = max_materials;
  c->bound = true;
  c->scene = false;
  c->trace_on = false;
  hipStream_t s = c->stream;
  launch_zero_f64(c->image, 3 * c->npx, s);
  launch_fill_f32(c->guide, c->npx, -1.0f, s);
  launch_zero_u32(c->rec.count, 1, s);
  launch_set_f64(c->alpha, 1.0, s);
  launch_zero_u32((uint32_t*)c->ctl, (sizeof(DepthCtl) * (NRRS_MAX_DEPTH + 2)) / 4, s);
  launch_zero_u32((uint32_t*)c->adam_m, kNParam, s);
  launch_zero_u32((uint32_t*)c->adam_v, kNParam, s);
  std::vector<float> w;
  init_params(c->cfg.seed, w);
  HIPC(c, hipMemcpyAsync(c->master, w.data(), sizeof(float) * kNParam, hipMemcpyHostToDevice, s));
  HIPC(c, hipMemcpyAsync(c->infer, w.data(), sizeof(float) * kNParam, hipMemcpyHostToDevice, s));
  launch_quantize(c->infer, c->bf16, c->fp8, c->fp8_scale, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  c->spp_total = 0;
  c->passes_done = 0;
  c->adam_step = 0;
  if (c->cfg.hash_log2) {
    std::vector<float> ws_, wr_, wt_, wa_, wtr_;
    init_nrrs_params(c->cfg.seed, ws_, wr_, wt_, c->ntab_n, wa_, wtr_);
    const int32_t r = upload_nrrs_state(c, ws_.data(), wr_.data(), wt_.data(), wa_.data(), wtr_.data());
    if (r != NRRS_OK) return r;
    launch_zero_f64(c->lum_start, c->npx, s);
    c->nrrs_frames = 0;
    c->nrrs_spp_start = 0;
    HIPC(c, hipStreamSynchronize(s));
  }
  return NRRS_OK;
}

namespace {

// A scene ready for the device: triangle slots (12 floats: v0, tag; e1, material; e2, 0), tree
// nodes (16 floats), the optional 4-wide copy, instance records (28 floats) with their uid index,
// the flattened triangles' world geometry for the light list, and the uid <-> flattened-index
// maps of the debug entry points.
struct SceneHost {
  std::vector<float> tri, nodes, nodes4, inst;
  std::vector<uint32_t> inst_uid;  // (first uid, record) pairs, ascending
  uint64_t n_nodes4 = 0;
  bool bvh4_ok = false;
  uint32_t root = 0, nt_base = 0, n_inst = 0;
  float amin[3] = {INFINITY, INFINITY, INFINITY}, amax[3] = {-INFINITY, -INFINITY, -INFINITY};
  std::vector<float> light_geo;  // 12 floats per emitting triangle, flattened order
  std::vector<double> light_w;   // lum(L_e) x area of each
  std::vector<uint32_t> uid_to_flat, flat_to_uid;
};

void grow_bounds(SceneHost& h, const float* p) {
  for (int a = 0; a < 3; ++a) {
    h.amin[a] = std::fmin(h.amin[a], p[a]);
    h.amax[a] = std::fmax(h.amax[a], p[a]);
  }
}

// The light list entry of a world-space triangle (v0, v1, v2 as float) with material m.
void add_light(SceneHost& h, const float* v0, const float* v1, const float* v2, uint32_t m, const float* mat_params) {
  const float* le = mat_params + 7ull * m + 4;
  const double l = 0.2126 * le[0] + 0.7152 * le[1] + 0.0722 * le[2];
  if (!(l > 0.0)) return;
  float g[12];
  for (int a = 0; a < 3; ++a) {
    g[a] = v0[a];
    g[4 + a] = v1[a] - v0[a];
    g[8 + a] = v2[a] - v0[a];
  }
  std::memcpy(&g[3], &m, 4);
  std::memcpy(&g[7], &m, 4);
  g[11] = 0.0f;
  const double cx = (double)g[5] * g[10] - (double)g[6] * g[9];
  const double cy = (double)g[6] * g[8] - (double)g[4] * g[10];
  const double cz = (double)g[4] * g[9] - (double)g[5] * g[8];
  const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
  if (!(area > 0.0)) return;
  h.light_geo.insert(h.light_geo.end(), g, g + 12);
  h.light_w.push_back(l * area);
}

// Checks shared by both uploads: a triangle list over nv vertices with materials below nm.
int32_t check_mesh(nrrs_ctx* c, const float* verts, uint64_t nv, const uint32_t* tris, uint64_t nt,
                   const uint32_t* tri_mat, uint32_t nm) {
  if (!finite_all(verts, 3 * nv)) return fail(c, NRRS_EINVAL, "non-finite scene value");
  for (uint64_t i = 0; i < 3 * nt; ++i)
    if (tris[i] >= nv) return fail(c, NRRS_EINVAL, "triangle vertex index out of range");
  for (uint64_t i = 0; i < nt; ++i)
    if (tri_mat[i] >= nm) return fail(c, NRRS_EINVAL, "triangle material out of range");
  return NRRS_OK;
}

int32_t check_tree(nrrs_ctx* c, const BvhOut& b) {
  if (b.max_depth > kMaxBvhDepth) return fail(c, NRRS_EINVAL, "BVH deeper than the traversal stack");
  for (uint64_t i = 0; i < 2 * b.n_nodes; ++i) {
    uint32_t l;
    std::memcpy(&l, &b.nodes[16 * (i / 2) + 12 + (i % 2)], 4);
    if ((l & 0x80000000u) && (l & 7u) + 1u > kLeafMaxTris) return fail(c, NRRS_EINVAL, "BVH leaf too large");
  }
  return NRRS_OK;
}

// Appends tree b to h.nodes: inner links move by the node offset, leaf links by first_slot
// (their triangles' or instances' first index), instance leaves get kInstLeaf.
void append_tree(SceneHost& h, const BvhOut& b, uint32_t first_slot, bool inst_leaves) {
  const uint32_t off = (uint32_t)(h.nodes.size() / 16);
  const size_t at = h.nodes.size();
  h.nodes.insert(h.nodes.end(), b.nodes.begin(), b.nodes.end());
  for (uint64_t i = 0; i < b.n_nodes; ++i)
    for (int c = 0; c < 2; ++c) {
      float* f = &h.nodes[at + 16 * i + 12 + c];
      uint32_t l;
      std::memcpy(&l, f, 4);
      if (l & 0x80000000u) {
        const uint32_t first = ((l >> 3) & 0x0fffffffu) + first_slot;
        l = 0x80000000u | (first << 3) | (l & 3u) | (inst_leaves ? kInstLeaf : 0u);
      } else {
        l += off;
      }
      std::memcpy(f, &l, 4);
    }
}

// Uploads h with the materials, camera and environment (validated by the caller).
int32_t commit_scene(nrrs_ctx* c, SceneHost& h, const uint32_t* mat_type, const float* mat_params, uint32_t nm,
                     const float* camera, const float* env) {
  const uint64_t n_nodes = h.nodes.size() / 16;
  if (n_nodes > c->max_tris + 2 || h.n_nodes4 > c->max_tris + 2) return fail(c, NRRS_ENOMEM, "BVH larger than reserved");
  if (h.tri.size() + h.inst.size() + (h.inst_uid.size() + 3) / 4 * 4 > 12 * c->max_tris)
    return fail(c, NRRS_ENOMEM, "triangles and instances larger than the bound workspace");
  if (c->cfg.nee && h.light_w.size() > c->max_tris) return fail(c, NRRS_ENOMEM, "more lights than the workspace holds");
  std::vector<float> mats(8ull * nm);
  for (uint32_t m = 0; m < nm; ++m) {
    for (int k = 0; k < 4; ++k) mats[8ull * m + k] = mat_params[7ull * m + k];
    for (int k = 0; k < 3; ++k) mats[8ull * m + 4 + k] = mat_params[7ull * m + 4 + k];
    std::memcpy(&mats[8ull * m + 7], &mat_type[m], 4);
  }
  // next-event estimation: lights chosen with probability lum(L_e) x area (CDF in double, stored
  // in float, last entry 1), pdf per unit area lum(L_e) / sum
  std::vector<float> light_cdf(1, 0.0f);
  double total = 0.0;
  if (c->cfg.nee) {
    std::vector<double> cum;
    for (double w : h.light_w) cum.push_back(total += w);
    for (double v : cum) light_cdf.push_back((float)(v / total));
    if (!h.light_w.empty()) light_cdf.back() = 1.0f;
  }
  // camera basis in double, then handed to the kernels in float
  const double eye[3] = {camera[0], camera[1], camera[2]};
  double fwd[3] = {camera[3] - eye[0], camera[4] - eye[1], camera[5] - eye[2]};
  const double up[3] = {camera[6], camera[7], camera[8]};
  double l = std::sqrt(fwd[0] * fwd[0] + fwd[1] * fwd[1] + fwd[2] * fwd[2]);
  if (!(l > 0.0)) return fail(c, NRRS_EINVAL, "camera eye equals look-at point");
  for (double& x : fwd) x /= l;
  double r[3] = {fwd[1] * up[2] - fwd[2] * up[1], fwd[2] * up[0] - fwd[0] * up[2], fwd[0] * up[1] - fwd[1] * up[0]};
  l = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(l > 0.0)) return fail(c, NRRS_EINVAL, "camera up is parallel to the view direction");
  for (double& x : r) x /= l;
  const double u[3] = {r[1] * fwd[2] - r[2] * fwd[1], r[2] * fwd[0] - r[0] * fwd[2], r[0] * fwd[1] - r[1] * fwd[0]};
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  if (c->cfg.nee && !h.light_w.empty()) {
    HIPC(c, hipMemcpy(c->light_geo, h.light_geo.data(), 4 * h.light_geo.size(), hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->light_cdf, light_cdf.data(), 4 * light_cdf.size(), hipMemcpyHostToDevice));
  }
  // instance records and their uid index follow the triangles in the triangle region
  float4* inst_dev = c->tri + h.tri.size() / 4;
  uint32_t* uid_dev = reinterpret_cast<uint32_t*>(inst_dev + h.inst.size() / 4);
  HIPC(c, hipMemcpy(c->tri, h.tri.data(), sizeof(float) * h.tri.size(), hipMemcpyHostToDevice));
  if (h.n_inst) {
    HIPC(c, hipMemcpy(inst_dev, h.inst.data(), sizeof(float) * h.inst.size(), hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(uid_dev, h.inst_uid.data(), sizeof(uint32_t) * h.inst_uid.size(), hipMemcpyHostToDevice));
  }
  HIPC(c, hipMemcpy(c->node, h.nodes.data(), sizeof(float) * h.nodes.size(), hipMemcpyHostToDevice));
  if (h.n_nodes4)
    HIPC(c, hipMemcpy(c->node4, h.nodes4.data(), sizeof(float) * h.nodes4.size(), hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(c->mat, mats.data(), sizeof(float) * mats.size(), hipMemcpyHostToDevice));
  DevScene& d = c->sc;
  d.tri = c->tri;
  d.node = c->node;
  d.node4 = c->node4;
  d.nn4 = (uint32_t)h.n_nodes4;
  d.mat = c->mat;
  d.nt = (uint32_t)(h.tri.size() / 12);
  d.nn = (uint32_t)n_nodes;
  d.nm = nm;
  d.light_geo = c->light_geo;
  d.light_cdf = c->light_cdf;
  d.nl = c->cfg.nee ? (uint32_t)h.light_w.size() : 0u;
  d.light_scale = d.nl ? (float)(1.0 / total) : 0.0f;
  d.inst = h.n_inst ? inst_dev : nullptr;
  d.inst_uid = h.n_inst ? uid_dev : nullptr;
  d.n_inst = h.n_inst;
  d.root = h.root;
  d.nt_base = h.nt_base;
  d.amin_x = h.amin[0];
  d.amin_y = h.amin[1];
  d.amin_z = h.amin[2];
  const double ex = h.amax[0] - h.amin[0], ey = h.amax[1] - h.amin[1], ez = h.amax[2] - h.amin[2];
  d.extent = (float)std::fmax(ex, std::fmax(ey, ez));
  d.tmin = 0.0f;                                  // hits count for t > 0 ...
  d.offset = (float)(1e-5 * d.extent);             // ... because child origins leave the surface
  d.env_r = env[0];
  d.env_g = env[1];
  d.env_b = env[2];
  const double th = std::tan((double)camera[9] * M_PI / 360.0);
  const double aspect = (double)c->cfg.width / (double)c->cfg.height;
  d.eye_x = (float)eye[0]; d.eye_y = (float)eye[1]; d.eye_z = (float)eye[2];
  d.fwd_x = (float)fwd[0]; d.fwd_y = (float)fwd[1]; d.fwd_z = (float)fwd[2];
  d.rx = (float)(r[0] * th * aspect); d.ry = (float)(r[1] * th * aspect); d.rz = (float)(r[2] * th * aspect);
  d.ux = (float)(u[0] * th); d.uy = (float)(u[1] * th); d.uz = (float)(u[2] * th);
  c->drop_graphs();  // captured passes hold the old scene in their kernel arguments
  // the traversal variants of this kind of scene, and a tuning that fits them
  for (int v = 0; v < 5; ++v) c->ext_occ[v] = h.n_inst ? c->ext_occ_inst[v] : c->ext_occ_flat[v];
  c->bvh4_ok = h.bvh4_ok;
  if (!c->bvh4_ok) c->ext_occ[4] = 0;
  if (c->ext_occ[c->tune.extend_variant] == 0) c->tune.extend_variant = 3;
  c->tune.extend_blocks_per_cu = std::max(1u, std::min(c->tune.extend_blocks_per_cu, c->ext_occ[c->tune.extend_variant]));
  c->bvh_order.swap(h.uid_to_flat);
  c->orig_to_bvh.swap(h.flat_to_uid);
  c->scene = true;
  return NRRS_OK;
}

int32_t check_common(nrrs_ctx* c, const uint32_t* mat_type, const float* mat_params, uint32_t nm,
                     const float* camera, const float* env) {
  if (!mat_type || !mat_params || !camera || !env || nm == 0) return fail(c, NRRS_EINVAL, "null array or no material");
  if (nm > c->max_mats) return fail(c, NRRS_ENOMEM, "scene larger than the bound workspace");
  if (!finite_all(mat_params, 7ull * nm) || !finite_all(camera, 10) || !finite_all(env, 3))
    return fail(c, NRRS_EINVAL, "non-finite scene value");
  for (uint32_t m = 0; m < nm; ++m)
    if (mat_type[m] > NRRS_MAT_EMITTER) return fail(c, NRRS_EINVAL, "unknown material type");
  if (!(camera[9] > 0.0f && camera[9] < 180.0f)) return fail(c, NRRS_EINVAL, "camera fov out of range");
  return NRRS_OK;
}

// Appends the triangles of one tree to h.tri in the tree's order; the tag (a0.w) is the
// triangle's original index (stored_index false) or its own slot in h.tri (true).
void append_tris(SceneHost& h, const float* verts, const uint32_t* tris, const uint32_t* tri_mat, const BvhOut& b,
                 bool stored_index) {
  const uint32_t first = (uint32_t)(h.tri.size() / 12);
  const uint64_t nt = b.order.size();
  h.tri.resize(h.tri.size() + 12 * nt);
  for (uint64_t k = 0; k < nt; ++k) {
    const uint32_t t = b.order[k];
    const float* v0 = verts + 3ull * tris[3 * t];
    const float* v1 = verts + 3ull * tris[3 * t + 1];
    const float* v2 = verts + 3ull * tris[3 * t + 2];
    float* o = &h.tri[12 * (first + k)];
    for (int a = 0; a < 3; ++a) {
      o[a] = v0[a];
      o[4 + a] = v1[a] - v0[a];
      o[8 + a] = v2[a] - v0[a];
    }
    const uint32_t tag = stored_index ? first + (uint32_t)k : t;
    std::memcpy(&o[3], &tag, 4);
    std::memcpy(&o[7], &tri_mat[t], 4);
    o[11] = 0.0f;
  }
}

}  // namespace

int32_t nrrs_upload_scene(nrrs_ctx* c, const float* verts, uint64_t nv, const uint32_t* tris, uint64_t nt,
                          const uint32_t* tri_mat, const uint32_t* mat_type, const float* mat_params, uint32_t nm,
                          const float* camera, const float* env) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "bind a workspace first");
  if (!verts || !tris || !tri_mat || nt == 0 || nv == 0) return fail(c, NRRS_EINVAL, "null array or empty scene");
  if (int32_t e = check_common(c, mat_type, mat_params, nm, camera, env)) return e;
  if (nt > c->max_tris) return fail(c, NRRS_ENOMEM, "scene larger than the bound workspace");
  if (int32_t e = check_mesh(c, verts, nv, tris, nt, tri_mat, nm)) return e;
  BvhOut bvh;
  build_bvh(verts, tris, nt, bvh, true);
  if (int32_t e = check_tree(c, bvh)) return e;
  SceneHost h;
  append_tris(h, verts, tris, tri_mat, bvh, false);
  h.nodes = std::move(bvh.nodes);
  h.nodes4 = std::move(bvh.nodes4);
  h.n_nodes4 = bvh.n_nodes4;
  h.bvh4_ok = bvh.max_depth4 <= kMaxBvh4Depth;
  h.nt_base = (uint32_t)nt;
  h.flat_to_uid.assign(nt, 0);
  for (uint64_t k = 0; k < nt; ++k) h.flat_to_uid[bvh.order[k]] = (uint32_t)k;
  for (uint64_t t = 0; t < nt; ++t) {
    const float* v[3] = {verts + 3ull * tris[3 * t], verts + 3ull * tris[3 * t + 1], verts + 3ull * tris[3 * t + 2]};
    for (const float* p : v) grow_bounds(h, p);
    // lights listed in the scene's own triangle order, so that a uniform picks the same light
    // whatever the BVH order
    if (c->cfg.nee) add_light(h, v[0], v[1], v[2], tri_mat[t], mat_params);
  }
  h.uid_to_flat = std::move(bvh.order);
  return commit_scene(c, h, mat_type, mat_params, nm, camera, env);
}

int32_t nrrs_upload_scene_instanced(nrrs_ctx* c, const float* verts, uint64_t nv, const uint32_t* tris, uint64_t nt,
                                    const uint32_t* tri_mat, const uint32_t* mat_type, const float* mat_params,
                                    uint32_t nm, const float* camera, const float* env, const nrrs_instances* in) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "bind a workspace first");
  if (!in) return fail(c, NRRS_EINVAL, "no instance description");
  if (nt && (!verts || !tris || !tri_mat || nv == 0)) return fail(c, NRRS_EINVAL, "null array in the base mesh");
  if (int32_t e = check_common(c, mat_type, mat_params, nm, camera, env)) return e;
  const uint32_t nmesh = in->n_meshes, ninst = in->n_inst;
  if (nmesh == 0 || ninst == 0 || !in->mesh_verts || !in->mesh_tris || !in->mesh_tri_mat || !in->mesh_tri_begin ||
      !in->inst_mesh || !in->inst_xform || !in->inst_mat || in->mesh_nv == 0)
    return fail(c, NRRS_EINVAL, "null array or no mesh / instance");
  const uint64_t* beg = in->mesh_tri_begin;
  if (beg[0] != 0) return fail(c, NRRS_EINVAL, "mesh_tri_begin[0] must be 0");
  for (uint32_t m = 0; m < nmesh; ++m)
    if (beg[m + 1] <= beg[m]) return fail(c, NRRS_EINVAL, "every mesh needs at least one triangle");
  const uint64_t mesh_nt = beg[nmesh];
  if (ninst >= (1u << 26)) return fail(c, NRRS_EINVAL, "too many instances");
  const uint64_t n_rec = ninst + (nt ? 1 : 0);
  if (nt + mesh_nt + 3 * n_rec > c->max_tris) return fail(c, NRRS_ENOMEM, "scene larger than the bound workspace");
  if (nt)
    if (int32_t e = check_mesh(c, verts, nv, tris, nt, tri_mat, nm)) return e;
  if (int32_t e = check_mesh(c, in->mesh_verts, in->mesh_nv, in->mesh_tris, mesh_nt, in->mesh_tri_mat, nm)) return e;
  uint64_t flat = nt;
  for (uint32_t j = 0; j < ninst; ++j) {
    if (in->inst_mesh[j] >= nmesh) return fail(c, NRRS_EINVAL, "instance mesh out of range");
    if (in->inst_mat[j] != NRRS_NO_MATERIAL && in->inst_mat[j] >= nm)
      return fail(c, NRRS_EINVAL, "instance material out of range");
    if (!finite_all(in->inst_xform + 12ull * j, 12)) return fail(c, NRRS_EINVAL, "non-finite instance transform");
    flat += beg[in->inst_mesh[j] + 1] - beg[in->inst_mesh[j]];
  }
  if (flat >= (1ull << 31)) return fail(c, NRRS_EINVAL, "more than 2^31 triangles after instancing");
  SceneHost h;
  h.nt_base = (uint32_t)nt;
  // the base mesh and each mesh: trees of their own, triangles in tree order
  BvhOut base;
  int max_blas_depth = 0;
  if (nt) {
    build_bvh(verts, tris, nt, base, false);
    if (int32_t e = check_tree(c, base)) return e;
    append_tris(h, verts, tris, tri_mat, base, false);
    append_tree(h, base, 0, false);
    max_blas_depth = base.max_depth;
  }
  std::vector<BvhOut> mesh(nmesh);
  std::vector<uint32_t> mesh_first(nmesh), mesh_root(nmesh);
  for (uint32_t m = 0; m < nmesh; ++m) {
    build_bvh(in->mesh_verts, in->mesh_tris + 3 * beg[m], beg[m + 1] - beg[m], mesh[m], false);
    if (int32_t e = check_tree(c, mesh[m])) return e;
    mesh_first[m] = (uint32_t)(h.tri.size() / 12);
    mesh_root[m] = (uint32_t)(h.nodes.size() / 16);
    append_tris(h, in->mesh_verts, in->mesh_tris + 3 * beg[m], in->mesh_tri_mat + beg[m], mesh[m], true);
    append_tree(h, mesh[m], mesh_first[m], false);
    max_blas_depth = std::max(max_blas_depth, mesh[m].max_depth);
  }
  // records: the base mesh (identity) first, then the instances; world boxes for the top tree
  struct Rec {
    double fwd[12], inv[12];
    uint32_t root, uoff, mat, uid;
  };
  std::vector<Rec> recs;
  std::vector<float> boxes;
  auto root_box = [&](const BvhOut& b, double lo[3], double hi[3]) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::fmin(b.nodes[a], b.nodes[6 + a]);
      hi[a] = std::fmax(b.nodes[3 + a], b.nodes[9 + a]);
    }
  };
  auto push_box = [&](const double lo[3], const double hi[3]) {
    for (int a = 0; a < 3; ++a) boxes.push_back(std::nextafter((float)lo[a], -INFINITY));
    for (int a = 0; a < 3; ++a) boxes.push_back(std::nextafter((float)hi[a], INFINITY));
  };
  if (nt) {
    Rec r{};
    for (int k = 0; k < 3; ++k) r.fwd[5 * k] = r.inv[5 * k] = 1.0;  // identity, no translation
    r.root = 0;  // the base tree went in first
    r.uoff = 0;
    r.mat = NRRS_NO_MATERIAL;
    r.uid = 0;
    recs.push_back(r);
    double lo[3], hi[3];
    root_box(base, lo, hi);
    push_box(lo, hi);
  }
  uint32_t uid = (uint32_t)nt;
  for (uint32_t j = 0; j < ninst; ++j) {
    const float* x = in->inst_xform + 12ull * j;
    Rec r{};
    for (int k = 0; k < 12; ++k) r.fwd[k] = x[k];
    // inverse of the 3x3 part and of the translation, in double
    const double* M = r.fwd;
    const double a00 = M[0], a01 = M[1], a02 = M[2], a10 = M[4], a11 = M[5], a12 = M[6], a20 = M[8], a21 = M[9],
                 a22 = M[10];
    const double c00 = a11 * a22 - a12 * a21, c01 = a02 * a21 - a01 * a22, c02 = a01 * a12 - a02 * a11;
    const double c10 = a12 * a20 - a10 * a22, c11 = a00 * a22 - a02 * a20, c12 = a02 * a10 - a00 * a12;
    const double c20 = a10 * a21 - a11 * a20, c21 = a01 * a20 - a00 * a21, c22 = a00 * a11 - a01 * a10;
    const double det = a00 * c00 + a01 * c10 + a02 * c20;
    const double scale = std::fmax(std::fabs(a00) + std::fabs(a01) + std::fabs(a02),
                                   std::fmax(std::fabs(a10) + std::fabs(a11) + std::fabs(a12),
                                             std::fabs(a20) + std::fabs(a21) + std::fabs(a22)));
    if (!(std::fabs(det) > 1e-12 * scale * scale * scale)) return fail(c, NRRS_EINVAL, "singular instance transform");
    const double inv3[9] = {c00 / det, c01 / det, c02 / det, c10 / det, c11 / det, c12 / det,
                            c20 / det, c21 / det, c22 / det};
    // rows of A^-1, each with the translation's component in w: the kernels map a point as
    // A^-1 (p - t), subtracting first, so that the rounding scales with |p - t| rather than |p|
    for (int row = 0; row < 3; ++row) {
      for (int k = 0; k < 3; ++k) r.inv[4 * row + k] = inv3[3 * row + k];
      r.inv[4 * row + 3] = M[4 * row + 3];
    }
    const uint32_t m = in->inst_mesh[j];
    r.root = mesh_root[m];
    r.uoff = uid - mesh_first[m];  // (modulo 2^32)
    r.mat = in->inst_mat[j];
    r.uid = uid;
    recs.push_back(r);
    // world box: the eight corners of the mesh's root box moved by the transform
    double blo[3], bhi[3], lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    root_box(mesh[m], blo, bhi);
    for (int corner = 0; corner < 8; ++corner) {
      const double p[3] = {(corner & 1) ? bhi[0] : blo[0], (corner & 2) ? bhi[1] : blo[1], (corner & 4) ? bhi[2] : blo[2]};
      for (int a = 0; a < 3; ++a) {
        const double w = M[4 * a] * p[0] + M[4 * a + 1] * p[1] + M[4 * a + 2] * p[2] + M[4 * a + 3];
        lo[a] = std::fmin(lo[a], w);
        hi[a] = std::fmax(hi[a], w);
      }
    }
    // and a relative allowance for the float32 transform of rays into object space
    const double pad = 1e-6 * std::fmax(std::fmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    for (int a = 0; a < 3; ++a) {
      lo[a] -= pad;
      hi[a] += pad;
    }
    push_box(lo, hi);
    uid += (uint32_t)(beg[m + 1] - beg[m]);
  }
  BvhOut top;
  build_bvh_boxes(boxes.data(), recs.size(), top);
  if (top.max_depth + max_blas_depth + 2 > kMaxBvhDepth)
    return fail(c, NRRS_EINVAL, "instance tree and mesh trees together deeper than the traversal stack");
  h.root = (uint32_t)(h.nodes.size() / 16);
  append_tree(h, top, 0, true);
  // records in the top tree's order (a leaf lists consecutive records)
  h.n_inst = (uint32_t)recs.size();
  h.inst.resize(28ull * recs.size());
  std::vector<std::pair<uint32_t, uint32_t>> by_uid;
  for (uint32_t k = 0; k < recs.size(); ++k) {
    const Rec& r = recs[top.order[k]];
    float* f = &h.inst[28ull * k];
    for (int q = 0; q < 12; ++q) f[q] = (float)r.inv[q];
    for (int q = 0; q < 12; ++q) f[12 + q] = (float)r.fwd[q];
    std::memcpy(&f[24], &r.root, 4);
    std::memcpy(&f[25], &r.uoff, 4);
    std::memcpy(&f[26], &r.mat, 4);
    std::memcpy(&f[27], &r.uid, 4);
    by_uid.push_back({r.uid, k});
  }
  std::sort(by_uid.begin(), by_uid.end());
  for (const auto& p : by_uid) {
    h.inst_uid.push_back(p.first);
    h.inst_uid.push_back(p.second);
  }
  // flattened order: the base triangles, then each instance's mesh triangles in the mesh's own
  // order; world vertices are ((m0 x + m1 y) + m2 z) + t in double, rounded to float
  h.uid_to_flat.resize(flat);
  h.flat_to_uid.resize(flat);
  for (uint64_t k = 0; k < nt; ++k) {
    h.uid_to_flat[k] = base.order[k];
    h.flat_to_uid[base.order[k]] = (uint32_t)k;
  }
  for (uint64_t t = 0; t < nt; ++t) {
    const float* v[3] = {verts + 3ull * tris[3 * t], verts + 3ull * tris[3 * t + 1], verts + 3ull * tris[3 * t + 2]};
    for (const float* p : v) grow_bounds(h, p);
    if (c->cfg.nee) add_light(h, v[0], v[1], v[2], tri_mat[t], mat_params);
  }
  uid = (uint32_t)nt;
  for (uint32_t j = 0; j < ninst; ++j) {
    const uint32_t m = in->inst_mesh[j];
    const float* x = in->inst_xform + 12ull * j;
    const uint64_t n_m = beg[m + 1] - beg[m];
    for (uint64_t k = 0; k < n_m; ++k) {
      h.uid_to_flat[uid + k] = uid + mesh[m].order[k];
      h.flat_to_uid[uid + mesh[m].order[k]] = uid + (uint32_t)k;
    }
    for (uint64_t i = 0; i < n_m; ++i) {
      const uint32_t* tv = in->mesh_tris + 3 * (beg[m] + i);
      float w[3][3];
      for (int q = 0; q < 3; ++q) {
        const float* p = in->mesh_verts + 3ull * tv[q];
        for (int a = 0; a < 3; ++a) {
          const double s0 = (double)x[4 * a] * p[0];
          const double s1 = (double)x[4 * a + 1] * p[1];
          const double s2 = (double)x[4 * a + 2] * p[2];
          const double s01 = s0 + s1;
          const double s012 = s01 + s2;
          w[q][a] = (float)(s012 + (double)x[4 * a + 3]);
        }
        grow_bounds(h, w[q]);
      }
      const uint32_t mt = in->inst_mat[j] != NRRS_NO_MATERIAL ? in->inst_mat[j] : in->mesh_tri_mat[beg[m] + i];
      if (c->cfg.nee) add_light(h, w[0], w[1], w[2], mt, mat_params);
    }
    uid += (uint32_t)n_m;
  }
  h.bvh4_ok = false;
  return commit_scene(c, h, mat_type, mat_params, nm, camera, env);
}

int32_t nrrs_set_launch_mode(nrrs_ctx* c, int32_t mode) {
  if (!c || (mode != 0 && mode != 1)) return NRRS_EINVAL;
  c->launch_mode = mode;
  return NRRS_OK;
}

int32_t nrrs_set_timing(nrrs_ctx* c, int32_t enabled) {
  if (!c) return NRRS_EINVAL;
  c->timing = enabled != 0;
  return NRRS_OK;
}

int32_t nrrs_set_mix_depth(nrrs_ctx* c, uint64_t net_depths) {
  if (!c) return NRRS_EINVAL;
  if (net_depths != c->net_depths) c->drop_graphs();  // captured passes hold the old launch sequence
  c->net_depths = net_depths;
  return NRRS_OK;
}

int32_t nrrs_set_pass_index(nrrs_ctx* c, uint64_t next_pass) {
  if (!c) return NRRS_EINVAL;
  if (next_pass > 0xFFFFFFFFull) return fail(c, NRRS_EINVAL, "pass index beyond 32 bits");
  c->passes_done = next_pass;
  return NRRS_OK;
}

int32_t nrrs_get_pass_index(const nrrs_ctx* c, uint64_t* next_pass) {
  if (!c || !next_pass) return NRRS_EINVAL;
  *next_pass = c->passes_done;
  return NRRS_OK;
}

int32_t nrrs_set_mix_depth_fixed(nrrs_ctx* c, uint64_t fixed_depths) {
  if (!c) return NRRS_EINVAL;
  if (fixed_depths != c->fixed_depths) c->drop_graphs();  // captured passes hold the old launch sequence
  c->fixed_depths = fixed_depths;
  return NRRS_OK;
}

int32_t nrrs_get_mix_depth_fixed(const nrrs_ctx* c, uint64_t* fixed_depths) {
  if (!c || !fixed_depths) return NRRS_EINVAL;
  *fixed_depths = c->fixed_depths;
  return NRRS_OK;
}

int32_t nrrs_get_mix_depth(const nrrs_ctx* c, uint64_t* net_depths) {
  if (!c || !net_depths) return NRRS_EINVAL;
  *net_depths = c->net_depths;
  return NRRS_OK;
}

int32_t nrrs_get_tuning(const nrrs_ctx* c, nrrs_tuning* out) {
  if (!c || !out) return NRRS_EINVAL;
  *out = c->tune;
  for (int v = 0; v < 5; ++v) out->extend_max_blocks_per_cu[v] = c->ext_occ[v];
  return NRRS_OK;
}

int32_t nrrs_set_precision(nrrs_ctx* c, int32_t precision) {
  if (!c) return NRRS_EINVAL;
  if (precision < NRRS_PREC_FP32 || precision > NRRS_PREC_FP8) return fail(c, NRRS_EINVAL, "unknown precision");
  if (precision != c->cfg.precision) c->drop_graphs();  // captured passes hold the old network launch
  c->cfg.precision = precision;
  return NRRS_OK;
}

int32_t nrrs_set_tuning(nrrs_ctx* c, const nrrs_tuning* t) {
  if (!c || !t) return NRRS_EINVAL;
  if (t->extend_variant == 4 && c->scene && !c->bvh4_ok)
    return fail(c, NRRS_EINVAL, "the scene's 4-wide tree is deeper than the traversal stack allows");
  if (t->extend_variant > 4 || t->extend_blocks_per_cu < 1 ||
      t->extend_blocks_per_cu > c->ext_occ[t->extend_variant] || t->extend_refill < 1 || t->extend_refill > 64 ||
      t->extend_leaf_batch < 1 || t->extend_leaf_batch > 64 || t->extend_chunk > 4096)
    return fail(c, NRRS_EINVAL,
                "tuning out of range (blocks per CU up to the variant's occupancy, lanes 1..64, chunk <= 4096)");
  c->tune.extend_variant = t->extend_variant;
  c->tune.extend_blocks_per_cu = t->extend_blocks_per_cu;
  c->tune.extend_refill = t->extend_refill;
  c->tune.extend_leaf_batch = t->extend_leaf_batch;
  c->tune.extend_chunk = t->extend_chunk;
  c->drop_graphs();  // captured passes hold the old grid and thresholds
  return NRRS_OK;
}

int32_t nrrs_render(nrrs_ctx* c, uint32_t spp, uint32_t max_depth, int32_t mode, nrrs_render_stats* stats) {
  if (!c) return NRRS_EINVAL;
  if (!c->scene) return fail(c, NRRS_ESTATE, "upload a scene first");
  if (spp == 0 || spp % c->cfg.s_batch != 0) return fail(c, NRRS_EINVAL, "spp must be a positive multiple of s_batch");
  if (max_depth < 1 || max_depth > NRRS_MAX_DEPTH) return fail(c, NRRS_EINVAL, "max_depth out of range");
  if (mode < NRRS_MODE_OFF || mode > NRRS_MODE_AID) return fail(c, NRRS_EINVAL, "unknown mode");
  if ((mode == NRRS_MODE_NRRS || mode == NRRS_MODE_AID) && !c->cfg.hash_log2)
    return fail(c, NRRS_ESTATE, "NRRS mode needs a context created with hash_log2 > 0");
  if (c->trace_on && max_depth > c->cfg.trace_depth)
    return fail(c, NRRS_EINVAL, "max_depth beyond the traced depths");
  if (c->f_fixed_n && mode != NRRS_MODE_OFF && max_depth > c->f_fixed_n + 1)
    return fail(c, NRRS_EINVAL, "max_depth beyond the depths with a given normalization factor");
  hipStream_t s = c->stream;
  const uint32_t passes = spp / c->cfg.s_batch;
  RenderArgs a = base_args(c);
  a.max_depth = max_depth;
  a.mode = (uint32_t)mode;
  a.records_on = (mode != NRRS_MODE_OFF && c->cfg.records_cap > 0 && c->cfg.p_train > 0.0) ? 1u : 0u;
  const NetArgs net = net_args(c, c->cfg.precision);
  const NrrsNet nnet = c->cfg.hash_log2 ? nrrs_net_args(c, true) : NrrsNet{};
  // persistent grid of the NRRS factor kernel: 5 blocks of 4 waves per CU, the 5 waves per SIMD
  // its registers allow (at most 22.7 KB of weights in LDS per block)
  const uint32_t nrrs_blocks = c->cus * 5;
  if (a.records_on) launch_zero_u32(a.rec.count, 1, s);
  launch_zero_u32((uint32_t*)c->st_n, 2 * (NRRS_MAX_DEPTH + 1), s);
  launch_zero_u32((uint32_t*)c->st_s, 2 * (NRRS_MAX_DEPTH + 1), s);
  launch_zero_u32((uint32_t*)c->st_r, 2 * (NRRS_MAX_DEPTH + 1), s);
  launch_zero_u32((uint32_t*)c->rays, 12, s);
  launch_zero_u32(c->overflow, 1, s);
  // stage timing: one event before the first launch and one after every stage
  size_t n_ev = 0;
  auto mark = [&](int stage) -> int32_t {
    if (!c->timing) return NRRS_OK;
    if (n_ev == c->events.size()) {
      hipEvent_t e;
      HIPC(c, hipEventCreate(&e));
      c->events.push_back(e);
      c->event_stage.push_back(stage);
    }
    c->event_stage[n_ev] = stage;
    HIPC(c, hipEventRecord(c->events[n_ev], s));
    ++n_ev;
    return NRRS_OK;
  };
  // One whole pass: advance the device pass state, camera, the bounce loop, statistics and
  // the guide refresh.  Its launches depend on nothing that changes between passes.
  auto enqueue_pass = [&](bool timed) -> int32_t {
#define MARK(stage)                             \
  do {                                          \
    if (timed) {                                \
      int32_t r_ = mark(stage);                 \
      if (r_ != NRRS_OK) return r_;             \
    }                                           \
  } while (0)
    RenderArgs b = a;
    launch_begin_pass(b, (double)c->cfg.s_batch, s);
    launch_camera(b, s);
    MARK(0);
    for (uint32_t d = 1; d <= max_depth; ++d) {
      b.depth = d;
      launch_extend(b, s);
      MARK(1);
      launch_shade(b, s);
      if (b.records_on && d <= (uint32_t)c->cfg.net_max_depth) launch_record_features(b, c->cfg.records_cap, s);
      if (c->cfg.nee && d < max_depth) launch_nee(b, s);
      MARK(2);
      if (d == max_depth) break;
      if (mode != NRRS_MODE_OFF && ((c->fixed_depths >> (d - 1)) & 1u)) {
        launch_fixed_factor(b, s);
        MARK(3);
      } else if (mode == NRRS_MODE_NET && ((c->net_depths >> (d - 1)) & 1u)) {
        launch_rrsnet(b, net, s);
        MARK(3);
      } else if ((mode == NRRS_MODE_NRRS || mode == NRRS_MODE_AID) && ((c->net_depths >> (d - 1)) & 1u)) {
        launch_nrrs_factor(b, nnet, nrrs_blocks, mode == NRRS_MODE_AID, s);
        MARK(3);
      }
      launch_sum_q(b, s);
      MARK(4);
      launch_roulette(b, s);
      if (b.records_on && b.rec.nqf && d <= (uint32_t)c->cfg.net_max_depth) launch_record_qnorm(b, s);
      MARK(5);
      launch_expand(b, s);
      MARK(6);
      std::swap(b.qin, b.qout);
    }
    launch_accumulate_stats(c->ctl, max_depth, c->st_n, c->st_s, c->st_r, c->st_sumq, c->st_f, s);
    launch_guide(b, c->guide, s);
    MARK(7);
#undef MARK
    return NRRS_OK;
  };
  // the device pass state continues from the host's counters
  launch_set_pass_state(c->pass_state, (uint32_t)(c->passes_done - 1), (double)c->spp_total, s);
  if (c->timing) {
    int32_t r0 = mark(-1);
    if (r0 != NRRS_OK) return r0;
  }
  // the null stream cannot be captured: direct launches there
  const bool use_graph = c->launch_mode == 1 && !c->timing && s != nullptr;
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    const auto key = std::make_tuple(max_depth, mode, a.records_on);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
      exec = it->second;
    } else {
      hipGraph_t graph = nullptr;
      HIPC(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const int32_t rq = enqueue_pass(false);
      hipError_t ec = hipStreamEndCapture(s, &graph);  // always ends the capture
      if (rq != NRRS_OK) {
        if (graph) hipGraphDestroy(graph);
        return rq;
      }
      if (ec != hipSuccess) return fail(c, NRRS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
      ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (ec != hipSuccess) return fail(c, NRRS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ec));
      c->graphs[key] = exec;
    }
  }
  for (uint32_t p = 0; p < passes; ++p) {
    if (use_graph) {
      HIPC(c, hipGraphLaunch(exec, s));
    } else {
      const int32_t rp = enqueue_pass(c->timing);
      if (rp != NRRS_OK) return rp;
    }
    c->spp_total += c->cfg.s_batch;
  }
  c->passes_done += passes;
  HIPC(c, hipGetLastError());
  if (stats) {
    HIPC(c, hipStreamSynchronize(s));
    std::memset(stats, 0, sizeof(*stats));
    stats->max_depth = max_depth;
    stats->passes = passes;
    HIPC(c, hipMemcpy(stats->n, c->st_n, sizeof(uint64_t) * (NRRS_MAX_DEPTH + 1), hipMemcpyDeviceToHost));
    HIPC(c, hipMemcpy(stats->S, c->st_s, sizeof(uint64_t) * (NRRS_MAX_DEPTH + 1), hipMemcpyDeviceToHost));
    HIPC(c, hipMemcpy(stats->retries, c->st_r, sizeof(uint64_t) * (NRRS_MAX_DEPTH + 1), hipMemcpyDeviceToHost));
    HIPC(c, hipMemcpy(stats->sumq, c->st_sumq, sizeof(double) * (NRRS_MAX_DEPTH + 1), hipMemcpyDeviceToHost));
    HIPC(c, hipMemcpy(stats->F, c->st_f, sizeof(double) * (NRRS_MAX_DEPTH + 1), hipMemcpyDeviceToHost));
    HIPC(c, hipMemcpy(&stats->alpha, c->alpha, sizeof(double), hipMemcpyDeviceToHost));
    unsigned long long work[3] = {0, 0, 0};
    HIPC(c, hipMemcpy(work, c->rays, sizeof(work), hipMemcpyDeviceToHost));
    stats->rays = work[0];
    stats->nodes_visited = work[1];
    stats->tris_tested = work[2];
    if (c->timing && n_ev > 1) {
      stats->timed = 1;
      for (size_t k = 1; k < n_ev; ++k) {
        float ms = 0.0f;
        HIPC(c, hipEventElapsedTime(&ms, c->events[k - 1], c->events[k]));
        const int st = c->event_stage[k];
        stats->stage_ms[st] += ms;
        stats->stage_launches[st] += 1;
      }
    }
    uint32_t cnt = 0, of = 0;
    HIPC(c, hipMemcpy(&cnt, c->rec.count, 4, hipMemcpyDeviceToHost));
    HIPC(c, hipMemcpy(&of, c->overflow, 4, hipMemcpyDeviceToHost));
    stats->records = a.records_on ? std::min<uint64_t>(cnt, c->cfg.records_cap) : 0;
    stats->overflow = of;
    if (of) return fail(c, NRRS_EOVERFLOW, "overflow guard found no alpha that fits the queue");
  }
  return NRRS_OK;
}

int32_t nrrs_read_image(nrrs_ctx* c, double* host_rgb, uint64_t* spp_total) {
  if (!c || !host_rgb) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  HIPC(c, hipStreamSynchronize(c->stream));
  HIPC(c, hipMemcpy(host_rgb, c->image, sizeof(double) * 3 * c->npx, hipMemcpyDeviceToHost));
  if (c->spp_total > 0)
    for (uint64_t i = 0; i < 3 * c->npx; ++i) host_rgb[i] /= (double)c->spp_total;
  if (spp_total) *spp_total = c->spp_total;
  return NRRS_OK;
}

int32_t nrrs_reset_image(nrrs_ctx* c) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  launch_zero_f64(c->image, 3 * c->npx, c->stream);
  launch_set_f64(c->alpha, 1.0, c->stream);
  c->spp_total = 0;
  if (c->cfg.hash_log2) {
    launch_zero_f64(c->lum_start, c->npx, c->stream);
    c->nrrs_frames = 0;
    c->nrrs_spp_start = 0;
  }
  HIPC(c, hipGetLastError());
  return NRRS_OK;
}

int32_t nrrs_autotune(nrrs_ctx* c, uint32_t max_depth, nrrs_tuning* best, nrrs_tuning* tried, uint32_t tried_cap,
                      uint32_t* n_tried) {
  if (!c) return NRRS_EINVAL;
  if (!c->scene) return fail(c, NRRS_ESTATE, "upload a scene first");
  if (max_depth < 1 || max_depth > NRRS_MAX_DEPTH) return fail(c, NRRS_EINVAL, "max_depth out of range");
  const bool timing = c->timing;
  const double p_train = c->cfg.p_train;
  c->timing = true;
  c->cfg.p_train = 0.0;  // the timing passes capture no training records
  // one candidate: the faster of two single-pass renders, by the traversal stage's event time
  auto measure = [&](const nrrs_tuning& t, float* ms) -> int32_t {
    int32_t r = nrrs_set_tuning(c, &t);
    if (r != NRRS_OK) return r;
    float m = INFINITY;
    for (int rep = 0; rep < 2; ++rep) {
      nrrs_render_stats st;
      r = nrrs_render(c, c->cfg.s_batch, max_depth, NRRS_MODE_HEURISTIC, &st);
      if (r != NRRS_OK) return r;
      m = std::fmin(m, (float)st.stage_ms[1]);
    }
    *ms = m;
    return NRRS_OK;
  };
  nrrs_tuning cur = c->tune, win = c->tune;
  float win_ms = INFINITY;
  int32_t r = NRRS_OK;
  uint32_t count = 0;
  auto consider = [&](const nrrs_tuning& t) {
    float ms = 0.0f;
    if (r != NRRS_OK) return;
    r = measure(t, &ms);
    if (r != NRRS_OK) return;
    if (tried && count < tried_cap) {
      tried[count] = t;
      for (int v = 0; v < 5; ++v) tried[count].extend_max_blocks_per_cu[v] = c->ext_occ[v];
      tried[count].extend_ms = ms;
    }
    ++count;
    if (ms < win_ms) {
      win_ms = ms;
      win = t;
    }
  };
  // 1: variant x refill threshold at full occupancy (claim chunk 64, leaf batch 16); 2: fewer
  // resident blocks per CU; 3: claim chunk; 4: leaf batch (variants that park leaves)
  for (uint32_t v = 0; v < 5; ++v) {
    if (c->ext_occ[v] == 0) continue;  // not available for this scene
    for (uint32_t refill : {8u, 16u, 32u, 48u}) {
      nrrs_tuning t = cur;
      t.extend_variant = v;
      t.extend_blocks_per_cu = c->ext_occ[v];
      t.extend_refill = refill;
      t.extend_leaf_batch = 16;
      t.extend_chunk = 64;
      consider(t);
    }
  }
  {
    const uint32_t occ = c->ext_occ[win.extend_variant];
    const uint32_t b1 = std::max(1u, (3 * occ) / 4), b2 = std::max(1u, occ / 2);
    const nrrs_tuning base = win;
    for (uint32_t bpc : {b1, b2}) {
      if (bpc == occ) continue;
      nrrs_tuning t = base;
      t.extend_blocks_per_cu = bpc;
      consider(t);
      if (b2 == b1) break;
    }
  }
  {
    const nrrs_tuning base = win;
    for (uint32_t ch : {0u, 32u, 128u}) {
      nrrs_tuning t = base;
      t.extend_chunk = ch;
      consider(t);
    }
  }
  if (win.extend_variant != 0) {
    const nrrs_tuning base = win;
    for (uint32_t lb : {8u, 12u, 16u, 24u, 32u}) {
      if (lb == base.extend_leaf_batch) continue;
      nrrs_tuning t = base;
      t.extend_leaf_batch = lb;
      consider(t);
    }
  }
  c->timing = timing;
  c->cfg.p_train = p_train;
  if (r != NRRS_OK) {
    nrrs_set_tuning(c, &cur);
    return r;
  }
  r = nrrs_set_tuning(c, &win);
  if (r != NRRS_OK) return r;
  r = nrrs_reset_image(c);
  if (r != NRRS_OK) return r;
  if (best) {
    nrrs_get_tuning(c, best);
    best->extend_ms = win_ms;
  }
  if (n_tried) *n_tried = count;
  return NRRS_OK;
}

int32_t nrrs_set_guide(nrrs_ctx* c, const float* host_lum) {
  if (!c || !host_lum) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  HIPC(c, hipStreamSynchronize(c->stream));
  HIPC(c, hipMemcpy(c->guide, host_lum, sizeof(float) * c->npx, hipMemcpyHostToDevice));
  return NRRS_OK;
}

int32_t nrrs_get_guide(nrrs_ctx* c, float* host_lum) {
  if (!c || !host_lum) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  HIPC(c, hipStreamSynchronize(c->stream));
  HIPC(c, hipMemcpy(host_lum, c->guide, sizeof(float) * c->npx, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_get_params(nrrs_ctx* c, float* master, float* adam_m, float* adam_v, uint64_t* step) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  HIPC(c, hipStreamSynchronize(c->stream));
  if (master) HIPC(c, hipMemcpy(master, c->master, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
  if (adam_m) HIPC(c, hipMemcpy(adam_m, c->adam_m, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
  if (adam_v) HIPC(c, hipMemcpy(adam_v, c->adam_v, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
  if (step) *step = c->adam_step;
  return NRRS_OK;
}

int32_t nrrs_set_params(nrrs_ctx* c, const float* master, const float* adam_m, const float* adam_v,
                        const uint64_t* step) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  HIPC(c, hipStreamSynchronize(c->stream));
  if (master) {
    HIPC(c, hipMemcpy(c->master, master, sizeof(float) * kNParam, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->infer, master, sizeof(float) * kNParam, hipMemcpyHostToDevice));
  }
  if (adam_m) HIPC(c, hipMemcpy(c->adam_m, adam_m, sizeof(float) * kNParam, hipMemcpyHostToDevice));
  if (adam_v) HIPC(c, hipMemcpy(c->adam_v, adam_v, sizeof(float) * kNParam, hipMemcpyHostToDevice));
  if (step) c->adam_step = *step;
  launch_quantize(c->infer, c->bf16, c->fp8, c->fp8_scale, c->stream);
  HIPC(c, hipGetLastError());
  return NRRS_OK;
}

int32_t nrrs_get_state(nrrs_ctx* c, float* infer, double* alpha) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  HIPC(c, hipStreamSynchronize(c->stream));
  if (infer) HIPC(c, hipMemcpy(infer, c->infer, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
  if (alpha) HIPC(c, hipMemcpy(alpha, c->alpha, sizeof(double), hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_set_state(nrrs_ctx* c, const float* infer, const double* alpha) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (infer && !finite_all(infer, kNParam)) return fail(c, NRRS_EINVAL, "non-finite inference weight");
  if (alpha && !(*alpha > 0.0 && *alpha <= 1.0)) return fail(c, NRRS_EINVAL, "alpha outside (0, 1]");
  HIPC(c, hipStreamSynchronize(c->stream));
  if (infer) {
    HIPC(c, hipMemcpy(c->infer, infer, sizeof(float) * kNParam, hipMemcpyHostToDevice));
    launch_quantize(c->infer, c->bf16, c->fp8, c->fp8_scale, c->stream);
  }
  if (alpha) HIPC(c, hipMemcpy(c->alpha, alpha, sizeof(double), hipMemcpyHostToDevice));
  HIPC(c, hipGetLastError());
  return NRRS_OK;
}

int32_t nrrs_set_trace(nrrs_ctx* c, int32_t enabled) {
  if (!c || (enabled != 0 && enabled != 1)) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (enabled && !c->trace) return fail(c, NRRS_ESTATE, "create the context with trace_depth > 0");
  if ((enabled != 0) != c->trace_on) c->drop_graphs();  // captured passes hold the old arguments
  c->trace_on = enabled != 0;
  if (c->trace_on) launch_zero_f64(c->trace, 3ull * c->cfg.trace_depth * c->nprim, c->stream);
  HIPC(c, hipGetLastError());
  return NRRS_OK;
}

int32_t nrrs_read_trace(nrrs_ctx* c, double* host_rgb) {
  if (!c || !host_rgb) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->trace) return fail(c, NRRS_ESTATE, "create the context with trace_depth > 0");
  HIPC(c, hipStreamSynchronize(c->stream));
  HIPC(c, hipMemcpy(host_rgb, c->trace, sizeof(double) * 3 * c->cfg.trace_depth * c->nprim,
                    hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_read_records(nrrs_ctx* c, uint64_t* n, float* features, float* lum_t, float* acc, uint32_t* depth,
                          uint32_t* pix, uint64_t* lineage) {
  if (!c || !n) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  HIPC(c, hipStreamSynchronize(c->stream));
  uint32_t cnt = 0;
  HIPC(c, hipMemcpy(&cnt, c->rec.count, 4, hipMemcpyDeviceToHost));
  const uint64_t k = std::min<uint64_t>(cnt, c->cfg.records_cap);
  *n = k;
  if (k == 0) return NRRS_OK;
  if (features) HIPC(c, hipMemcpy(features, c->rec.feat, sizeof(float) * 20 * k, hipMemcpyDeviceToHost));
  if (lum_t) HIPC(c, hipMemcpy(lum_t, c->rec.lum_t, sizeof(float) * k, hipMemcpyDeviceToHost));
  if (acc) HIPC(c, hipMemcpy(acc, c->rec.acc, sizeof(float) * k, hipMemcpyDeviceToHost));
  if (depth) HIPC(c, hipMemcpy(depth, c->rec.depth, sizeof(uint32_t) * k, hipMemcpyDeviceToHost));
  if (pix) HIPC(c, hipMemcpy(pix, c->rec.pix, sizeof(uint32_t) * k, hipMemcpyDeviceToHost));
  if (lineage) HIPC(c, hipMemcpy(lineage, c->rec.lineage, sizeof(uint64_t) * k, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_train_step(nrrs_ctx* c, uint32_t n_records, uint32_t minibatch, float lr, float* loss_or_null) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (n_records == 0 || minibatch == 0 || minibatch > kMaxMinibatch || n_records % minibatch != 0 ||
      !(lr > 0.0f) || !std::isfinite(lr))
    return fail(c, NRRS_EINVAL, "n_records must be a positive multiple of minibatch (<= 65536), lr > 0");
  if (n_records > c->cfg.records_cap) return fail(c, NRRS_ESTATE, "more records requested than the buffer holds");
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  uint32_t cnt = 0;
  HIPC(c, hipMemcpy(&cnt, c->rec.count, 4, hipMemcpyDeviceToHost));
  if (std::min<uint32_t>(cnt, c->cfg.records_cap) < n_records)
    return fail(c, NRRS_ESTATE, "fewer records captured than requested");
  launch_record_targets(c->rec, c->target, n_records, s);
  launch_zero_u32((uint32_t*)c->loss_accum, 1, s);
  const uint32_t batches = n_records / minibatch;
  for (uint32_t b = 0; b < batches; ++b) {
    uint32_t nb = 0;
    launch_mlp_grad(c->rec.feat + 20ull * b * minibatch, c->target + (uint64_t)b * minibatch, nullptr, minibatch,
                    c->master, c->cfg.loss, c->grad_partial, c->loss_partial, &nb, s);
    c->adam_step += 1;
    launch_grad_adam_ema(c->grad_partial, nb, c->grad, c->loss_partial, c->loss_accum, minibatch, c->master,
                         c->adam_m, c->adam_v, c->adam_step, lr, c->infer, (float)c->cfg.ema_decay, s);
  }
  launch_quantize(c->infer, c->bf16, c->fp8, c->fp8_scale, s);
  HIPC(c, hipGetLastError());
  if (loss_or_null) {
    HIPC(c, hipStreamSynchronize(s));
    float l = 0.0f;
    HIPC(c, hipMemcpy(&l, c->loss_accum, 4, hipMemcpyDeviceToHost));
    *loss_or_null = l / (float)batches;
  }
  return NRRS_OK;
}

// ------------------------------------------------------------------------- NRRS proper
int32_t nrrs_set_nrrs_params(nrrs_ctx* c, const float* stat, const float* rrs, const float* table) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  if ((stat && !finite_all(stat, kStatParams)) || (rrs && !finite_all(rrs, kRrsParams)) ||
      (table && !finite_all(table, c->ntab_n)))
    return fail(c, NRRS_EINVAL, "non-finite NRRS parameter");
  HIPC(c, hipStreamSynchronize(c->stream));
  return upload_nrrs_state(c, stat, rrs, table);
}

int32_t nrrs_get_nrrs_params(nrrs_ctx* c, float* stat, float* rrs, float* table) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  HIPC(c, hipStreamSynchronize(c->stream));
  if (stat) HIPC(c, hipMemcpy(stat, c->nstat.w, sizeof(float) * kStatParams, hipMemcpyDeviceToHost));
  if (rrs) HIPC(c, hipMemcpy(rrs, c->nrrs_net.w, sizeof(float) * kRrsParams, hipMemcpyDeviceToHost));
  if (table) HIPC(c, hipMemcpy(table, c->ntab.w, sizeof(float) * c->ntab_n, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_set_aid_params(nrrs_ctx* c, const float* aid, const float* table_r) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  if ((aid && !finite_all(aid, kAidParams)) || (table_r && !finite_all(table_r, c->ntab_n)))
    return fail(c, NRRS_EINVAL, "non-finite AID-NRRS parameter");
  HIPC(c, hipStreamSynchronize(c->stream));
  return upload_nrrs_state(c, nullptr, nullptr, nullptr, aid, table_r);
}

int32_t nrrs_get_aid_params(nrrs_ctx* c, float* aid, float* table_r) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  HIPC(c, hipStreamSynchronize(c->stream));
  if (aid) HIPC(c, hipMemcpy(aid, c->naid.w, sizeof(float) * kAidParams, hipMemcpyDeviceToHost));
  if (table_r) HIPC(c, hipMemcpy(table_r, c->ntab_r.w, sizeof(float) * c->ntab_n, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

namespace {
bool train_args_ok(const nrrs_nrrs_train* hp) {
  auto pos = [](float x) { return x > 0.0f && std::isfinite(x); };
  auto nonneg = [](float x) { return x >= 0.0f && std::isfinite(x); };
  return hp && pos(hp->lr_stat) && pos(hp->lr_rrs) && nonneg(hp->g_avg) && nonneg(hp->g_min) &&
         nonneg(hp->g_rrs) && hp->a_mix > 0.0f && hp->a_mix <= 1.0f && hp->radius >= 0 && hp->radius <= 8 &&
         (hp->rrs_step == 1 || hp->rrs_step == 2) && hp->variant >= 0 && hp->variant <= 2;
}
}  // namespace

int32_t nrrs_train_step_nrrs(nrrs_ctx* c, uint32_t n_records, const nrrs_nrrs_train* hp, nrrs_nrrs_loss* out) {
  if (!c) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  if (!train_args_ok(hp)) return fail(c, NRRS_EINVAL, "NRRS training parameters out of range");
  if (n_records == 0 || n_records > c->cfg.records_cap) return fail(c, NRRS_EINVAL, "n_records out of range");
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  uint32_t cnt = 0;
  HIPC(c, hipMemcpy(&cnt, c->rec.count, 4, hipMemcpyDeviceToHost));
  if (std::min<uint32_t>(cnt, c->cfg.records_cap) < n_records)
    return fail(c, NRRS_ESTATE, "fewer records captured than requested");
  if (c->spp_total <= c->nrrs_spp_start) return fail(c, NRRS_ESTATE, "no frame rendered since the last step");
  const NrrsRows r{c->rec.nraw, c->rec.lum_t, c->rec.acc, nullptr, c->rec.ntq, c->rec.nqf, c->rec.pix, n_records};
  const uint32_t nb = nrrs_grad_blocks(n_records);
  const float decay = (float)c->cfg.ema_decay, eps = 0.01f;
  // StatNet (hash grid and MLP), Eq. (15)
  launch_statnet_grad(r, c->nstat.w, c->ntab.w, c->cfg.hash_log2, eps, c->npartial, c->nloss_part, c->ntab.g, s);
  launch_partial_sum(c->npartial, nb, kStatParams, c->nstat.g, c->nloss_part, c->nloss, c->ngroups, s);
  c->nrrs_step += 1;
  launch_adam(c->nstat.w, c->nstat.m, c->nstat.v, c->nstat.g, kStatParams, c->nrrs_step, hp->lr_stat, c->nstat.infer,
              decay, false, s);
  launch_adam(c->ntab.w, c->ntab.m, c->ntab.v, c->ntab.g, c->ntab_n, c->nrrs_step, hp->lr_stat, c->ntab.infer, decay,
              true, s);
  // the frame's pixel error (kept up to date in both steps so that step 2 starts mixed)
  const double spp_frame = (double)(c->spp_total - c->nrrs_spp_start);
  const bool first = c->nrrs_frames == 0;
  const bool has_ref = c->nrrs_spp_start > 0;
  launch_frame_lum(c->image, c->lum_start, (uint32_t)c->npx, spp_frame, (double)c->nrrs_spp_start, c->pcur, c->pref,
                   s);
  PixelErrArgs pe{};
  pe.cur = c->pcur;
  pe.ref = c->pref;
  pe.acc = c->pacc;
  pe.Ep = c->pEp;
  pe.E = c->pE;
  pe.wpx = c->pwpx;
  pe.part = c->pix_part;
  pe.eavg = c->eavg;
  pe.w = c->cfg.width;
  pe.h = c->cfg.height;
  pe.first = first ? 1u : 0u;
  pe.radius = hp->radius;
  pe.a_mix = hp->a_mix;
  // variance of a one-sample pixel estimate from the squared error of the mixed frame estimate
  pe.var_scale = (float)(spp_frame * (first ? 1.0 : (2.0 - hp->a_mix) / hp->a_mix));
  pe.g_avg = hp->g_avg;
  pe.g_min = hp->g_min;
  pe.eps = eps;
  launch_pixel_error(pe, s);
  launch_count_pix(c->rec.pix, n_records, c->kpix, (uint32_t)c->npx, s);
  c->nrrs_frames += 1;
  c->nrrs_spp_start = c->spp_total;
  // RRSNet with StatNet's updated weights
  const bool rrs_train = hp->rrs_step == 1 || has_ref;
  if (rrs_train && (hp->variant == 0 || hp->variant == 2)) {
    launch_rrsnet_grad(r, c->nstat.w, c->ntab.w, c->cfg.hash_log2, c->nrrs_net.w, hp->rrs_step, c->pwpx, c->kpix,
                       hp->g_rrs, eps, c->npartial, c->nloss_part, s);
    launch_partial_sum(c->npartial, nb, kRrsParams, c->nrrs_net.g, c->nloss_part, c->nloss + 1, c->ngroups, s);
    c->nrrs_rstep += 1;
    launch_adam(c->nrrs_net.w, c->nrrs_net.m, c->nrrs_net.v, c->nrrs_net.g, kRrsParams, c->nrrs_rstep, hp->lr_rrs,
                c->nrrs_net.infer, decay, false, s);
  }
  if (rrs_train && (hp->variant == 1 || hp->variant == 2)) {
    // AID-NRRS: RRSNet's MLP and its own hash grid (StatNet's statistics supervise)
    launch_aid_grad(r, c->nstat.w, c->ntab.w, c->cfg.hash_log2, c->naid.w, c->ntab_r.w, hp->rrs_step, c->pwpx,
                    c->kpix, hp->g_rrs, eps, c->npartial, c->nloss_part, c->ntab_r.g, s);
    launch_partial_sum(c->npartial, nb, kAidParams, c->naid.g, c->nloss_part, c->nloss + 1, c->ngroups, s);
    c->nrrs_astep += 1;
    launch_adam(c->naid.w, c->naid.m, c->naid.v, c->naid.g, kAidParams, c->nrrs_astep, hp->lr_rrs, c->naid.infer,
                decay, false, s);
    launch_adam(c->ntab_r.w, c->ntab_r.m, c->ntab_r.v, c->ntab_r.g, c->ntab_n, c->nrrs_astep, hp->lr_rrs,
                c->ntab_r.infer, decay, true, s);
  }
  HIPC(c, hipGetLastError());
  if (out) {
    HIPC(c, hipStreamSynchronize(s));
    float l[2] = {0.0f, 0.0f};
    HIPC(c, hipMemcpy(l, c->nloss, sizeof(l), hipMemcpyDeviceToHost));
    HIPC(c, hipMemcpy(&out->e_avg, c->eavg, sizeof(double), hipMemcpyDeviceToHost));
    out->loss_stat = l[0];
    out->loss_rrs = rrs_train ? l[1] : 0.0f;
    out->records = n_records;
    out->rrs_trained = rrs_train ? 1u : 0u;
  }
  return NRRS_OK;
}

int32_t nrrs_debug_nrrs_forward(nrrs_ctx* c, const float* raw, const float* t, const float* I, uint32_t n, float* mv,
                                float* q, float* enc) {
  if (!c || (n && (!raw || !t || !I || !mv || !q))) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  if ((uint64_t)n * 4 * 46 + 4096 > c->qb_pool_bytes) return fail(c, NRRS_ENOMEM, "too many rows for the scratch space");
  if (n == 0) return NRRS_OK;
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  Carve k{c->qb_pool};
  float* praw = k.take<float>(7ull * n);
  float* pt = k.take<float>(3ull * n);
  float* pI = k.take<float>(n);
  float* pmv = k.take<float>(2ull * n);
  float* pq = k.take<float>(n);
  float* penc = enc ? k.take<float>(32ull * n) : nullptr;
  HIPC(c, hipMemcpy(praw, raw, sizeof(float) * 7 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pt, t, sizeof(float) * 3 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pI, I, sizeof(float) * n, hipMemcpyHostToDevice));
  launch_nrrs_rows(praw, pt, pI, n, nrrs_net_args(c, true), pmv, pq, penc, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpy(mv, pmv, sizeof(float) * 2 * n, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(q, pq, sizeof(float) * n, hipMemcpyDeviceToHost));
  if (enc) HIPC(c, hipMemcpy(enc, penc, sizeof(float) * 32 * n, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_debug_aid_forward(nrrs_ctx* c, const float* raw, const float* t, const float* I, uint32_t n, float* q,
                               float* enc) {
  if (!c || (n && (!raw || !t || !I || !q))) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  if ((uint64_t)n * 4 * 44 + 4096 > c->qb_pool_bytes) return fail(c, NRRS_ENOMEM, "too many rows for the scratch space");
  if (n == 0) return NRRS_OK;
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  Carve k{c->qb_pool};
  float* praw = k.take<float>(7ull * n);
  float* pt = k.take<float>(3ull * n);
  float* pI = k.take<float>(n);
  float* pq = k.take<float>(n);
  float* penc = enc ? k.take<float>(32ull * n) : nullptr;
  HIPC(c, hipMemcpy(praw, raw, sizeof(float) * 7 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pt, t, sizeof(float) * 3 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pI, I, sizeof(float) * n, hipMemcpyHostToDevice));
  launch_aid_rows(praw, pt, pI, n, nrrs_net_args(c, true), pq, penc, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpy(q, pq, sizeof(float) * n, hipMemcpyDeviceToHost));
  if (enc) HIPC(c, hipMemcpy(enc, penc, sizeof(float) * 32 * n, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_debug_nrrs_grads(nrrs_ctx* c, const float* raw, const float* I, const float* L, const float* lum_t,
                              const float* t, const float* q_norm, const float* F, const uint32_t* pix, uint32_t n,
                              const float* wpx, const uint32_t* kk, uint32_t npx, int32_t rrs_step, float g_rrs,
                              float* g_stat, float* g_rrs_out, float* g_table, float* loss_stat, float* loss_rrs) {
  if (!c || n == 0 || !raw || !I || !L || !lum_t || !t || !q_norm || !F || !pix || npx == 0 || !wpx || !kk ||
      !g_stat || !g_rrs_out || !g_table || !loss_stat || !loss_rrs || (rrs_step != 1 && rrs_step != 2) ||
      !(g_rrs >= 0.0f))
    return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  if (n > c->cfg.records_cap) return fail(c, NRRS_EINVAL, "n beyond records_cap");
  for (uint32_t i = 0; i < n; ++i)
    if (pix[i] >= npx) return fail(c, NRRS_EINVAL, "pixel index beyond npx");
  if ((uint64_t)n * 4 * 18 + (uint64_t)npx * 8 + 8192 > c->qb_pool_bytes)
    return fail(c, NRRS_ENOMEM, "too many rows for the scratch space");
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  std::vector<float> rows(8ull * n), tq(4ull * n), qf(2ull * n);
  for (uint32_t i = 0; i < n; ++i) {
    for (int k = 0; k < 7; ++k) rows[8ull * i + k] = raw[7ull * i + k];
    rows[8ull * i + 7] = I[i];
    for (int k = 0; k < 3; ++k) tq[4ull * i + k] = t[3ull * i + k];
    tq[4ull * i + 3] = 0.0f;
    qf[2ull * i] = q_norm[i];
    qf[2ull * i + 1] = F[i];
  }
  Carve k{c->qb_pool};
  float* prow = k.take<float>(8ull * n);
  float* pL = k.take<float>(n);
  float* plum = k.take<float>(n);
  float4* ptq = k.take<float4>(n);
  float2* pqf = k.take<float2>(n);
  uint32_t* ppix = k.take<uint32_t>(n);
  float* pw = k.take<float>(npx);
  uint32_t* pk = k.take<uint32_t>(npx);
  HIPC(c, hipMemcpy(prow, rows.data(), sizeof(float) * 8 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pL, L, sizeof(float) * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(plum, lum_t, sizeof(float) * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(ptq, tq.data(), sizeof(float) * 4 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pqf, qf.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(ppix, pix, sizeof(uint32_t) * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pw, wpx, sizeof(float) * npx, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pk, kk, sizeof(uint32_t) * npx, hipMemcpyHostToDevice));
  const NrrsRows r{prow, plum, nullptr, pL, ptq, pqf, ppix, n};
  const uint32_t nb = nrrs_grad_blocks(n);
  launch_zero_u32((uint32_t*)c->ntab.g, c->ntab_n, s);
  launch_statnet_grad(r, c->nstat.w, c->ntab.w, c->cfg.hash_log2, 0.01f, c->npartial, c->nloss_part, c->ntab.g, s);
  launch_partial_sum(c->npartial, nb, kStatParams, c->nstat.g, c->nloss_part, c->nloss, c->ngroups, s);
  launch_rrsnet_grad(r, c->nstat.w, c->ntab.w, c->cfg.hash_log2, c->nrrs_net.w, rrs_step, pw, pk, g_rrs, 0.01f,
                     c->npartial, c->nloss_part, s);
  launch_partial_sum(c->npartial, nb, kRrsParams, c->nrrs_net.g, c->nloss_part, c->nloss + 1, c->ngroups, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  float l[2];
  HIPC(c, hipMemcpy(g_stat, c->nstat.g, sizeof(float) * kStatParams, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(g_rrs_out, c->nrrs_net.g, sizeof(float) * kRrsParams, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(g_table, c->ntab.g, sizeof(float) * c->ntab_n, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(l, c->nloss, sizeof(l), hipMemcpyDeviceToHost));
  *loss_stat = l[0];
  *loss_rrs = l[1];
  // leave the training state as it was: the grid gradient starts each step at zero
  launch_zero_u32((uint32_t*)c->ntab.g, c->ntab_n, s);
  HIPC(c, hipStreamSynchronize(s));
  return NRRS_OK;
}

int32_t nrrs_debug_aid_grads(nrrs_ctx* c, const float* raw, const float* I, const float* lum_t, const float* t,
                             const float* q_norm, const float* F, const uint32_t* pix, uint32_t n, const float* wpx,
                             const uint32_t* kk, uint32_t npx, int32_t rrs_step, float g_rrs, float* g_aid,
                             float* g_table_r, float* loss) {
  if (!c || n == 0 || !raw || !I || !lum_t || !t || !q_norm || !F || !pix || npx == 0 || !wpx || !kk || !g_aid ||
      !g_table_r || !loss || (rrs_step != 1 && rrs_step != 2) || !(g_rrs >= 0.0f))
    return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  if (n > c->cfg.records_cap) return fail(c, NRRS_EINVAL, "n beyond records_cap");
  for (uint32_t i = 0; i < n; ++i)
    if (pix[i] >= npx) return fail(c, NRRS_EINVAL, "pixel index beyond npx");
  if ((uint64_t)n * 4 * 18 + (uint64_t)npx * 8 + 8192 > c->qb_pool_bytes)
    return fail(c, NRRS_ENOMEM, "too many rows for the scratch space");
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  std::vector<float> rows(8ull * n), tq(4ull * n), qf(2ull * n);
  for (uint32_t i = 0; i < n; ++i) {
    for (int k = 0; k < 7; ++k) rows[8ull * i + k] = raw[7ull * i + k];
    rows[8ull * i + 7] = I[i];
    for (int k = 0; k < 3; ++k) tq[4ull * i + k] = t[3ull * i + k];
    tq[4ull * i + 3] = 0.0f;
    qf[2ull * i] = q_norm[i];
    qf[2ull * i + 1] = F[i];
  }
  Carve k{c->qb_pool};
  float* prow = k.take<float>(8ull * n);
  float* plum = k.take<float>(n);
  float4* ptq = k.take<float4>(n);
  float2* pqf = k.take<float2>(n);
  uint32_t* ppix = k.take<uint32_t>(n);
  float* pw = k.take<float>(npx);
  uint32_t* pk = k.take<uint32_t>(npx);
  HIPC(c, hipMemcpy(prow, rows.data(), sizeof(float) * 8 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(plum, lum_t, sizeof(float) * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(ptq, tq.data(), sizeof(float) * 4 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pqf, qf.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(ppix, pix, sizeof(uint32_t) * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pw, wpx, sizeof(float) * npx, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pk, kk, sizeof(uint32_t) * npx, hipMemcpyHostToDevice));
  const NrrsRows r{prow, plum, nullptr, nullptr, ptq, pqf, ppix, n};
  const uint32_t nb = nrrs_grad_blocks(n);
  launch_zero_u32((uint32_t*)c->ntab_r.g, c->ntab_n, s);
  launch_aid_grad(r, c->nstat.w, c->ntab.w, c->cfg.hash_log2, c->naid.w, c->ntab_r.w, rrs_step, pw, pk, g_rrs, 0.01f,
                  c->npartial, c->nloss_part, c->ntab_r.g, s);
  launch_partial_sum(c->npartial, nb, kAidParams, c->naid.g, c->nloss_part, c->nloss + 1, c->ngroups, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpy(g_aid, c->naid.g, sizeof(float) * kAidParams, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(g_table_r, c->ntab_r.g, sizeof(float) * c->ntab_n, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(loss, c->nloss + 1, sizeof(float), hipMemcpyDeviceToHost));
  launch_zero_u32((uint32_t*)c->ntab_r.g, c->ntab_n, s);
  HIPC(c, hipStreamSynchronize(s));
  return NRRS_OK;
}

int32_t nrrs_debug_pixel_error(nrrs_ctx* c, const float* cur, float* acc, const float* ref, uint32_t w, uint32_t h,
                               int32_t first, float a_mix, int32_t radius, float var_scale, float g_avg, float g_min,
                               float* E, float* wpx, double* e_avg) {
  if (!c || !cur || !acc || !ref || !E || !wpx || !e_avg || w == 0 || h == 0 || !(a_mix > 0.0f && a_mix <= 1.0f) ||
      radius < 0 || radius > 8)
    return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (!c->cfg.hash_log2) return fail(c, NRRS_ESTATE, "context created without NRRS (hash_log2 = 0)");
  const uint64_t npx = (uint64_t)w * h;
  if (npx > c->npx) return fail(c, NRRS_EINVAL, "image larger than the context's");
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipMemcpy(c->pcur, cur, sizeof(float) * npx, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(c->pref, ref, sizeof(float) * npx, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(c->pacc, acc, sizeof(float) * npx, hipMemcpyHostToDevice));
  PixelErrArgs pe{};
  pe.cur = c->pcur;
  pe.ref = c->pref;
  pe.acc = c->pacc;
  pe.Ep = c->pEp;
  pe.E = c->pE;
  pe.wpx = c->pwpx;
  pe.part = c->pix_part;
  pe.eavg = c->eavg;
  pe.w = w;
  pe.h = h;
  pe.first = first ? 1u : 0u;
  pe.radius = radius;
  pe.a_mix = a_mix;
  pe.var_scale = var_scale;
  pe.g_avg = g_avg;
  pe.g_min = g_min;
  pe.eps = 0.01f;
  launch_pixel_error(pe, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpy(acc, c->pacc, sizeof(float) * npx, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(E, c->pE, sizeof(float) * npx, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(wpx, c->pwpx, sizeof(float) * npx, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(e_avg, c->eavg, sizeof(double), hipMemcpyDeviceToHost));
  return NRRS_OK;
}

// ------------------------------------------------------------------------- test entry points
int32_t nrrs_debug_rrs_expand(nrrs_ctx* c, const float* q_orig, const uint32_t* id_lo, const uint32_t* id_hi,
                              uint32_t n, uint32_t depth, double budget_base, double f_rate, double* alpha,
                              int32_t norm_mode, uint32_t cap, uint32_t* X, uint32_t* offset,
                              uint32_t* parent_of_child, uint32_t* S, double* F, float* q_norm, uint32_t* retries) {
  if (!c || !alpha || !X || !offset || !S || !F || !retries || (n && (!q_orig || !id_lo || !id_hi))) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (n > c->cap || cap > c->cap || depth < 1 || depth >= NRRS_MAX_DEPTH || !(budget_base >= 0.0) ||
      !std::isfinite(budget_base) || !(f_rate > 0.0) || !std::isfinite(f_rate) || !(*alpha > 0.0 && *alpha <= 1.0) || (norm_mode != NRRS_NORM_TWO_SIDED && norm_mode != NRRS_NORM_DOWNSCALE))
    return fail(c, NRRS_EINVAL, "debug_rrs_expand: argument out of range");
  if (!finite_all(q_orig, n)) return fail(c, NRRS_EINVAL, "non-finite factor");
  for (uint32_t i = 0; i < n; ++i)
    if (q_orig[i] < 0.0f) return fail(c, NRRS_EINVAL, "negative factor");
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  std::vector<uint2> ids(n);
  for (uint32_t i = 0; i < n; ++i) ids[i] = make_uint2(id_lo[i], id_hi[i]);
  DepthCtl ctl[2];
  std::memset(ctl, 0, sizeof(ctl));
  ctl[0].n = n;
  if (n) {
    HIPC(c, hipMemcpy(c->q, q_orig, sizeof(float) * n, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->qa.id, ids.data(), sizeof(uint2) * n, hipMemcpyHostToDevice));
  }
  HIPC(c, hipMemcpy(c->ctl + depth, ctl, sizeof(ctl), hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(c->alpha, alpha, sizeof(double), hipMemcpyHostToDevice));
  uint32_t of0 = 0;
  HIPC(c, hipMemcpy(c->overflow, &of0, 4, hipMemcpyHostToDevice));
  RenderArgs a = base_args(c);
  a.depth = depth;
  a.max_depth = depth + 1;
  a.mode = NRRS_MODE_HEURISTIC;
  a.norm_mode = (uint32_t)norm_mode;
  a.f_rate = f_rate;
  a.budget_base = budget_base;
  a.cap = cap;
  a.dbg_parent = (uint32_t*)c->qb_pool;
  if ((uint64_t)cap * 4 > c->qb_pool_bytes) return fail(c, NRRS_ENOMEM, "scratch too small");
  launch_sum_q(a, s);
  launch_roulette(a, s);
  launch_parents(a, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpy(ctl, c->ctl + depth, sizeof(ctl), hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(alpha, c->alpha, sizeof(double), hipMemcpyDeviceToHost));
  uint32_t of = 0;
  HIPC(c, hipMemcpy(&of, c->overflow, 4, hipMemcpyDeviceToHost));
  *S = ctl[0].S;
  *F = ctl[0].F;
  *retries = ctl[0].retries;
  if (n) HIPC(c, hipMemcpy(offset, c->offs, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
  for (uint32_t i = 0; i < n; ++i) X[i] = (i + 1 < n ? offset[i + 1] : *S) - offset[i];
  if (parent_of_child && *S)
    HIPC(c, hipMemcpy(parent_of_child, c->qb_pool, sizeof(uint32_t) * (*S), hipMemcpyDeviceToHost));
  if (q_norm)
    for (uint32_t i = 0; i < n; ++i) q_norm[i] = (float)(ctl[0].F * (double)q_orig[i]);
  if (of) return fail(c, NRRS_EOVERFLOW, "overflow guard found no alpha that fits");
  return NRRS_OK;
}

// ------------------------------------------------- the entry point that allocates nothing
// Its partial sums, block counts, guard candidates and control words live in one fixed
// device array per GPU (the code object's own memory, held until the process ends) instead
// of the workspace.  In host code `scratch` names a host-side stand-in: the array's device
// address comes from hipGetSymbolAddress, looked up once per device and kept per device.
namespace {

constexpr uint64_t kNoallocScratchBytes = 320ull << 10;
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
uint8_t* g_scratch_dev[kNoallocMaxDevices] = {};

struct NoallocScratch {
  double* partial;
  uint32_t *bsum, *boff, *gsum;
  DepthCtl* ctl;
  double* alpha;
  uint32_t* overflow;
  uint64_t bytes;
};

NoallocScratch noalloc_layout(uint8_t* base) {
  Carve k{base};
  NoallocScratch r;
  r.partial = k.take<double>(kScanBlocks);
  r.bsum = k.take<uint32_t>(kScanBlocks);
  r.boff = k.take<uint32_t>(kScanBlocks);
  r.gsum = k.take<uint32_t>((uint64_t)kScanBlocks * kGuardSteps);
  r.ctl = k.take<DepthCtl>(NRRS_MAX_DEPTH + 2);
  r.alpha = k.take<double>(1);
  r.overflow = k.take<uint32_t>(1);
  r.bytes = k.off;
  return r;
}

// Device address of this device's scratch array (looked up on the first call on a device).
int32_t noalloc_scratch(nrrs_ctx* c, uint8_t** out) {
  int dev = -1;
  HIPC(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoallocMaxDevices) return fail(c, NRRS_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, NRRS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch_dev[dev];
  return NRRS_OK;
}

// Control words of the depth: entries n, nothing emitted yet; alpha and the overflow flag.
__global__ void k_noalloc_begin(DepthCtl* ctl, uint32_t depth, uint32_t n, double* alpha_slot, double alpha,
                                uint32_t* overflow) {
  DepthCtl z{};
  ctl[depth + 1] = z;
  z.n = n;
  ctl[depth] = z;
  *alpha_slot = alpha;
  *overflow = 0;
}

__global__ void k_noalloc_end(const DepthCtl* ctl, uint32_t depth, const double* alpha, const uint32_t* overflow,
                              nrrs_expand_result* out) {
  nrrs_expand_result r{};
  r.F = ctl[depth].F;
  r.alpha = *alpha;
  r.S = ctl[depth].S;
  r.retries = ctl[depth].retries;
  r.overflow = *overflow;
  *out = r;
}

}  // namespace

int32_t nrrs_rrs_expand_noalloc(nrrs_ctx* c, const float* q_dev, const uint32_t* lineage_dev, uint32_t n,
                                uint32_t depth, double budget_base, double f_rate, double alpha, int32_t norm_mode,
                                uint32_t cap, uint32_t* offset_dev, uint32_t* parent_dev,
                                nrrs_expand_result* result_dev) {
  if (!c || !result_dev || (n && (!q_dev || !lineage_dev || !offset_dev))) return NRRS_EINVAL;
  if (n > (1u << 31) || cap > (1u << 31))
    return fail(c, NRRS_EINVAL, "rrs_expand_noalloc: n and cap are limited to 2^31 entries");
  if (depth < 1 || depth >= NRRS_MAX_DEPTH || !(budget_base >= 0.0) || !std::isfinite(budget_base) ||
      !(f_rate > 0.0) || !std::isfinite(f_rate) || !(alpha > 0.0 && alpha <= 1.0) ||
      (norm_mode != NRRS_NORM_TWO_SIDED && norm_mode != NRRS_NORM_DOWNSCALE))
    return fail(c, NRRS_EINVAL, "rrs_expand_noalloc: argument out of range");
  const NoallocScratch need = noalloc_layout(nullptr);
  if (need.bytes > kNoallocScratchBytes) return fail(c, NRRS_ENOMEM, "rrs_expand_noalloc: scratch array too small");
  uint8_t* base = nullptr;
  const int32_t rs = noalloc_scratch(c, &base);
  if (rs != NRRS_OK) return rs;
  const NoallocScratch sc = noalloc_layout(base);
  hipStream_t s = c->stream;
  RenderArgs a{};
  a.q = const_cast<float*>(q_dev);
  a.qin.id = reinterpret_cast<uint2*>(const_cast<uint32_t*>(lineage_dev));
  a.offs = offset_dev;
  a.partial = sc.partial;
  a.bsum = sc.bsum;
  a.boff = sc.boff;
  a.gsum = sc.gsum;
  a.ctl = sc.ctl;
  a.alpha = sc.alpha;
  a.overflow = sc.overflow;
  a.key = make_uint2((uint32_t)c->cfg.seed, (uint32_t)(c->cfg.seed >> 32));
  a.depth = depth;
  a.max_depth = depth + 1;
  a.mode = NRRS_MODE_HEURISTIC;
  a.norm_mode = (uint32_t)norm_mode;
  a.f_rate = f_rate;
  a.budget_base = budget_base;
  a.cap = cap;
  a.dbg_parent = parent_dev;
  hipLaunchKernelGGL(k_noalloc_begin, dim3(1), dim3(1), 0, s, sc.ctl, depth, n, sc.alpha, alpha, sc.overflow);
  launch_sum_q(a, s);
  launch_roulette(a, s);
  if (parent_dev) launch_parents(a, s);
  hipLaunchKernelGGL(k_noalloc_end, dim3(1), dim3(1), 0, s, sc.ctl, depth, sc.alpha, sc.overflow, result_dev);
  HIPC(c, hipGetLastError());
  return NRRS_OK;
}

int32_t nrrs_debug_set_norm_factors(nrrs_ctx* c, const double* F, uint32_t n) {
  if (!c || (n && !F)) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (n >= NRRS_MAX_DEPTH) return fail(c, NRRS_EINVAL, "more factors than depths");
  for (uint32_t d = 0; d < n; ++d)
    if (!(F[d] >= 0.0) || !std::isfinite(F[d])) return fail(c, NRRS_EINVAL, "factor not finite and >= 0");
  HIPC(c, hipStreamSynchronize(c->stream));
  if (n) {
    std::vector<double> h(NRRS_MAX_DEPTH + 1, 0.0);
    for (uint32_t d = 0; d < n; ++d) h[d + 1] = F[d];
    HIPC(c, hipMemcpy(c->f_fixed, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
  }
  if ((n != 0) != (c->f_fixed_n != 0)) c->drop_graphs();  // captured passes hold the old arguments
  c->f_fixed_n = n;
  return NRRS_OK;
}

int32_t nrrs_debug_load_records(nrrs_ctx* c, const float* features, const float* lum_t, const float* acc,
                                uint32_t n) {
  if (!c || (n && (!features || !lum_t || !acc))) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (n > c->cfg.records_cap) return fail(c, NRRS_ENOMEM, "more records than records_cap");
  HIPC(c, hipStreamSynchronize(c->stream));
  if (n) {
    HIPC(c, hipMemcpy(c->rec.feat, features, sizeof(float) * 20 * n, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->rec.lum_t, lum_t, sizeof(float) * n, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->rec.acc, acc, sizeof(float) * n, hipMemcpyHostToDevice));
  }
  HIPC(c, hipMemcpy(c->rec.count, &n, 4, hipMemcpyHostToDevice));
  return NRRS_OK;
}

int32_t nrrs_debug_read_queue(nrrs_ctx* c, int32_t which, uint32_t n, float* orig, float* dir, float* thr,
                              float* hit) {
  if (!c || (which != 0 && which != 1)) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (n > c->cap) return fail(c, NRRS_EINVAL, "n exceeds the queue capacity");
  if (n == 0) return NRRS_OK;
  const Queue& q = which == 0 ? c->qa : c->qb;
  HIPC(c, hipStreamSynchronize(c->stream));
  if (orig) HIPC(c, hipMemcpy(orig, q.orig, sizeof(float4) * n, hipMemcpyDeviceToHost));
  if (dir) HIPC(c, hipMemcpy(dir, q.dir, sizeof(float4) * n, hipMemcpyDeviceToHost));
  if (thr) HIPC(c, hipMemcpy(thr, q.thr, sizeof(float4) * n, hipMemcpyDeviceToHost));
  if (hit) HIPC(c, hipMemcpy(hit, c->hit, sizeof(float4) * n, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_debug_trace(nrrs_ctx* c, const float* rays, const uint32_t* exclude, uint32_t n, uint32_t* prim,
                         float* t, float* b1, float* b2) {
  if (!c || (n && (!rays || !prim || !t || !b1 || !b2))) return NRRS_EINVAL;
  if (!c->scene) return fail(c, NRRS_ESTATE, "upload a scene first");
  if (n == 0) return NRRS_OK;
  std::vector<float> o(4ull * n), d(4ull * n);
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t ex = exclude ? exclude[i] : 0xffffffffu;
    if (ex != 0xffffffffu) {
      if (ex >= c->orig_to_bvh.size()) return fail(c, NRRS_EINVAL, "exclude index out of range");
      ex = c->orig_to_bvh[ex];
    }
    for (int k = 0; k < 3; ++k) {
      o[4ull * i + k] = rays[6ull * i + k];
      d[4ull * i + k] = rays[6ull * i + 3 + k];
    }
    std::memcpy(&o[4ull * i + 3], &ex, 4);
    d[4ull * i + 3] = 0.0f;
  }
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  if (n > c->cap) return fail(c, NRRS_ENOMEM, "more rays than the queue capacity");
  // the rays go through the render's own traversal kernel as queue entries of depth 1
  std::vector<float> th(4ull * n, 1.0f);
  for (uint32_t i = 0; i < n; ++i) th[4ull * i + 3] = 0.0f;  // flags = 0
  HIPC(c, hipMemcpy(c->qa.orig, o.data(), sizeof(float4) * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(c->qa.dir, d.data(), sizeof(float4) * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(c->qa.thr, th.data(), sizeof(float4) * n, hipMemcpyHostToDevice));
  DepthCtl ctl;
  std::memset(&ctl, 0, sizeof(ctl));
  ctl.n = n;
  HIPC(c, hipMemcpy(c->ctl + 1, &ctl, sizeof(ctl), hipMemcpyHostToDevice));
  launch_zero_u32(c->work, (uint64_t)(NRRS_MAX_DEPTH + 2) * kWorkSlices * kWorkStride, s);
  RenderArgs a = base_args(c);
  a.depth = 1;
  a.max_depth = 2;
  launch_extend(a, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  float4* ph = c->hit;
  std::vector<float> h(4ull * n);
  HIPC(c, hipMemcpy(h.data(), ph, sizeof(float4) * n, hipMemcpyDeviceToHost));
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t p;
    std::memcpy(&p, &h[4ull * i + 3], 4);
    prim[i] = p == 0xffffffffu ? p : c->bvh_order[p];
    t[i] = h[4ull * i];
    b1[i] = h[4ull * i + 1];
    b2[i] = h[4ull * i + 2];
  }
  return NRRS_OK;
}

int32_t nrrs_debug_philox(nrrs_ctx* c, const uint32_t* ctr, const uint32_t* key, uint32_t n, uint32_t* out) {
  if (!c || !key || (n && (!ctr || !out))) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if ((uint64_t)n * 32 > c->qb_pool_bytes) return fail(c, NRRS_ENOMEM, "too many counters for the scratch space");
  if (n == 0) return NRRS_OK;
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  uint4* pc = (uint4*)c->qb_pool;
  uint4* po = pc + n;
  HIPC(c, hipMemcpy(pc, ctr, 16ull * n, hipMemcpyHostToDevice));
  launch_philox(pc, make_uint2(key[0], key[1]), po, n, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpy(out, po, 16ull * n, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_debug_mlp_forward(nrrs_ctx* c, const float* x, uint32_t n, int32_t precision, float* y, float* z) {
  if (!c || (n && (!x || !y))) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (precision < NRRS_PREC_FP32 || precision > NRRS_PREC_FP8) return fail(c, NRRS_EINVAL, "precision");
  if ((uint64_t)n * 88 + 1024 > c->qb_pool_bytes) return fail(c, NRRS_ENOMEM, "too many rows for the scratch space");
  if (n == 0) return NRRS_OK;
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  float* px = (float*)c->qb_pool;
  float* py = px + 20ull * n;
  float* pz = py + n;
  HIPC(c, hipMemcpy(px, x, sizeof(float) * 20 * n, hipMemcpyHostToDevice));
  launch_mlp_forward_rows(px, n, net_args(c, precision), py, pz, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpy(y, py, sizeof(float) * n, hipMemcpyDeviceToHost));
  if (z) HIPC(c, hipMemcpy(z, pz, sizeof(float) * n, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_debug_mlp_codes(nrrs_ctx* c, const float* x, uint32_t n, int32_t precision, float* y, uint16_t* codes,
                             int8_t* scale_exp) {
  if (!c || (n && (!x || !y || !codes || !scale_exp))) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (precision != NRRS_PREC_BF16 && precision != NRRS_PREC_FP8)
    return fail(c, NRRS_EINVAL, "codes exist for the BF16 and FP8 networks only");
  if ((uint64_t)n * 480 + 4096 > c->qb_pool_bytes) return fail(c, NRRS_ENOMEM, "too many rows for the scratch space");
  if (n == 0) return NRRS_OK;
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  Carve k{c->qb_pool};
  float* px = k.take<float>(20ull * n);
  float* py = k.take<float>(n);
  uint16_t* pc = k.take<uint16_t>(192ull * n);
  int8_t* pse = k.take<int8_t>(3ull * n);
  HIPC(c, hipMemcpy(px, x, sizeof(float) * 20 * n, hipMemcpyHostToDevice));
  launch_codes_mfma(px, n, net_args(c, precision), py, pc, pse, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpy(y, py, sizeof(float) * n, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(codes, pc, sizeof(uint16_t) * 192 * n, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(scale_exp, pse, 3ull * n, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

int32_t nrrs_debug_mlp_grad(nrrs_ctx* c, const float* x, const float* target, uint32_t n, float* grad, float* loss) {
  if (!c || !grad || !loss || n == 0 || !x || !target) return NRRS_EINVAL;
  if (!c->bound) return fail(c, NRRS_ESTATE, "no workspace");
  if (n > kMaxMinibatch) return fail(c, NRRS_EINVAL, "at most 65536 rows");
  if ((uint64_t)n * 84 + 1024 > c->qb_pool_bytes) return fail(c, NRRS_ENOMEM, "too many rows for the scratch space");
  hipStream_t s = c->stream;
  HIPC(c, hipStreamSynchronize(s));
  float* px = (float*)c->qb_pool;
  float* pt = px + 20ull * n;
  HIPC(c, hipMemcpy(px, x, sizeof(float) * 20 * n, hipMemcpyHostToDevice));
  HIPC(c, hipMemcpy(pt, target, sizeof(float) * n, hipMemcpyHostToDevice));
  launch_zero_u32((uint32_t*)c->loss_accum, 1, s);
  uint32_t nb = 0;
  launch_mlp_grad(px, pt, nullptr, n, c->master, c->cfg.loss, c->grad_partial, c->loss_partial, &nb, s);
  launch_grad_reduce(c->grad_partial, nb, c->grad, c->loss_partial, c->loss_accum, n, s);
  HIPC(c, hipStreamSynchronize(s));
  HIPC(c, hipGetLastError());
  HIPC(c, hipMemcpy(grad, c->grad, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
  HIPC(c, hipMemcpy(loss, c->loss_accum, 4, hipMemcpyDeviceToHost));
  return NRRS_OK;
}

}  // extern "C"
