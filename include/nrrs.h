/* nrrs.h -- C ABI of the MI355X (gfx950) normalized-RRS wavefront path tracer.
 *
 * The library renders with unidirectional path tracing in a wavefront loop
 * (extend -> shade -> [RRS network] -> normalization -> roulette/split ->
 * compaction), following NRRS: Neural Russian Roulette and Splitting
 * (arXiv 2510.07868):
 *   - one-sample estimator of the rendering equation      Sec. 3, Eqs. (1)-(2)
 *   - stochastic rounding of an RRS factor into children  Sec. 3, Eq. (8)
 *   - per-depth normalization of the factors              Sec. 4.1.2, Eqs. (9)-(11)
 *   - rate control and adaptive alpha on overflow          Sec. 4.1.4, Eqs. (12)-(14)
 *   - downscale-only normalization                         Sec. 5, "Compromise"
 *   - RRS network output activation (modified softplus)    Sec. 5, Eq. (22)
 *   - depth-gated use of the network (Mix-Depth)           Sec. 4.3
 *   - ADRRS ratio for the factor from a radiance estimate  Sec. 2.2
 *
 * Conventions common to every call:
 *   - Every call returns an nrrs_status (0 = NRRS_OK, negative = error).  On
 *     error the context is left as it was before the call unless stated.
 *   - No C++ exception crosses this boundary.  A context is used from one host
 *     thread at a time.
 *   - "host" pointers are ordinary CPU memory owned by the caller and only read
 *     or written during the call.  "device" pointers are HIP device memory owned
 *     by the caller.
 *   - Work is queued on the HIP stream given to nrrs_create; calls that return
 *     host data synchronize that stream first.
 */
#ifndef NRRS_H
#define NRRS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nrrs_ctx nrrs_ctx;

enum nrrs_status {
  NRRS_OK = 0,
  NRRS_EINVAL = -1,      /* bad argument; context unchanged */
  NRRS_ESTATE = -2,      /* call out of order (e.g. render before upload) */
  NRRS_ENOMEM = -3,      /* bound workspace too small for the request */
  NRRS_EHIP = -4,        /* HIP runtime error; nrrs_last_error has the message */
  NRRS_EOVERFLOW = -5,   /* the overflow guard could not fit the queue (see nrrs_render) */
  NRRS_EUNSUPPORTED = -6 /* device is not gfx950, or feature not available */
};

enum nrrs_mode {
  NRRS_MODE_OFF = 0,       /* plain path tracing: factor 1, no normalization */
  NRRS_MODE_HEURISTIC = 1, /* normalized RRS with q = lum(throughput * albedo) */
  NRRS_MODE_NET = 2,       /* normalized RRS with the network factor at the depths of the Mix-Depth
                              table (nrrs_set_mix_depth; default: depth <= net_max_depth) */
  NRRS_MODE_NRRS = 3,      /* normalized RRS with the NRRS factor (StatNet + RRSNet, Sec. 4.2) at the
                              depths of the Mix-Depth table; needs hash_log2 > 0 at creation */
  NRRS_MODE_AID = 4        /* as NRRS_MODE_NRRS with the AID-NRRS RRSNet (its own hash grid and
                              one-blob inputs, no StatNet at inference; Sec. 4.2.1) */
};

enum nrrs_norm { NRRS_NORM_TWO_SIDED = 0, NRRS_NORM_DOWNSCALE = 1 };

enum nrrs_precision { NRRS_PREC_FP32 = 0, NRRS_PREC_BF16 = 1, NRRS_PREC_FP8 = 2 };

enum nrrs_material_type { NRRS_MAT_LAMBERT = 0, NRRS_MAT_GGX = 1, NRRS_MAT_EMITTER = 2 };

/* Training loss of the network's radiance estimate y against a record's one-sample target L:
 * relative L2 (y - L)^2 / (sg(y)^2 + 0.01), the statistic loss of Sec. 4.2.2 Eq. (15) whose
 * minimiser is the mean radiance; or (ln(y + 0.01) - ln(L + 0.01))^2. */
enum nrrs_loss { NRRS_LOSS_REL_L2 = 0, NRRS_LOSS_LOG_MSE = 1 };

#define NRRS_MAX_DEPTH 64
#define NRRS_NSTAGES 8 /* camera, extend, shade, network, sum, roulette+scan, expand, pass end */
#define NRRS_NPARAM 9729 /* 20-64-64-64-1 network: weights and biases */

typedef struct {
  uint32_t width, height; /* image size in pixels, each >= 1 */
  uint32_t s_batch;       /* samples per pixel traced together in one wavefront pass (>= 1) */
  double cap_factor;      /* queue capacity C = floor(cap_factor * W * H * s_batch), >= 1 */
  double f_rate;          /* rate-control factor of Eq. (12); 1.0 = plain normalization */
  int32_t norm_mode;      /* nrrs_norm */
  uint64_t seed;          /* Philox4x32-10 key */
  int32_t net_max_depth;  /* training records are taken at depth <= this (0..4); also the default
                             Mix-Depth table: the network at depths 1..net_max_depth in NET mode */
  int32_t precision;      /* nrrs_precision of network inference */
  uint32_t records_cap;   /* capacity of the training-record buffer (0 = no records) */
  double p_train;         /* probability that a primary path records training vertices */
  int32_t loss;           /* nrrs_loss used by nrrs_train_step */
  double ema_decay;       /* inference uses an exponential moving average of the weights with this
                             decay per Adam step (Sec. 5 "Training"); 0 = the latest weights */
  uint32_t trace_depth;   /* > 0: reserve workspace for nrrs_set_trace (per-path radiance of
                             depths 1..trace_depth: 8 B per queue slot + 24 * trace_depth B per
                             primary path); 0: not available */
  uint32_t hash_log2;     /* > 0 (14..22): reserve NRRS proper (Sec. 4.2): StatNet's hash grid of
                             2^hash_log2 entries per level, StatNet, RRSNet and their training
                             state (about 80 * 2^hash_log2 B); 0: not available */
  uint32_t nee;           /* 1: next-event estimation (the paper's experiments enable it, Sec. 6): at
                             every vertex that may continue, one light sample (an emitting triangle
                             with probability lum(L_e) x area, a point uniform on it), a shadow ray
                             from the offset hit point, and power-heuristic MIS against the BSDF's
                             sampling (also weighting the BSDF-sampled light hits); its contribution
                             reaches the image, the ancestors' training records and the per-path
                             radiance at the vertex's depth.  0: off */
} nrrs_config;

typedef struct {
  uint32_t max_depth, passes;
  uint64_t n[NRRS_MAX_DEPTH + 1];       /* queue entries entering depth d, summed over passes */
  uint64_t S[NRRS_MAX_DEPTH + 1];       /* children emitted at depth d, summed over passes */
  uint64_t retries[NRRS_MAX_DEPTH + 1]; /* overflow-guard alpha reductions at depth d */
  double sumq[NRRS_MAX_DEPTH + 1];      /* FP64 sum of the raw factors at depth d (last pass) */
  double F[NRRS_MAX_DEPTH + 1];         /* normalization factor at depth d (last pass) */
  double alpha;                         /* adaptive-rate alpha after the render */
  uint64_t rays;                        /* rays traced (queue entries that were not dead) */
  uint64_t nodes_visited;               /* BVH nodes visited by all traversals */
  uint64_t tris_tested;                 /* ray-triangle tests by all traversals */
  uint64_t records;                     /* training records held after the render */
  uint32_t overflow;                    /* 1 if the guard could not fit a depth (pass truncated) */
  uint32_t timed;                       /* 1 if stage_ms / stage_launches were measured */
  double stage_ms[NRRS_NSTAGES];        /* GPU time per stage (HIP events on the context stream) */
  uint64_t stage_launches[NRRS_NSTAGES];/* launches (kernel groups) per stage */
} nrrs_render_stats;

/* Create a context.  cfg: see nrrs_config (copied).  hip_stream: a hipStream_t owned by
 * the caller (may be NULL for the null stream); it must outlive the context.  *out
 * receives the context.  EINVAL on a bad config, EUNSUPPORTED if the current device is
 * not gfx950, EHIP on a runtime failure. */
int32_t nrrs_create(const nrrs_config* cfg, void* hip_stream, nrrs_ctx** out);

/* Bytes of device workspace needed for scenes of up to max_tris triangles and
 * max_materials materials.  The caller allocates it (any HIP allocator). */
int32_t nrrs_workspace_size(const nrrs_ctx* ctx, uint64_t max_tris, uint32_t max_materials,
                            uint64_t* bytes);

/* Bind caller-owned device memory of `bytes` bytes (256-byte aligned) as the workspace.
 * The library never allocates device memory itself.  The memory must stay valid until
 * nrrs_destroy or the next bind.  Binding clears the image, records and guide. */
int32_t nrrs_bind_workspace(nrrs_ctx* ctx, void* device_ptr, uint64_t bytes, uint64_t max_tris,
                            uint32_t max_materials);

/* Upload a triangle scene (host arrays, copied during the call; nothing is retained):
 *   verts[nv*3] float xyz; tris[nt*3] vertex indices; tri_mat[nt] material per triangle;
 *   mat_type[nm] nrrs_material_type; mat_params[nm*7] = (rho rgb, ggx alpha, Le rgb) where
 *   rho is the Lambertian albedo or the GGX F0; camera[10] = eye xyz, look-at xyz, up xyz,
 *   vertical fov in degrees; env[3] constant radiance seen by rays that miss.
 * A triangle emits (Le) on the side of cross(v1-v0, v2-v0).  Builds a BVH on the host
 * (binned SAH, leaves of at most 4 triangles) and copies it to the workspace.  EINVAL on
 * out-of-range indices, non-finite values, nt == 0 or a tree deeper than the traversal
 * stack allows; ENOMEM if nt or nm exceed the bound workspace. */
int32_t nrrs_upload_scene(nrrs_ctx* ctx, const float* verts, uint64_t nv, const uint32_t* tris,
                          uint64_t nt, const uint32_t* tri_mat, const uint32_t* mat_type,
                          const float* mat_params, uint32_t nm, const float* camera, const float* env);

/* Instanced geometry for nrrs_upload_scene_instanced (host arrays, copied during the call).
 *   Meshes in object space: mesh_verts[mesh_nv*3]; mesh_tris[*3] vertex indices and
 *   mesh_tri_mat[] materials of all meshes' triangles concatenated; mesh m is triangles
 *   [mesh_tri_begin[m], mesh_tri_begin[m+1]) (n_meshes + 1 entries, the first 0, each mesh
 *   non-empty).
 *   Instances: inst_mesh[n_inst] the mesh; inst_xform[n_inst*12] the object-to-world affine
 *   map as a row-major 3x4 matrix (world = A * object + t, A invertible; det A < 0 mirrors the
 *   emitting side with the triangles); inst_mat[n_inst] a material for all of the instance's
 *   triangles, or NRRS_NO_MATERIAL to keep the mesh's own. */
#define NRRS_NO_MATERIAL 0xFFFFFFFFu
typedef struct nrrs_instances {
  const float* mesh_verts;
  uint64_t mesh_nv;
  const uint32_t* mesh_tris;
  const uint32_t* mesh_tri_mat;
  const uint64_t* mesh_tri_begin;
  uint32_t n_meshes;
  const uint32_t* inst_mesh;
  const float* inst_xform;
  const uint32_t* inst_mat;
  uint32_t n_inst;
} nrrs_instances;

/* Upload a two-level scene: the base mesh (as in nrrs_upload_scene, world space; nt may be 0)
 * plus instances of object-space meshes (the paper's batched scenes instance their boxes,
 * Sec. 6; its wavefront renderer traces them through two-level hardware trees, Sec. 3).  One
 * BVH per mesh and one for the base mesh (binned SAH, leaves of at most 4 triangles), and a
 * BVH over the instances' world boxes (the base mesh one of them, with the identity map);
 * rays are moved into each instance's object space during traversal, a mesh is stored once.
 * Renders equal those of the flattened scene (base triangles, then every instance's mesh
 * triangles in mesh order, at world positions ((a00 x + a01 y) + a02 z) + t0, ... rounded to
 * float) up to float32 rounding; nrrs_debug_trace numbers triangles in that flattened order.
 * The workspace must hold nt + (all meshes' triangles) + 3 per instance (+ 3 for the base
 * mesh) in max_tris.  Traversal variants 2 and 4 are not available for such scenes (the
 * tuning switches to variant 3).  EINVAL on bad indices, non-finite values, a singular map,
 * 2^26 instances or more, more than 2^31 triangles after flattening, or trees together deeper
 * than the traversal stack; ENOMEM if the workspace is too small. */
int32_t nrrs_upload_scene_instanced(nrrs_ctx* ctx, const float* verts, uint64_t nv, const uint32_t* tris,
                                    uint64_t nt, const uint32_t* tri_mat, const uint32_t* mat_type,
                                    const float* mat_params, uint32_t nm, const float* camera,
                                    const float* env, const nrrs_instances* instances);

/* Render spp samples per pixel (spp a multiple of s_batch: spp / s_batch wavefront passes)
 * with paths of at most max_depth vertices (1..64) and the given nrrs_mode.  Radiance is
 * accumulated in FP64 per pixel across calls until nrrs_reset_image.  In HEURISTIC and
 * NET modes training records are captured when records_cap > 0.  Asynchronous unless
 * stats is non-NULL, in which case the stream is synchronized and the per-depth
 * statistics of this call are written.  NET mode without a guide image (no earlier
 * render, nor nrrs_set_guide) uses the heuristic factor.  When a depth's children would
 * exceed the queue capacity, the roulette is repeated with the same uniforms and alpha
 * reduced by the factor 0.99 until they fit (Eq. 14; alpha persists across passes until
 * nrrs_reset_image).  EOVERFLOW is returned (with stats) when alpha fell below 1e-3 first;
 * that pass was truncated at that depth. */
int32_t nrrs_render(nrrs_ctx* ctx, uint32_t spp, uint32_t max_depth, int32_t mode,
                    nrrs_render_stats* stats);

/* One training epoch of the network on the first n_records records of the last render
 * (records are cleared by each render that captures them): minibatches of `minibatch`
 * records, one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) each, with the
 * configured nrrs_loss (mean over the minibatch) and L = acc / lum_t the record's reflected-
 * radiance target.
 * *loss_or_null receives the mean loss of the epoch (synchronizes).  ESTATE if fewer than
 * n_records records exist; EINVAL if minibatch is 0 or does not divide n_records. */
int32_t nrrs_train_step(nrrs_ctx* ctx, uint32_t n_records, uint32_t minibatch, float lr,
                        float* loss_or_null);

/* Copy the mean radiance (sum / spp_total, W*H*3 doubles, row-major from the top image row)
 * to host_rgb, and the samples per pixel so far to *spp_total.  Synchronizes. */
int32_t nrrs_read_image(nrrs_ctx* ctx, double* host_rgb, uint64_t* spp_total);

/* Zero the image accumulator and the sample count and reset alpha to 1.  The guide is kept,
 * and the pass counter that keys the random numbers keeps counting (a new render after a
 * reset draws fresh random numbers). */
int32_t nrrs_reset_image(nrrs_ctx* ctx);

/* Guide image: per-pixel luminance of the previous mean radiance, used as the pixel
 * estimate in the NET factor (Sec. 5 "Compromise").  set: host lum[W*H] (negative = no
 * history for that pixel).  get: copies it out.  Each render pass refreshes it. */
int32_t nrrs_set_guide(nrrs_ctx* ctx, const float* host_lum);
int32_t nrrs_get_guide(nrrs_ctx* ctx, float* host_lum);

/* Network state: FP32 master parameters[NRRS_NPARAM], Adam m and v (same size) and the
 * Adam step count.  Layout of the parameter vector: W1[64][20], b1[64], W2[64][64], b2[64],
 * W3[64][64], b3[64], W4[64], b4.  Any pointer may be NULL to skip that part.  set also
 * resets the inference weights (and their moving average) to the given master and
 * refreshes the BF16 / FP8 inference copies. */
int32_t nrrs_get_params(nrrs_ctx* ctx, float* master, float* adam_m, float* adam_v, uint64_t* step);
int32_t nrrs_set_params(nrrs_ctx* ctx, const float* master, const float* adam_m,
                        const float* adam_v, const uint64_t* step);

/* Network state that nrrs_get_params leaves out, for a checkpoint that resumes exactly:
 * infer[NRRS_NPARAM], the inference weights (the moving average of the masters that the
 * renders use, Sec. 5 "Training"), and *alpha, the adaptive rate of the overflow guard
 * (Eq. 14), which persists across passes.  Either pointer may be NULL.  set: call it after
 * nrrs_set_params (which resets the inference weights to the masters); it refreshes the
 * BF16 / FP8 inference copies.  EINVAL for a non-finite weight or alpha outside (0, 1]. */
int32_t nrrs_get_state(nrrs_ctx* ctx, float* infer, double* alpha);
int32_t nrrs_set_state(nrrs_ctx* ctx, const float* infer, const double* alpha);

/* --- NRRS proper (Sec. 4.2; Sec. 5 "Network Architecture", "Input Encoding", "Training") ------
 * Needs a context created with hash_log2 > 0 (ESTATE otherwise).
 * StatNet: hash grid of the vertex position (8 levels x 2 features, coarsest resolution 16,
 * doubling per level; dense where a level's corners fit the 2^hash_log2 entries, else the
 * spatial hash) + one-blob w_o (theta / pi and phi / 2pi + 1/2, 4 bins each) + one-blob remapped
 * roughness (8 bins) -> 32 -> 32 -> 32 -> 2 (leaky ReLU 0.01): the luminance mean m and variance
 * v of the radiance reflected at the vertex.  RRSNet: Box-Cox (lambda 1/2) of m, v + m^2, the
 * throughput (rgb) and the pixel value, and the remapped roughness -> 32 -> 32 -> 32 -> 1,
 * modified softplus (Eq. 22): the RRS factor.  Parameter vectors: W1[32][in], b1[32], W2[32][32],
 * b2, W3[32][32], b3, W4[out][32], b4 (NRRS_STAT_NPARAM, NRRS_RRS_NPARAM floats); hash grid
 * [8][2^hash_log2][2] floats.  Renders in NRRS_MODE_NRRS use the inference copies (the moving
 * average of the masters with cfg.ema_decay per Adam step). */
#define NRRS_STAT_NPARAM 3234
#define NRRS_RRS_NPARAM 2401
#define NRRS_AID_NPARAM 3201 /* AID-NRRS RRSNet: 32 -> 32 -> 32 -> 32 -> 1 */

/* Set (masters and inference copies; Adam moments and step cleared) or get (masters) the NRRS
 * networks from host arrays; any pointer may be NULL to skip that part.  set: EINVAL for a
 * non-finite value. */
int32_t nrrs_set_nrrs_params(nrrs_ctx* ctx, const float* stat, const float* rrs, const float* table);
int32_t nrrs_get_nrrs_params(nrrs_ctx* ctx, float* stat, float* rrs, float* table);

typedef struct {
  float lr_stat, lr_rrs;      /* Adam learning rates (the paper's 0.005 and 0.0003) */
  float g_avg, g_min, g_rrs;  /* gamma1 (L_avg), gamma2 (L_min), gamma3 (L_rrs) of Eq. (16) */
  float a_mix;                /* temporal mix of the error image, Eq. (23), in (0, 1] */
  int32_t radius;             /* box-filter radius (pixels, 0..8) of the error image, in place of
                                 the paper's denoiser */
  int32_t rrs_step;           /* 1: RRSNet fitted to the output 1; 2: trained by Eq. (16) */
  int32_t variant;            /* which RRSNet trains: 0 NRRS (StatNet's statistics as inputs), 1 AID-NRRS
                                 (its own hash grid + one-blob inputs; StatNet only supervises), 2 both
                                 (loss_rrs then reports the AID-NRRS one) */
} nrrs_nrrs_train;

typedef struct {
  float loss_stat;  /* Eq. (15), mean over the records */
  float loss_rrs;   /* step 1: relative L2 to 1 (mean); step 2: gamma3 L_rrs (sum) */
  double e_avg;     /* mean relative pixel error E_avg of the frame (Eq. 20) */
  uint32_t records; /* records used */
  uint32_t rrs_trained;  /* 0 when step 2 had no previous frame to compare with */
} nrrs_nrrs_loss;

/* One NRRS training step over the records of the frame rendered since the previous call (or
 * since the image was reset): one Adam step of StatNet (Eq. 15; hash grid and MLP) over all
 * of them, then one of RRSNet with StatNet's updated weights.  Step 2 also forms the frame's
 * pixel error: the frame's luminance per pixel against the mean of the previous frames, mixed
 * over frames (Eq. 23), box-filtered, and turned into the derivative of gamma1 L_avg +
 * gamma2 L_min with respect to each pixel's variance, which reaches each record's factor through
 * Eqs. (17)-(18) (shared by the pixel's records).  The error image is taken at the variance of a
 * one-sample pixel estimate: the squared error scaled by the frame's samples per pixel (and by
 * (2 - a) / a once mixed).  n_records: how many of the captured records to use (<= the count
 * captured, <= records_cap).  Synchronous when out != NULL. */
int32_t nrrs_train_step_nrrs(nrrs_ctx* ctx, uint32_t n_records, const nrrs_nrrs_train* hp, nrrs_nrrs_loss* out);

/* AID-NRRS RRSNet (Sec. 4.2.1; Sec. 5 "Input Encoding"): inputs = its own hash grid of the
 * position (same shape as StatNet's, 16) + one-blob w_o (8) + Box-Cox of the throughput (3) and
 * of the pixel value (1) + one-blob remapped roughness with 4 bins (4) -> 32 -> 32 -> 32 -> 1,
 * modified softplus.  Set (masters and inference copies; its Adam state cleared) or get
 * (masters) aid[NRRS_AID_NPARAM] and its hash grid table_r (layout as StatNet's); either
 * pointer may be NULL. */
int32_t nrrs_set_aid_params(nrrs_ctx* ctx, const float* aid, const float* table_r);
int32_t nrrs_get_aid_params(nrrs_ctx* ctx, float* aid, float* table_r);

/* Test entry points (host arrays, synchronous).
 * nrrs_debug_aid_forward: the AID-NRRS factor q[n] (and, if enc is not NULL, its 32 inputs
 * enc[32n]) with the inference copies, vertices as in nrrs_debug_nrrs_forward.
 * nrrs_debug_aid_grads: the AID-NRRS RRSNet's gradients (no Adam step): MLP into g_aid, its hash
 * grid into g_table_r, loss as nrrs_nrrs_loss.loss_rrs; StatNet (masters) supplies the
 * statistics of step 2; records as in nrrs_debug_nrrs_grads.
 * nrrs_debug_nrrs_forward: StatNet (m, v) into mv[2n], the factor into q[n] and, if enc is
 * not NULL, StatNet's 32 inputs into enc[32n], for vertices raw[7n] = (position in [0,1]^3,
 * w_o, remapped roughness), throughput t[3n] and pixel value I[n], with the inference copies.
 * nrrs_debug_nrrs_grads: the gradients (no Adam step) of StatNet (Eq. 15, mean over n; MLP
 * into g_stat, hash grid into g_table) and of RRSNet (rrs_step 1 or 2) for records given as
 * raw[7n], I[n], StatNet target L[n], lum_t[n], t[3n], q_norm[n], F[n], pix[n] and per-pixel
 * wpx[npx], k[npx] (pix < npx), with the masters; losses as in nrrs_nrrs_loss.
 * nrrs_debug_pixel_error: the pixel-error stage on host images cur, ref (< 0: no reference)
 * and acc (in/out) of w x h pixels: E[w h], wpx[w h] and *e_avg. */
int32_t nrrs_debug_nrrs_forward(nrrs_ctx* ctx, const float* raw, const float* t, const float* I, uint32_t n,
                                float* mv, float* q, float* enc);
int32_t nrrs_debug_nrrs_grads(nrrs_ctx* ctx, const float* raw, const float* I, const float* L, const float* lum_t,
                              const float* t, const float* q_norm, const float* F, const uint32_t* pix, uint32_t n,
                              const float* wpx, const uint32_t* k, uint32_t npx, int32_t rrs_step, float g_rrs,
                              float* g_stat, float* g_rrs_out, float* g_table, float* loss_stat, float* loss_rrs);
int32_t nrrs_debug_aid_forward(nrrs_ctx* ctx, const float* raw, const float* t, const float* I, uint32_t n, float* q,
                               float* enc);
int32_t nrrs_debug_aid_grads(nrrs_ctx* ctx, const float* raw, const float* I, const float* lum_t, const float* t,
                             const float* q_norm, const float* F, const uint32_t* pix, uint32_t n, const float* wpx,
                             const uint32_t* k, uint32_t npx, int32_t rrs_step, float g_rrs, float* g_aid,
                             float* g_table_r, float* loss);
int32_t nrrs_debug_pixel_error(nrrs_ctx* ctx, const float* cur, float* acc, const float* ref, uint32_t w, uint32_t h,
                               int32_t first, float a_mix, int32_t radius, float var_scale, float g_avg, float g_min,
                               float* E, float* wpx, double* e_avg);

/* Per-path radiance by depth (a parity aid for the one-sample estimator of Sec. 3,
 * Eqs. (1)-(2)): while enabled, every emission collected at vertex depth d is also added
 * (FP64) to entry (k, d) of the primary path k it descends from, so that a path that takes a
 * different near-tie decision at some depth can still be compared at the depths before it.
 * Primary path k of a pass is sample k mod s_batch of pixel k / s_batch; the sums accumulate
 * over passes until nrrs_set_trace(ctx, 1) is called again (which zeroes them).  Enabling
 * needs a context created with trace_depth > 0 (ESTATE otherwise); while enabled, renders
 * deeper than trace_depth return EINVAL.  Switching drops the captured pass graphs.  read:
 * copies host_rgb[W*H*s_batch][trace_depth][3] (synchronizes). */
int32_t nrrs_set_trace(nrrs_ctx* ctx, int32_t enabled);
int32_t nrrs_read_trace(nrrs_ctx* ctx, double* host_rgb);

/* Precision of the network factor for the following renders (NRRS_PREC_FP32 / BF16 / FP8,
 * Sec. 5 "Network Architecture"; all three weight copies are kept current by every
 * parameter update, so a switch needs no conversion).  EINVAL for another value.  Captured
 * pass graphs are rebuilt on the next render. */
int32_t nrrs_set_precision(nrrs_ctx* ctx, int32_t precision);

/* How nrrs_render enqueues a pass: 1 (default) captures the pass's launch sequence once per
 * (max_depth, mode, records on/off) into a hipGraph and replays it for every pass; 0 launches
 * the kernels directly.  Per-stage timing, and a context on the null stream (which cannot be
 * captured), always launch directly. */
int32_t nrrs_set_launch_mode(nrrs_ctx* ctx, int32_t mode);

/* Enable (1) or disable (0) per-stage GPU timing of nrrs_render with HIP events recorded on
 * the context stream between the stages; results appear in nrrs_render_stats. */
int32_t nrrs_set_timing(nrrs_ctx* ctx, int32_t enabled);

/* Mix-Depth (Sec. 4.3): the RRS method is chosen per bounce.  In NET mode the network factor
 * is evaluated at depth d (1..64) when bit d-1 of net_depths is set; every other depth keeps the
 * heuristic factor lum(throughput * albedo), normalized the same way (Sec. 4.1 Eqs. 9-10).  The
 * table only changes inference: training records are still taken at depth <= net_max_depth.
 * The default after nrrs_create is (1 << net_max_depth) - 1.  Setting a different table drops
 * the captured pass graphs.  EINVAL on a NULL context or output. */
int32_t nrrs_set_mix_depth(nrrs_ctx* ctx, uint64_t net_depths);
int32_t nrrs_get_mix_depth(const nrrs_ctx* ctx, uint64_t* net_depths);

/* Mix-Depth's third method, the fixed rate (Sec. 4.3): at depth d with bit d-1 of fixed_depths
 * set, every vertex that continues gets the raw factor 1 in HEURISTIC and NET modes, so the
 * normalization gives all paths at that depth one rate.  It takes precedence over the network
 * bit of the same depth.  Default 0; setting a different value drops the captured pass graphs.
 * EINVAL on a NULL context or output. */
int32_t nrrs_set_mix_depth_fixed(nrrs_ctx* ctx, uint64_t fixed_depths);
int32_t nrrs_get_mix_depth_fixed(const nrrs_ctx* ctx, uint64_t* fixed_depths);

/* The pass index the next rendered pass takes (the second word of a primary path's lineage id,
 * so it selects the pass's random numbers; Sec. 3 wavefront passes).  It starts at 0 and each
 * pass advances it by one.  Setting it back renders a pass on the same random numbers again
 * (common random numbers for comparing RRS settings); the image is unaffected.  EINVAL beyond
 * 2^32 - 1. */
int32_t nrrs_set_pass_index(nrrs_ctx* ctx, uint64_t next_pass);
int32_t nrrs_get_pass_index(const nrrs_ctx* ctx, uint64_t* next_pass);

/* Launch parameters of the persistent traversal (extend) kernel.  The grid is
 * blocks_per_cu * (compute units) blocks of 128 lanes, each lane one ray at a time. */
typedef struct nrrs_tuning {
  uint32_t extend_variant;        /* 0: a lane intersects a hit leaf at once; 1: a lane parks
                                   * the leaf it reaches and waits, the wave intersects parked
                                   * leaves together; 2: as 1, but lanes with a parked leaf keep
                                   * descending meanwhile; 3: as 1, with the parked leaves'
                                   * triangles shared out over all lanes of the wave (four
                                   * lanes per leaf of at most 4 triangles); 4: as 3
                                   * over the 4-wide tree (EINVAL if the scene's 4-wide tree
                                   * is deeper than 30 levels) */
  uint32_t extend_blocks_per_cu;  /* 1 .. extend_max_blocks_per_cu[variant] */
  uint32_t extend_refill;         /* idle lanes of a wave (1..64) that make it fetch new rays */
  uint32_t extend_leaf_batch;     /* parked leaves (1..64) that trigger intersection (1-4) */
  uint32_t extend_chunk;          /* queue entries a wave claims per atomic (0: exactly what its
                                   * idle lanes need; else at least this many, up to 4096).
                                   * The queue is claimed in 8 contiguous slices with a counter
                                   * each; a wave starts in slice (block index mod 8) */
  uint32_t extend_max_blocks_per_cu[5]; /* out: occupancy limit of each variant (ignored by set) */
  float extend_ms;                /* out (nrrs_autotune): traversal time of the winner's pass */
} nrrs_tuning;

/* Current traversal launch parameters and the occupancy limits. */
int32_t nrrs_get_tuning(const nrrs_ctx* ctx, nrrs_tuning* out);

/* Set traversal launch parameters (EINVAL when out of range; the context is then unchanged).
 * Captured pass graphs are rebuilt on the next render. */
int32_t nrrs_set_tuning(nrrs_ctx* ctx, const nrrs_tuning* tuning);

/* Autotuner: times the traversal kernel of one heuristic-RRS pass of depth max_depth on the
 * uploaded scene for each candidate (variant x refill threshold, then fewer blocks per CU,
 * then the claim chunk, then the leaf batch) with HIP events, keeps the fastest and returns it in *best (may be NULL).
 * The first min(tried_cap, candidates) candidates with their times are written to tried
 * (caller-owned host array, may be NULL) and the candidate count to *n_tried (may be NULL).
 * The timing passes accumulate into the image, which is then cleared as by nrrs_reset_image;
 * they capture no training records.  Synchronous.  ESTATE without a scene. */
int32_t nrrs_autotune(nrrs_ctx* ctx, uint32_t max_depth, nrrs_tuning* best, nrrs_tuning* tried,
                      uint32_t tried_cap, uint32_t* n_tried);

/* Training records of the last render: count, and optionally (each may be NULL)
 * features[n*20], lum_t[n], acc[n] (descendant emission luminance), depth[n], pix[n],
 * lineage id[n] (64-bit).  The record order is not deterministic. */
int32_t nrrs_read_records(nrrs_ctx* ctx, uint64_t* n, float* features, float* lum_t, float* acc,
                          uint32_t* depth, uint32_t* pix, uint64_t* lineage);

/* --- test entry points: the same kernels on caller-provided inputs (host arrays) ----- */

/* Normalization, stochastic rounding, overflow guard and exclusive scan (Eqs. 8-14) of
 * n raw factors q_orig[n] whose uniforms come from Philox keyed by lineage ids
 * id_lo[n], id_hi[n] at `depth` (purpose 1).  budget_base is N_px; *alpha in/out.
 * Outputs X[n], offset[n], parent_of_child[S] (parent-major compaction), *S, *F,
 * q_norm[n] (may be NULL), *retries (alpha reductions applied).  cap is the queue capacity
 * (at most the context's).  *alpha must lie in (0, 1].  Returns EOVERFLOW (with *alpha and
 * *retries of the reduction that fell below 1e-3, S = 0) when no reduction fits. */
int32_t nrrs_debug_rrs_expand(nrrs_ctx* ctx, const float* q_orig, const uint32_t* id_lo,
                              const uint32_t* id_hi, uint32_t n, uint32_t depth, double budget_base,
                              double f_rate, double* alpha, int32_t norm_mode, uint32_t cap,
                              uint32_t* X, uint32_t* offset, uint32_t* parent_of_child,
                              uint32_t* S, double* F, float* q_norm, uint32_t* retries);

/* --- allocation-free variant of nrrs_debug_rrs_expand -------------------------------- */

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Computes what nrrs_debug_rrs_expand computes
 * (normalization, stochastic rounding, overflow guard, exclusive scan and parent map of one
 * depth, with the same kernels and the context's seed) on caller device arrays, queued on the
 * context's stream.  Its partial sums, block counts, guard candidates and control words live
 * in a fixed 320 KiB array of the library's own device memory, one per GPU, held until the
 * process ends; neither this call nor its kernels allocate, and the context needs no bound
 * workspace.
 *   q_dev[n]          device: raw factors, finite and >= 0 (device data, not checked)
 *   lineage_dev[2n]   device: lineage id (lo, hi) pairs keying the roulette uniforms
 *   offset_dev[n]     device out: first child slot of each entry (X_i = offset[i+1] - offset[i],
 *                     the last entry's X = S - offset[n-1])
 *   parent_dev[cap]   device out, may be NULL: the parent of each of the S children
 *   result_dev        device out: F, alpha after the guard, S, retries, overflow flag (1 when
 *                     alpha fell below 1e-3 before the children fit; then S = 0)
 * n and cap are limited to 2^31; depth 1..NRRS_MAX_DEPTH-1; alpha in (0, 1]; budget_base,
 * f_rate and norm_mode as for nrrs_debug_rrs_expand (EINVAL otherwise, nothing queued).
 * Asynchronous: returns once the work is queued.  Every call on a GPU uses that GPU's one
 * array and keeps the last call's contents; each call first sets the control words it reads.
 * Calls that overlap in time on one GPU (other streams or threads) race; calls in order on
 * one stream do not. */
typedef struct nrrs_expand_result {
  double F;          /* normalization factor used */
  double alpha;      /* adaptive rate after the guard */
  uint32_t S;        /* children emitted */
  uint32_t retries;  /* alpha reductions applied */
  uint32_t overflow; /* 1: no reduction fit before alpha fell below 1e-3 */
  uint32_t pad;
} nrrs_expand_result;
int32_t nrrs_rrs_expand_noalloc(nrrs_ctx* ctx, const float* q_dev, const uint32_t* lineage_dev, uint32_t n,
                                uint32_t depth, double budget_base, double f_rate, double alpha, int32_t norm_mode,
                                uint32_t cap, uint32_t* offset_dev, uint32_t* parent_dev,
                                nrrs_expand_result* result_dev);

/* Test entry point: normalization factors given by the caller.  With n > 0, renders in
 * HEURISTIC / NET mode use F[d-1] (host, finite, >= 0) at depth d = 1..n in place of the
 * factor of Eqs. (10)-(14) (the overflow guard then cannot lower it); renders deeper than
 * n + 1 return EINVAL.  n = 0 restores the computed factors.  The factor couples every path
 * of a depth, so a near-tie decision on one path moves it for all the others; a comparison
 * path by path against another implementation gives both the same factors.  Captured pass
 * graphs are rebuilt on the next render.  Synchronizes the stream. */
int32_t nrrs_debug_set_norm_factors(nrrs_ctx* ctx, const double* F, uint32_t n);

/* Replace the record buffer with n host records: features[n*20], lum_t[n], acc[n] (the
 * target is acc / lum_t).  ENOMEM if n > records_cap. */
int32_t nrrs_debug_load_records(nrrs_ctx* ctx, const float* features, const float* lum_t,
                                const float* acc, uint32_t n);

/* Copy the first n entries of queue `which` (0 or 1; a render's passes start in queue 0 and
 * the queues alternate by depth) and of the per-slot hit buffer of the last extended depth:
 * orig[n*4] (origin, excluded triangle bits), dir[n*4] (direction, pixel bits), thr[n*4]
 * (throughput, flag bits), hit[n*4] (t, b1, b2, triangle bits).  Any pointer may be NULL. */
int32_t nrrs_debug_read_queue(nrrs_ctx* ctx, int32_t which, uint32_t n, float* orig, float* dir,
                              float* thr, float* hit);

/* Closest hit of n rays[n*6] (origin, unit direction) against the uploaded scene, skipping
 * triangle exclude[n] (original index; 0xffffffff = none).  Outputs the original triangle
 * index (0xffffffff = miss), t, and barycentrics b1, b2. */
int32_t nrrs_debug_trace(nrrs_ctx* ctx, const float* rays, const uint32_t* exclude, uint32_t n,
                         uint32_t* prim, float* t, float* b1, float* b2);

/* Philox4x32-10 on n counters ctr[n*4] with key[2] -> out[n*4]. */
int32_t nrrs_debug_philox(nrrs_ctx* ctx, const uint32_t* ctr, const uint32_t* key, uint32_t n,
                          uint32_t* out);

/* Network forward y[n] (and raw output z[n], may be NULL) of features x[n*20] with the
 * current parameters in the given nrrs_precision. */
int32_t nrrs_debug_mlp_forward(nrrs_ctx* ctx, const float* x, uint32_t n, int32_t precision,
                               float* y, float* z);

/* The matrix-core forward of nrrs_debug_mlp_forward (precision NRRS_PREC_BF16 or NRRS_PREC_FP8
 * only), also giving the bit patterns of every quantized operand: codes[n][3][64] (host) holds
 * per row the inputs (0..19, the rest 0), hidden layer 1 and hidden layer 2 in unit order (BF16
 * bits, or the E4M3 code in the low byte), scale_exp[n][3] (host) the FP8 block-scale exponents
 * of those three operands (0 for BF16), y[n] the output.  Sec. 5 "Network Architecture". */
int32_t nrrs_debug_mlp_codes(nrrs_ctx* ctx, const float* x, uint32_t n, int32_t precision, float* y,
                             uint16_t* codes, int8_t* scale_exp);

/* Loss (the configured nrrs_loss) and its gradient grad[NRRS_NPARAM] over n (features x[n*20],
 * target[n]) rows with the current FP32 masters; no parameter update. */
int32_t nrrs_debug_mlp_grad(nrrs_ctx* ctx, const float* x, const float* target, uint32_t n,
                            float* grad, float* loss);

/* Status text (static storage) and the context's last error message (valid until the next
 * call on ctx). */
const char* nrrs_status_string(int32_t status);
const char* nrrs_last_error(const nrrs_ctx* ctx);

/* Destroy a context (NULL is ignored).  Does not free the caller's workspace. */
void nrrs_destroy(nrrs_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* NRRS_H */
