/* FP64 CPU oracle of the normalized-RRS wavefront path tracer (NRRS, arXiv 2510.07868).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product path.  It shares no code
 * with the HIP library.  Everything is double precision and written as plain
 * loops in the order the paper states the steps.  The only float32 step is the
 * rounding of the normalized RRS factor that decides the integer child count:
 * that decision is taken in the precision the kernels use (Eq. 8 with q_norm
 * rounded to float32), and the same rounded factor weights the children, so the
 * estimator stays unbiased.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter =
 * (lineage id low, lineage id high, purpose | depth << 8, child index), key =
 * the 64-bit seed.  A primary path's lineage id is (path index in the pass, pass);
 * a child's id is words 2..3 of the Philox block that also gives its BSDF
 * sample, so a path's random numbers do not depend on where it sits in a queue.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MISS 0xffffffffu
#define MAXREC 4
#define PURPOSE_CAMERA 0u
#define PURPOSE_ROULETTE 1u
#define PURPOSE_CHILD 2u
#define PURPOSE_TRAIN 3u
#define PURPOSE_NEE 4u

static const double LUM[3] = {0.2126, 0.7152, 0.0722}; /* Rec. 709 luminance */

/* ------------------------------------------------------------------ Philox */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_philox_batch(const uint32_t* ctr, const uint32_t key[2], uint64_t n, uint32_t* out) {
  for (uint64_t i = 0; i < n; ++i) or_philox(ctr + 4 * i, key, out + 4 * i);
}

static double u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

static void rng_block(uint64_t seed, uint32_t id_lo, uint32_t id_hi, uint32_t purpose, uint32_t depth,
                      uint32_t j, uint32_t out[4]) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {id_lo, id_hi, purpose | (depth << 8), j};
  or_philox(ctr, key, out);
}

/* ------------------------------------------------------------ vector math */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static void sub3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2];
}
static void normalize3(double a[3]) {
  double l = sqrt(dot3(a, a));
  a[0] /= l; a[1] /= l; a[2] /= l;
}
static double lum3(const double c[3]) { return LUM[0] * c[0] + LUM[1] * c[1] + LUM[2] * c[2]; }

/* Orthonormal basis around unit n (Duff et al., "Building an Orthonormal Basis, Revisited", 2017). */
static void onb(const double n[3], double t[3], double b[3]) {
  double sign = n[2] >= 0.0 ? 1.0 : -1.0;
  double a = -1.0 / (sign + n[2]);
  double c = n[0] * n[1] * a;
  t[0] = 1.0 + sign * n[0] * n[0] * a; t[1] = sign * c; t[2] = -sign * n[0];
  b[0] = c; b[1] = sign + n[1] * n[1] * a; b[2] = -n[1];
}

/* ------------------------------------------------------------------ scene */
typedef struct {
  double lo[3], hi[3];
  uint32_t left, right, first, count; /* count > 0: leaf over order[first..first+count) */
} bnode;

struct or_scene {
  uint64_t nt;
  double* tri;      /* nt * 9: v0, v1, v2 */
  uint32_t* tmat;
  uint32_t nm;
  uint32_t* mtype;
  double* mpar;     /* nm * 7 */
  double cam[10];
  double env[3];
  double amin[3], amax[3], extent, diag, tmin, offset;
  double perr_max;  /* float32 position error up to which paths are compared (near-tie flags only) */
  bnode* nodes;
  uint64_t nnodes;
  uint32_t* order;
  /* lights for next-event estimation: the triangles whose material emits, chosen with
   * probability proportional to lum(L_e) x area (CDF over them), a point uniform on the chosen
   * triangle; lpdf[p] = that probability per unit area (lum(L_e) / sum), 0 for non-emitters */
  uint32_t nl;
  uint32_t* light_tri;
  double* light_cdf;  /* nl + 1 entries, 0 .. 1 */
  double* lpdf;       /* nt */
};

static void tri_bounds(const or_scene* s, uint32_t p, double lo[3], double hi[3]) {
  const double* v = s->tri + 9 * (uint64_t)p;
  for (int a = 0; a < 3; ++a) {
    lo[a] = fmin(v[a], fmin(v[3 + a], v[6 + a]));
    hi[a] = fmax(v[a], fmax(v[3 + a], v[6 + a]));
  }
}

static double centroid(const or_scene* s, uint32_t p, int axis) {
  const double* v = s->tri + 9 * (uint64_t)p;
  return (v[axis] + v[3 + axis] + v[6 + axis]) / 3.0;
}

static void quickselect(const or_scene* s, uint32_t* a, int64_t n, int64_t k, int axis) {
  int64_t lo = 0, hi = n - 1;
  while (hi > lo) {
    double pv = centroid(s, a[lo + (hi - lo) / 2], axis);
    int64_t i = lo, j = hi;
    while (i <= j) {
      while (centroid(s, a[i], axis) < pv) ++i;
      while (centroid(s, a[j], axis) > pv) --j;
      if (i <= j) {
        uint32_t t = a[i]; a[i] = a[j]; a[j] = t;
        ++i; --j;
      }
    }
    if (k <= j) hi = j;
    else if (k >= i) lo = i;
    else return;
  }
}

static uint32_t bvh_build(or_scene* s, uint64_t a, uint64_t b) {
  uint32_t id = (uint32_t)s->nnodes++;
  bnode* nd = &s->nodes[id];
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = 0; k < 3; ++k) { nd->lo[k] = INFINITY; nd->hi[k] = -INFINITY; }
  for (uint64_t i = a; i < b; ++i) {
    double lo[3], hi[3];
    tri_bounds(s, s->order[i], lo, hi);
    for (int k = 0; k < 3; ++k) {
      nd->lo[k] = fmin(nd->lo[k], lo[k]);
      nd->hi[k] = fmax(nd->hi[k], hi[k]);
      double c = centroid(s, s->order[i], k);
      clo[k] = fmin(clo[k], c);
      chi[k] = fmax(chi[k], c);
    }
  }
  int axis = 0;
  for (int k = 1; k < 3; ++k)
    if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
  if (b - a <= 4 || chi[axis] - clo[axis] <= 0.0) {
    nd->first = (uint32_t)a;
    nd->count = (uint32_t)(b - a);
    nd->left = nd->right = 0;
    return id;
  }
  uint64_t mid = (a + b) / 2;
  quickselect(s, s->order + a, (int64_t)(b - a), (int64_t)(mid - a), axis);
  nd->count = 0;
  uint32_t l = bvh_build(s, a, mid);
  uint32_t r = bvh_build(s, mid, b);
  s->nodes[id].left = l;
  s->nodes[id].right = r;
  return id;
}

static double tri_altitude(const or_scene* s, uint32_t p);
static int cmp_double(const void* a, const void* b) {
  const double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

or_scene* or_scene_create(const float* verts, uint64_t nv, const uint32_t* tris, uint64_t nt,
                          const uint32_t* tri_mat, const uint32_t* mat_type, const float* mat_params,
                          uint32_t nm, const float* camera, const float* env, int32_t build_bvh) {
  if (nt == 0 || nm == 0) return NULL;
  or_scene* s = (or_scene*)calloc(1, sizeof(or_scene));
  s->nt = nt;
  s->tri = (double*)malloc(sizeof(double) * 9 * nt);
  s->tmat = (uint32_t*)malloc(sizeof(uint32_t) * nt);
  for (int k = 0; k < 3; ++k) { s->amin[k] = INFINITY; s->amax[k] = -INFINITY; }
  for (uint64_t i = 0; i < nt; ++i) {
    for (int c = 0; c < 3; ++c) {
      uint32_t vi = tris[3 * i + c];
      if (vi >= nv) { or_scene_destroy(s); return NULL; }
      for (int k = 0; k < 3; ++k) {
        double x = (double)verts[3 * (uint64_t)vi + k];
        s->tri[9 * i + 3 * c + k] = x;
        s->amin[k] = fmin(s->amin[k], x);
        s->amax[k] = fmax(s->amax[k], x);
      }
    }
    s->tmat[i] = tri_mat[i];
    if (tri_mat[i] >= nm) { or_scene_destroy(s); return NULL; }
  }
  s->nm = nm;
  s->mtype = (uint32_t*)malloc(sizeof(uint32_t) * nm);
  s->mpar = (double*)malloc(sizeof(double) * 7 * nm);
  for (uint32_t m = 0; m < nm; ++m) {
    s->mtype[m] = mat_type[m];
    for (int k = 0; k < 7; ++k) s->mpar[7 * m + k] = (double)mat_params[7 * m + k];
  }
  for (int k = 0; k < 10; ++k) s->cam[k] = (double)camera[k];
  for (int k = 0; k < 3; ++k) s->env[k] = (double)env[k];
  double e[3];
  sub3(s->amax, s->amin, e);
  s->extent = fmax(e[0], fmax(e[1], e[2]));
  s->diag = sqrt(dot3(e, e));
  s->tmin = 0.0;                   /* hits count for t > 0; child origins are offset instead */
  s->offset = 1e-5 * s->extent;     /* origin offset along the face-forwarded normal */
  /* A quarter of the median triangle altitude: a float32 ray whose position error stays below
   * it is traced with box paddings of at most that much; beyond it the near-tie flags stop
   * comparing the path (median over at most 4096 evenly spaced triangles). */
  {
    const uint64_t ns = nt < 4096 ? nt : 4096;
    double* h = (double*)malloc(sizeof(double) * (ns ? ns : 1));
    for (uint64_t k = 0; k < ns; ++k) h[k] = tri_altitude(s, (uint32_t)(k * (nt / ns)));
    qsort(h, ns, sizeof(double), cmp_double);
    s->perr_max = ns ? 0.25 * h[ns / 2] : 0.0;
    free(h);
  }
  {
    s->lpdf = (double*)calloc(nt, sizeof(double));
    s->light_tri = (uint32_t*)malloc(sizeof(uint32_t) * nt);
    s->light_cdf = (double*)malloc(sizeof(double) * (nt + 1));
    double total = 0.0;
    s->nl = 0;
    s->light_cdf[0] = 0.0;
    for (uint64_t i = 0; i < nt; ++i) {
      const double* mp = s->mpar + 7 * (uint64_t)s->tmat[i];
      const double le = lum3(mp + 4);
      if (!(le > 0.0)) continue;
      const double* v = s->tri + 9 * i;
      double e1[3], e2[3], cr[3];
      sub3(v + 3, v, e1);
      sub3(v + 6, v, e2);
      cross3(e1, e2, cr);
      const double area = 0.5 * sqrt(dot3(cr, cr));
      if (!(area > 0.0)) continue;
      total += le * area;
      s->light_tri[s->nl] = (uint32_t)i;
      s->light_cdf[++s->nl] = total;
    }
    for (uint32_t k = 1; k <= s->nl; ++k) s->light_cdf[k] /= total;
    for (uint32_t k = 0; k < s->nl; ++k) {
      const uint32_t i = s->light_tri[k];
      s->lpdf[i] = lum3(s->mpar + 7 * (uint64_t)s->tmat[i] + 4) / total;
    }
  }
  if (build_bvh) {
    s->order = (uint32_t*)malloc(sizeof(uint32_t) * nt);
    for (uint64_t i = 0; i < nt; ++i) s->order[i] = (uint32_t)i;
    s->nodes = (bnode*)malloc(sizeof(bnode) * 2 * nt);
    s->nnodes = 0;
    bvh_build(s, 0, nt);
  }
  return s;
}

void or_scene_destroy(or_scene* s) {
  if (!s) return;
  free(s->tri); free(s->tmat); free(s->mtype); free(s->mpar); free(s->nodes); free(s->order);
  free(s->lpdf); free(s->light_tri); free(s->light_cdf);
  free(s);
}

/* ------------------------------------------------------------ intersection */
/* Moller-Trumbore (1997).  Returns 0 for a ray parallel to the plane, else 1 with t, b1, b2,
 * the signed barycentric margin (min of the three weights) and |cos| of the angle between the
 * ray and the triangle's normal: float32 barycentrics and distances carry errors growing as
 * 1/|cos|, so near-tie tests scale their margins by it. */
static int tri_test(const or_scene* s, uint32_t p, const double o[3], const double d[3], double* t,
                    double* b1, double* b2, double* margin, double* cosn) {
  const double* v = s->tri + 9 * (uint64_t)p;
  double e1[3], e2[3], pv[3], sv[3], qv[3];
  sub3(v + 3, v, e1);
  sub3(v + 6, v, e2);
  cross3(d, e2, pv);
  double det = dot3(e1, pv);
  if (det == 0.0) return 0;
  double inv = 1.0 / det;
  sub3(o, v, sv);
  *b1 = dot3(sv, pv) * inv;
  cross3(sv, e1, qv);
  *b2 = dot3(d, qv) * inv;
  *t = dot3(e2, qv) * inv;
  *margin = fmin(*b1, fmin(*b2, 1.0 - *b1 - *b2));
  double nv[3];
  cross3(e1, e2, nv);
  *cosn = fabs(det) / sqrt(dot3(nv, nv));
  return 1;
}

typedef struct {
  uint32_t prim;
  double t, b1, b2, margin, cosn;  /* margin of the winner, scaled by its |cos| */
  double gm;                       /* the winner's margin equivalent of the ray's position error */
  int ncand;
  double cand_t[16], cand_c[16], cand_e[16];
  uint32_t cand_p[16];
  double perr, derr;               /* float32 error bounds of the ray: origin (m), direction (rad) */
} trace_state;

/* Smallest altitude of triangle p: a position error e along its plane moves the barycentric
 * coordinates by at most e / h. */
static double tri_altitude(const or_scene* s, uint32_t p) {
  const double* v = s->tri + 9 * (uint64_t)p;
  double e1[3], e2[3], e3[3], nv[3];
  sub3(v + 3, v, e1);
  sub3(v + 6, v, e2);
  sub3(v + 6, v + 3, e3);
  cross3(e1, e2, nv);
  double L = fmax(sqrt(dot3(e1, e1)), fmax(sqrt(dot3(e2, e2)), sqrt(dot3(e3, e3))));
  return L > 0.0 ? sqrt(dot3(nv, nv)) / L : 0.0;
}

static void consider(const or_scene* s, uint32_t p, const double o[3], const double d[3], uint32_t excl,
                     double tau, trace_state* st) {
  if (p == excl) return;
  double t, b1, b2, m, cn;
  if (!tri_test(s, p, o, d, &t, &b1, &b2, &m, &cn)) return;
  /* position error of the float32 ray where it meets this triangle's plane (perpendicular to the
   * ray; in the m * cos units of the margins: e / altitude) */
  const double err = tau > 0.0 ? st->perr + fabs(t) * st->derr : 0.0;
  const double h = tau > 0.0 ? tri_altitude(s, p) : 0.0;
  const double g = err > 0.0 ? (h > 0.0 ? err / h : INFINITY) : 0.0;
  if (m >= 0.0 && t > s->tmin) {
    if (t < st->t || (t == st->t && p < st->prim)) {
      st->prim = p; st->t = t; st->b1 = b1; st->b2 = b2; st->margin = m * cn; st->cosn = cn; st->gm = g;
    }
  }
  if (tau > 0.0 && m * cn > -(tau + g) && t > s->tmin - (tau * s->diag + err) / fmax(cn, 1e-300)) {
    /* keep the 16 nearest candidates; a farther one cannot decide a near-tie that these miss */
    if (st->ncand < 16) {
      st->cand_t[st->ncand] = t;
      st->cand_c[st->ncand] = cn;
      st->cand_e[st->ncand] = err;
      st->cand_p[st->ncand] = p;
      st->ncand++;
    } else {
      int far = 0;
      for (int i = 1; i < 16; ++i)
        if (st->cand_t[i] > st->cand_t[far]) far = i;
      if (t < st->cand_t[far]) {
        st->cand_t[far] = t;
        st->cand_c[far] = cn;
        st->cand_e[far] = err;
        st->cand_p[far] = p;
      }
    }
  }
}

static int box_hit(const bnode* nd, const double o[3], const double d[3], double tlim, double pad_rel,
                   double pad_abs) {
  double tn = 0.0, tf = tlim;
  for (int a = 0; a < 3; ++a) {
    double ext = nd->hi[a] - nd->lo[a];
    double pad = 1e-7 * (fabs(nd->lo[a]) + fabs(nd->hi[a]) + ext) + pad_rel * ext + pad_abs;
    double lo = nd->lo[a] - pad, hi = nd->hi[a] + pad;
    if (d[a] == 0.0) {
      if (o[a] < lo || o[a] > hi) return 0;
      continue;
    }
    double t0 = (lo - o[a]) / d[a], t1 = (hi - o[a]) / d[a];
    if (t0 > t1) { double x = t0; t0 = t1; t1 = x; }
    if (t0 > tn) tn = t0;
    if (t1 < tf) tf = t1;
    if (tn > tf) return 0;
  }
  return 1;
}

/* Closest hit with t > tmin, excluding prim `excl`; ties go to the smaller prim id.
 * Returns 1 when the decision is within `tau` of changing (near-tie), widened by what the
 * float32 ray's own error could move: its origin by up to perr (m) and its direction by up to
 * derr (rad).  *gerr receives that position error at the hit, perpendicular to the ray. */
static int trace_one(const or_scene* s, const double o[3], const double d[3], uint32_t excl, int use_bvh,
                     double tau, double perr, double derr, uint32_t* prim, double* t, double* b1, double* b2,
                     double* gerr) {
  trace_state st;
  st.prim = MISS; st.t = INFINITY; st.b1 = st.b2 = 0.0; st.margin = 0.0; st.cosn = 1.0; st.gm = 0.0; st.ncand = 0;
  st.perr = perr; st.derr = derr;
  if (use_bvh && s->nodes) {
    uint32_t stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
      const bnode* nd = &s->nodes[stack[--sp]];
      double lim = st.t + (tau > 0.0 ? tau * s->diag : 0.0);
      double pad_abs = tau > 0.0 ? perr + (isinf(lim) ? s->diag : lim) * derr : 0.0;
      if (!box_hit(nd, o, d, isinf(lim) ? INFINITY : lim * (1.0 + 1e-9) + 1e-12 + pad_abs, tau, pad_abs)) continue;
      if (nd->count > 0) {
        for (uint32_t i = 0; i < nd->count; ++i) consider(s, s->order[nd->first + i], o, d, excl, tau, &st);
      } else {
        stack[sp++] = nd->left;
        stack[sp++] = nd->right;
      }
    }
  } else {
    for (uint64_t p = 0; p < s->nt; ++p) consider(s, (uint32_t)p, o, d, excl, tau, &st);
  }
  *prim = st.prim; *t = st.t; *b1 = st.b1; *b2 = st.b2;
  if (gerr) *gerr = st.prim != MISS ? perr + st.t * derr : 0.0;
  if (tau <= 0.0) return 0;
  const double werr = st.prim != MISS ? perr + st.t * derr : 0.0;
  if (st.prim != MISS && (st.margin < tau + st.gm || st.t < s->tmin + tau * s->diag + werr / fmax(st.cosn, 1e-300)))
    return 1;
  for (int i = 0; i < st.ncand; ++i) {
    if (st.cand_p[i] == st.prim) continue;
    if (st.prim == MISS ||
        (st.cand_t[i] - st.t) * fmin(st.cand_c[i], st.cosn) < tau * s->diag + st.cand_e[i] + werr)
      return 1;
  }
  return 0;
}

void or_trace(const or_scene* s, const double* rays, const uint32_t* exclude, uint64_t n, uint32_t* prim,
              double* t, double* b1, double* b2, int32_t use_bvh, double tau, uint8_t* fragile) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    double o[3] = {rays[6 * i], rays[6 * i + 1], rays[6 * i + 2]};
    double d[3] = {rays[6 * i + 3], rays[6 * i + 4], rays[6 * i + 5]};
    int f = trace_one(s, o, d, exclude ? exclude[i] : MISS, use_bvh, tau, 0.0, 0.0, &prim[i], &t[i], &b1[i], &b2[i],
                      NULL);
    if (fragile) fragile[i] = (uint8_t)f;
  }
}

/* ----------------------------------------------------------------- BSDFs */
/* GGX / Trowbridge-Reitz normal distribution, Smith Lambda for GGX, local frame n = +z. */
double or_ggx_D(double alpha, const double h[3]) {
  if (h[2] <= 0.0) return 0.0;
  double a2 = alpha * alpha;
  double c2 = h[2] * h[2];
  double den = c2 * (a2 - 1.0) + 1.0;
  return a2 / (M_PI * den * den);
}

static double ggx_lambda(double alpha, const double w[3]) {
  double c2 = w[2] * w[2];
  double s2 = fmax(0.0, 1.0 - c2);
  if (s2 == 0.0) return 0.0;
  double tan2 = s2 / c2;
  return 0.5 * (-1.0 + sqrt(1.0 + alpha * alpha * tan2));
}

double or_ggx_G1(double alpha, const double w[3]) { return 1.0 / (1.0 + ggx_lambda(alpha, w)); }

/* Height-correlated Smith masking-shadowing. */
double or_ggx_G2(double alpha, const double wo[3], const double wi[3]) {
  return 1.0 / (1.0 + ggx_lambda(alpha, wo) + ggx_lambda(alpha, wi));
}

static double schlick(double f0, double c) {
  double m = 1.0 - c;
  double m2 = m * m;
  return f0 + (1.0 - f0) * m2 * m2 * m;
}

/* f * cos(theta_i) of the Cook-Torrance GGX model (scalar F0). */
double or_ggx_eval_cos(double alpha, double f0, const double wo[3], const double wi[3]) {
  if (wo[2] <= 0.0 || wi[2] <= 0.0) return 0.0;
  double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
  normalize3(h);
  double f = or_ggx_D(alpha, h) * or_ggx_G2(alpha, wo, wi) * schlick(f0, dot3(wo, h)) / (4.0 * wo[2] * wi[2]);
  return f * wi[2];
}

/* Visible-normal sampling (Heitz, "Sampling the GGX Distribution of Visible Normals", JCGT 2018),
 * written from the published construction: stretch wo, sample the projected hemisphere, unstretch. */
static void ggx_sample_vndf(double alpha, const double wo[3], double u1, double u2, double h[3]) {
  double vh[3] = {alpha * wo[0], alpha * wo[1], wo[2]};
  normalize3(vh);
  double lensq = vh[0] * vh[0] + vh[1] * vh[1];
  double t1[3], t2[3];
  if (lensq > 0.0) {
    double il = 1.0 / sqrt(lensq);
    t1[0] = -vh[1] * il; t1[1] = vh[0] * il; t1[2] = 0.0;
  } else {
    t1[0] = 1.0; t1[1] = 0.0; t1[2] = 0.0;
  }
  cross3(vh, t1, t2);
  double r = sqrt(u1);
  double phi = 2.0 * M_PI * u2;
  double p1 = r * cos(phi);
  double p2 = r * sin(phi);
  double sh = 0.5 * (1.0 + vh[2]);
  p2 = (1.0 - sh) * sqrt(fmax(0.0, 1.0 - p1 * p1)) + sh * p2;
  double p3 = sqrt(fmax(0.0, 1.0 - p1 * p1 - p2 * p2));
  double nh[3];
  for (int k = 0; k < 3; ++k) nh[k] = p1 * t1[k] + p2 * t2[k] + p3 * vh[k];
  h[0] = alpha * nh[0]; h[1] = alpha * nh[1]; h[2] = fmax(0.0, nh[2]);
  normalize3(h);
}

int32_t or_ggx_sample(double alpha, double f0, const double wo[3], double u1, double u2, double wi[3],
                      double* weight, double* pdf) {
  double h[3];
  ggx_sample_vndf(alpha, wo, u1, u2, h);
  double c = dot3(wo, h);
  for (int k = 0; k < 3; ++k) wi[k] = 2.0 * c * h[k] - wo[k];
  *pdf = or_ggx_G1(alpha, wo) * or_ggx_D(alpha, h) / (4.0 * wo[2]);
  if (wi[2] <= 0.0) { *weight = 0.0; return 0; }
  *weight = schlick(f0, c) * or_ggx_G2(alpha, wo, wi) / or_ggx_G1(alpha, wo);
  return 1;
}

void or_lambert_sample(double u1, double u2, double wi[3], double* pdf) {
  double r = sqrt(u1);
  double phi = 2.0 * M_PI * u2;
  wi[0] = r * cos(phi);
  wi[1] = r * sin(phi);
  wi[2] = sqrt(fmax(0.0, 1.0 - u1));
  *pdf = wi[2] / M_PI;
}

/* Solid-angle pdf of visible-normal GGX sampling for the direction wi (local frame). */
static double ggx_pdf(double alpha, const double wo[3], const double wi[3]) {
  if (wo[2] <= 0.0 || wi[2] <= 0.0) return 0.0;
  double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
  normalize3(h);
  return or_ggx_G1(alpha, wo) * or_ggx_D(alpha, h) / (4.0 * wo[2]);
}

double or_ggx_pdf(double alpha, const double wo[3], const double wi[3]) { return ggx_pdf(alpha, wo, wi); }

/* ---------------------------------------------------------------- network */
#define W1 0
#define B1 1280
#define W2 1344
#define B2 5440
#define W3 5504
#define B3 9600
#define W4 9664
#define B4 9728

/* Eq. (22): ln(1+e^z) below zero, 0.5 z + ln 2 at and above zero. */
double or_softplus_mod(double z) { return z < 0.0 ? log1p(exp(z)) : 0.5 * z + M_LN2; }
double or_softplus_mod_grad(double z) { return z < 0.0 ? 1.0 / (1.0 + exp(-z)) : 0.5; }

static void mlp_row(const double* P, const double* x, double a1[64], double a2[64], double a3[64], double* z) {
  for (int o = 0; o < 64; ++o) {
    double acc = P[B1 + o];
    for (int i = 0; i < 20; ++i) acc += P[W1 + 20 * o + i] * x[i];
    a1[o] = acc;
  }
  for (int o = 0; o < 64; ++o) {
    double acc = P[B2 + o];
    for (int i = 0; i < 64; ++i) acc += P[W2 + 64 * o + i] * fmax(a1[i], 0.0);
    a2[o] = acc;
  }
  for (int o = 0; o < 64; ++o) {
    double acc = P[B3 + o];
    for (int i = 0; i < 64; ++i) acc += P[W3 + 64 * o + i] * fmax(a2[i], 0.0);
    a3[o] = acc;
  }
  double acc = P[B4];
  for (int i = 0; i < 64; ++i) acc += P[W4 + i] * fmax(a3[i], 0.0);
  *z = acc;
}

void or_mlp_forward(const double* params, const double* x, uint64_t n, double* y, double* z) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < (int64_t)n; ++r) {
    double a1[64], a2[64], a3[64], zz;
    mlp_row(params, x + 20 * r, a1, a2, a3, &zz);
    if (z) z[r] = zz;
    y[r] = or_softplus_mod(zz);
  }
}

double or_mlp_loss_grad(const double* params, const double* x, const double* target, uint64_t n, double eps,
                        int32_t kind, double* grad) {
  memset(grad, 0, sizeof(double) * OR_NPARAM);
  double loss = 0.0;
  for (uint64_t r = 0; r < n; ++r) {
    const double* xr = x + 20 * r;
    double a1[64], a2[64], a3[64], z;
    mlp_row(params, xr, a1, a2, a3, &z);
    double y = or_softplus_mod(z);
    double dy;
    if (kind == OR_LOSS_LOG_MSE) {
      /* (ln(y + eps) - ln(L + eps))^2 */
      double diff = log(y + eps) - log(target[r] + eps);
      loss += diff * diff;
      dy = 2.0 * diff / (y + eps);
    } else {
      /* relative L2 with the prediction held constant in the denominator (Sec. 4.2.2, Eq. 15) */
      double den = y * y + eps;
      double diff = y - target[r];
      loss += diff * diff / den;
      dy = 2.0 * diff / den;
    }
    double dz = dy / (double)n * or_softplus_mod_grad(z);
    double d3[64], d2[64], d1[64];
    grad[B4] += dz;
    for (int i = 0; i < 64; ++i) {
      grad[W4 + i] += dz * fmax(a3[i], 0.0);
      d3[i] = a3[i] > 0.0 ? dz * params[W4 + i] : 0.0;
    }
    for (int o = 0; o < 64; ++o) {
      grad[B3 + o] += d3[o];
      for (int i = 0; i < 64; ++i) grad[W3 + 64 * o + i] += d3[o] * fmax(a2[i], 0.0);
    }
    for (int i = 0; i < 64; ++i) {
      double acc = 0.0;
      for (int o = 0; o < 64; ++o) acc += params[W3 + 64 * o + i] * d3[o];
      d2[i] = a2[i] > 0.0 ? acc : 0.0;
    }
    for (int o = 0; o < 64; ++o) {
      grad[B2 + o] += d2[o];
      for (int i = 0; i < 64; ++i) grad[W2 + 64 * o + i] += d2[o] * fmax(a1[i], 0.0);
    }
    for (int i = 0; i < 64; ++i) {
      double acc = 0.0;
      for (int o = 0; o < 64; ++o) acc += params[W2 + 64 * o + i] * d2[o];
      d1[i] = a1[i] > 0.0 ? acc : 0.0;
    }
    for (int o = 0; o < 64; ++o) {
      grad[B1 + o] += d1[o];
      for (int i = 0; i < 20; ++i) grad[W1 + 20 * o + i] += d1[o] * xr[i];
    }
  }
  return loss / (double)n;
}

/* ---------------------------------------------- reduced-precision network evaluation */
/* float -> bfloat16 -> float with round to nearest, ties to even (on the float's bits). */
double or_round_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  uint32_t lower = u & 0xFFFFu, upper = u >> 16;
  if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u))) upper += 1;
  u = upper << 16;
  memcpy(&f, &u, 4);
  return (double)f;
}

/* Value of the nearest OCP E4M3 number (max 448, 3 mantissa bits, subnormals 2^-9 apart)
 * to x, ties to even, saturating at +-448. */
double or_round_e4m3(double x) {
  double a = fabs(x);
  double s = x < 0 ? -1.0 : 1.0;
  if (a >= 448.0) return s * 448.0;
  if (a < ldexp(1.0, -6)) {  /* subnormal grid */
    double q = a / ldexp(1.0, -9);
    double r = nearbyint(q);  /* default rounding mode: ties to even */
    return s * r * ldexp(1.0, -9);
  }
  int e;
  frexp(a, &e);               /* a = m 2^e, m in [0.5, 1) -> a in [2^(e-1), 2^e) */
  double ulp = ldexp(1.0, e - 1 - 3);
  double r = nearbyint(a / ulp) * ulp;
  if (r > 448.0) r = 448.0;
  return s * r;
}

/* Distance of x to the nearest rounding midpoint of the bfloat16 grid, in units of the grid
 * spacing at x (0 = exactly on a midpoint, 0.5 = on a grid point). */
static double midpoint_gap_bf16(double x) {
  double a = fabs(x);
  if (a == 0.0) return 0.5;
  int e;
  frexp(a, &e);
  double ulp = ldexp(1.0, e - 1 - 7);
  double f = a / ulp - floor(a / ulp);
  return fabs(f - 0.5);
}

/* Power-of-two scale 2^e, e the smallest integer with 2^e >= amax / 448 (float quotient). */
static double block_scale(double amax) {
  float r = (float)amax / 448.0f;
  if (!(r > 0.0f)) return 1.0;
  int ex;
  float m = frexpf(r, &ex);
  int e = (m == 0.5f) ? ex - 1 : ex;
  if (e < -120) e = -120;
  if (e > 120) e = 120;
  return ldexp(1.0, e);
}

/* Absolute distance of x (>= 0, in E4M3 units) to the nearest E4M3 rounding midpoint. */
static double midpoint_dist_e4m3(double x) {
  double a = fabs(x);
  if (a >= 448.0) return INFINITY;
  double ulp;
  if (a < ldexp(1.0, -6)) ulp = ldexp(1.0, -9);
  else {
    int e;
    frexp(a, &e);
    ulp = ldexp(1.0, e - 1 - 3);
  }
  double f = a / ulp - floor(a / ulp);
  return fabs(f - 0.5) * ulp;
}

/* Bound on how far an FP8 matrix-core dot product sum_k w_k x_k (E4M3 codes, exact products)
 * can land from its exact value.  The FP8 matrix core does not add every product in FP32: it
 * aligns each small group of products to the group's largest one and drops the bits more than
 * 13 binary places below it, then adds the group sums in FP32.  Bounding every group's largest
 * product by the largest product overall: a product that is not a multiple of
 * 2^(floor(log2 max|p|) - 13) may lose up to that unit, plus FP32 rounding of the group sums. */
static double fp8_dot_error_bound(const double* w, const double* x, int n) {
  double pmax = 0.0, sabs = 0.0;
  for (int k = 0; k < n; ++k) {
    double p = fabs(w[k] * x[k]);
    pmax = fmax(pmax, p);
    sabs += p;
  }
  if (pmax == 0.0) return 0.0;
  int e;
  frexp(pmax, &e); /* pmax in [2^(e-1), 2^e) */
  const double unit = ldexp(1.0, e - 1 - 13);
  double b = 0.0;
  for (int k = 0; k < n; ++k) {
    double p = fabs(w[k] * x[k]);
    if (fmod(p, unit) != 0.0) b += fmin(p, unit);
  }
  return b + 16.0 * ldexp(1.0, -24) * sabs;
}

/* Bit patterns of values already on the E4M3 / BF16 grids (the codes the matrix cores read). */
static uint16_t e4m3_bits(double v) {
  uint16_t sign = signbit(v) ? 0x80 : 0; /* a negative value rounded to zero keeps its sign */
  double a = fabs(v);
  if (a == 0.0) return sign;
  int e;
  double m = frexp(a, &e); /* a = m 2^e, m in [0.5, 1) */
  int be = e - 1 + 7;      /* biased exponent of 1.xxx 2^(e-1) */
  if (be <= 0) return (uint16_t)(sign | (uint16_t)nearbyint(a * 512.0)); /* subnormal: k 2^-9 */
  int mant = (int)nearbyint((m * 2.0 - 1.0) * 8.0);
  return (uint16_t)(sign | (be << 3) | mant);
}
static uint16_t bf16_bits(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}

double or_fp8_dot_error_bound(const double* w, const double* x, int32_t n) {
  return fp8_dot_error_bound(w, x, n);
}

void or_mlp_forward_quant(const double* params, const double* x, uint64_t n, int32_t prec, double* y, double* z,
                          uint8_t* fragile) {
  or_mlp_forward_quant_codes(params, x, n, prec, y, z, fragile, NULL, NULL, NULL);
}

void or_mlp_forward_quant_codes(const double* params, const double* x, uint64_t n, int32_t prec, double* y,
                                double* z, uint8_t* fragile, uint16_t* codes, uint8_t* near_act, int8_t* scale_exp) {
  /* BF16: rounding decisions this close to a midpoint (in grid steps) are near-ties, a few
   * times the FP32 accumulation error relative to the grid's spacing.  FP8: a decision is a
   * near-tie when the midpoint lies within fp8_dot_error_bound of the exact pre-activation. */
  const double gap = 2e-4;
  /* quantized weight copies */
  static const int woff[3] = {W1, W2, W3}, wcnt[3] = {1280, 4096, 4096};
  double* Wq = (double*)malloc(sizeof(double) * OR_NPARAM);
  memcpy(Wq, params, sizeof(double) * OR_NPARAM);
  double wscale[3] = {1.0, 1.0, 1.0};
  for (int L = 0; L < 3; ++L) {
    if (prec == 1) {
      for (int k = 0; k < wcnt[L]; ++k) Wq[woff[L] + k] = or_round_bf16(params[woff[L] + k]);
    } else {
      float amax = 0.0f;
      for (int k = 0; k < wcnt[L]; ++k) amax = fmaxf(amax, fabsf((float)params[woff[L] + k]));
      float sc = amax > 0.0f ? amax / 448.0f : 1.0f;
      wscale[L] = (double)sc;
      for (int k = 0; k < wcnt[L]; ++k) Wq[woff[L] + k] = or_round_e4m3((double)((float)params[woff[L] + k] / sc));
    }
  }
  for (uint64_t r = 0; r < n; ++r) {
    double in[64], out[64], code[64], err[64];
    double bs_in = 1.0;
    int kin = 20;
    int near = 0;
    for (int i = 0; i < 20; ++i) in[i] = (double)(float)x[20 * r + i];
    uint16_t* cr = codes ? codes + 192 * r : NULL;
    uint8_t* nr = near_act ? near_act + 192 * r : NULL;
    if (cr) memset(cr, 0, sizeof(uint16_t) * 192);
    if (nr) memset(nr, 0, 192);
    if (scale_exp) scale_exp[3 * r] = scale_exp[3 * r + 1] = scale_exp[3 * r + 2] = 0;
    if (prec == 1) {
      for (int i = 0; i < 20; ++i) in[i] = or_round_bf16(in[i]);
      if (cr)
        for (int i = 0; i < 20; ++i) cr[i] = bf16_bits(in[i]);
    } else {
      double amax = 0.0;
      for (int i = 0; i < 20; ++i) amax = fmax(amax, fabs(in[i]));
      bs_in = block_scale(amax);
      for (int i = 0; i < 20; ++i) {
        code[i] = or_round_e4m3(in[i] / bs_in);
        in[i] = code[i] * bs_in;
        if (cr) cr[i] = e4m3_bits(code[i]);
      }
      if (scale_exp) scale_exp[3 * r] = (int8_t)ilogb(bs_in);
    }
    for (int L = 0; L < 3; ++L) {
      const double* Wl = Wq + woff[L];
      const double* bl = params + (L == 0 ? B1 : (L == 1 ? B2 : B3));
      int relu_near[64];
      double ebv[64];
      for (int o = 0; o < 64; ++o) {
        double acc = 0.0, mag = 0.0;
        for (int i = 0; i < kin; ++i) {
          acc += Wl[kin * o + i] * in[i];
          mag += fabs(Wl[kin * o + i] * in[i]);
        }
        out[o] = acc * wscale[L] + bl[o];
        err[o] = prec == 2 ? fp8_dot_error_bound(Wl + kin * o, code, kin) * wscale[L] * bs_in : 0.0;
        /* the ReLU decision max(pre, 0) is a near-tie when the exact pre-activation lies within
         * the float32 error of zero: BF16 products are exact in float32, so the bound is that of
         * summing kin products and the bias in any order (gamma_{kin+1} of the magnitudes); FP8
         * adds the rounding of the scale-and-bias step to its dot-product bound */
        const double u = ldexp(1.0, -24), g = (kin + 1) * u / (1.0 - (kin + 1) * u);
        const double eb = prec == 2 ? err[o] + 2.0 * u * (fabs(acc * wscale[L]) + fabs(bl[o]))
                                    : g * (mag * wscale[L] + fabs(bl[o]));
        relu_near[o] = eb > 0.0 && fabs(out[o]) <= eb; /* all-zero terms sum to exactly 0 anywhere */
        ebv[o] = eb;
      }
      for (int o = 0; o < 64; ++o) out[o] = out[o] > 0.0 ? out[o] : 0.0;
      if (L < 2) {
        if (prec == 1) {
          for (int o = 0; o < 64; ++o) {
            /* row flag (output comparisons, which have their own tolerance): a rounding within
             * 2e-4 grid steps of its midpoint, or a ReLU near-tie.  Activation flag (code-by-code
             * comparisons, which are exact): also a midpoint within the float32 summation bound
             * of the exact value, which matters where the terms cancel (a small activation from
             * large products) */
            const double mg = midpoint_gap_bf16(out[o]);
            const int na = (out[o] > 0.0 && mg < gap) || relu_near[o];
            int e2;
            frexp(out[o], &e2);
            const int na_act = na || (out[o] > 0.0 && mg * ldexp(1.0, e2 - 8) <= ebv[o]);
            if (na) near = 1;
            in[o] = or_round_bf16(out[o]);
            if (cr) cr[64 * (L + 1) + o] = bf16_bits(in[o]);
            if (nr) nr[64 * (L + 1) + o] = (uint8_t)na_act;
          }
        } else {
          /* one power-of-two scale for the vertex's 64 activations */
          double amax = 0.0, amax_err = 0.0;
          for (int o = 0; o < 64; ++o) {
            if (out[o] >= amax) amax_err = fmax(amax_err, err[o]);
            amax = fmax(amax, out[o]);
          }
          double bs = block_scale(amax);
          double ratio = amax / 448.0;
          int scale_near = 0;
          if (ratio > 0.0) {
            /* the scale changes where amax / 448 crosses a power of two */
            int e;
            frexp(ratio, &e);
            const double tol = 1e-6 * ratio + amax_err / 448.0;
            if (ratio - ldexp(1.0, e - 1) <= tol || ldexp(1.0, e) - ratio <= tol) scale_near = near = 1;
          }
          for (int o = 0; o < 64; ++o) {
            const int na = (out[o] > 0.0 && midpoint_dist_e4m3(out[o] / bs) * bs <= err[o] + 1e-6 * out[o]) ||
                           relu_near[o];
            if (na) near = 1;
            code[o] = or_round_e4m3(out[o] / bs);
            in[o] = code[o] * bs;
            if (cr) cr[64 * (L + 1) + o] = e4m3_bits(code[o]);
            /* a scale that may change changes every code of the layer */
            if (nr) nr[64 * (L + 1) + o] = (uint8_t)(na || scale_near);
          }
          if (scale_exp) scale_exp[3 * r + L + 1] = (int8_t)ilogb(bs);
          bs_in = bs;
        }
        kin = 64;
      }
    }
    double zz = params[B4];
    for (int i = 0; i < 64; ++i) zz += params[W4 + i] * out[i];
    if (z) z[r] = zz;
    y[r] = or_softplus_mod(zz);
    if (fragile) fragile[r] = (uint8_t)near;
  }
  free(Wq);
}

/* Adam (Kingma & Ba) with bias correction; `step` is the 1-based update count. */
void or_adam(double* params, double* m, double* v, const double* grad, uint64_t np, uint64_t step, double lr,
             double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, (double)step);
  double c2 = 1.0 - pow(b2, (double)step);
  for (uint64_t i = 0; i < np; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
    v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
    double mh = m[i] / c1;
    double vh = v[i] / c2;
    params[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ---------------------------------------------------- normalization + roulette */
int32_t or_rrs_expand(const double* q_orig, const double* u, uint64_t n, double budget_base, double f_rate,
                      double* alpha, int32_t norm_mode, uint64_t cap, uint32_t* X, uint64_t* offset,
                      uint32_t* parent_of_child, uint64_t* S_out, double* F_out, float* q_norm,
                      uint32_t* retries) {
  double sum = 0.0;
  for (uint64_t i = 0; i < n; ++i) sum += q_orig[i]; /* slot order */
  *retries = 0;
  if (sum == 0.0) {
    for (uint64_t i = 0; i < n; ++i) { X[i] = 0; offset[i] = 0; if (q_norm) q_norm[i] = 0.0f; }
    *S_out = 0;
    *F_out = 0.0;
    return 0;
  }
  uint64_t S;
  double F;
  for (;;) {
    /* Eq. (10) with the rate control of Eqs. (12)-(14): budget = f_rate * alpha * N_px. */
    double budget = f_rate * (*alpha) * budget_base;
    F = budget / sum;
    if (norm_mode == OR_NORM_DOWNSCALE && F > 1.0) F = 1.0;
    if (norm_mode == 2) F = 1.0; /* no normalization (plain path tracing) */
    S = 0;
    for (uint64_t i = 0; i < n; ++i) {
      float q = (float)(F * q_orig[i]);             /* Eq. (9), rounded to the kernels' float32 */
      float k = floorf(q);
      float r = q - k;                              /* exact (Sterbenz) */
      uint32_t x = (uint32_t)k + (((float)u[i] < r) ? 1u : 0u); /* Eq. (8) */
      X[i] = x;
      if (q_norm) q_norm[i] = q;
      S += x;
    }
    if (S <= cap) break;
    *alpha *= 0.99; /* Eq. (14), eps = 0.01 */
    (*retries)++;
    if (*alpha < 1e-3) return -5;
  }
  uint64_t run = 0;
  for (uint64_t i = 0; i < n; ++i) {
    offset[i] = run;
    if (parent_of_child)
      for (uint32_t j = 0; j < X[i]; ++j) parent_of_child[run + j] = (uint32_t)i;
    run += X[i];
  }
  *S_out = S;
  *F_out = F;
  return 0;
}

/* ------------------------------------------------------------------ render */
/* Unit roundoff of float32 and the bound on the throughput error up to which a path's radiance
 * is compared at 1e-4 relative. */
#define F32_UNIT (1.0 / 16777216.0)
#define KERR_COMPARED 3e-5
typedef struct {
  double o[3], d[3], t[3];
  /* Forward error bounds of the float32 computation of the same entry (used only to flag
   * near-ties): origin position (m), direction (rad), throughput (relative). */
  double perr, derr, kerr;
  uint32_t pix, excl, id_lo, id_hi;
  uint32_t k0; /* primary path this entry descends from (index within its pass) */
  double pdfb;  /* solid-angle pdf with which the BSDF sampled this entry's direction (0: camera) */
  int32_t rec[MAXREC];
  uint8_t dead, train;
} entry;

typedef struct {
  uint32_t prim;
  double thit, b1, b2;
  double perr;  /* float32 error bound of the hit point along the surface (m) */
  double kq;    /* relative float32 error bound of the raw factor q */
  int fragile;
  /* vertex data after shading */
  double p[3], n[3], wo[3];
  uint32_t mat;
  double q;
  float q32;
  /* next-event estimation at this vertex: radiance arriving from the light sample (before the
   * throughput), and whether a near-tie decision took part in it */
  double nee[3];
  uint8_t has_nee, nee_fragile;
} vstate;

static void camera_ray(const or_scene* s, uint32_t W, uint32_t H, uint32_t px, uint32_t py, double u0, double u1,
                       double o[3], double d[3]) {
  const double* c = s->cam;
  double eye[3] = {c[0], c[1], c[2]}, look[3] = {c[3], c[4], c[5]}, up[3] = {c[6], c[7], c[8]};
  double fwd[3], right[3], upv[3];
  sub3(look, eye, fwd);
  normalize3(fwd);
  cross3(fwd, up, right);
  normalize3(right);
  cross3(right, fwd, upv);
  double th = tan(c[9] * M_PI / 360.0);
  double aspect = (double)W / (double)H;
  double sx = (2.0 * ((double)px + u0) / (double)W - 1.0) * th * aspect;
  double sy = (1.0 - 2.0 * ((double)py + u1) / (double)H) * th;
  for (int k = 0; k < 3; ++k) {
    o[k] = eye[k];
    d[k] = fwd[k] + sx * right[k] + sy * upv[k];
  }
  normalize3(d);
}

/* The 20 network inputs at a vertex (Sec. 5 encodings where the paper gives them). */
static void features(const or_scene* s, const entry* e, const vstate* v, uint32_t depth, uint32_t D, double f[20]) {
  const double* mp = s->mpar + 7 * (uint64_t)v->mat;
  double pn[3];
  for (int k = 0; k < 3; ++k) pn[k] = (v->p[k] - s->amin[k]) / s->extent;
  for (int k = 0; k < 3; ++k) f[k] = 2.0 * pn[k] - 1.0;
  for (int k = 0; k < 3; ++k) f[3 + k] = v->n[k];
  for (int k = 0; k < 3; ++k) f[6 + k] = v->wo[k];
  for (int k = 0; k < 3; ++k) f[9 + k] = 2.0 * (sqrt(e->t[k]) - 1.0); /* Box-Cox, lambda = 0.5 */
  for (int k = 0; k < 3; ++k) f[12 + k] = mp[k];
  double rough = s->mtype[v->mat] == 1 ? mp[3] : 1.0;
  f[15] = 1.0 - exp(-rough);                                     /* roughness remap */
  f[16] = (double)depth / (double)D;
  for (int k = 0; k < 3; ++k) f[17 + k] = sin(16.0 * M_PI * pn[k]);
}

typedef struct {
  const or_scene* s;
  const or_cfg* cfg;
  const double* params;
  const double* guide;
  double* image;
  uint8_t* fragile;
  double* rec_feat; double* rec_lumt; double* rec_acc; uint32_t* rec_depth; uint32_t* rec_pix; uint64_t* rec_id;
  uint64_t nrec;
  double ew; /* weight of emission added to the image (enumeration branch probability) */
  double* path_rgb;      /* optional: radiance per primary path and vertex depth [nprim][D][3],
                            summed over passes */
  uint8_t* path_first;   /* optional: per primary path, the smallest depth at which it or a
                            descendant took a near-tie decision (D + 1 = none) */
} rctx;

/* A near-tie decision on entry e at `depth`: its pixel, and its primary path's radiance from
 * this depth on, are not compared exactly. */
static void mark_fragile(rctx* c, const entry* e, uint32_t depth) {
  if (c->fragile) c->fragile[e->pix] = 1;
  if (c->path_first && depth < c->path_first[e->k0]) c->path_first[e->k0] = (uint8_t)depth;
}

static void add_emission(rctx* c, const entry* e, const double le[3], uint32_t depth) {
  double contrib[3] = {c->ew * e->t[0] * le[0], c->ew * e->t[1] * le[1], c->ew * e->t[2] * le[2]};
  if (c->image)
    for (int k = 0; k < 3; ++k) c->image[3 * (uint64_t)e->pix + k] += contrib[k];
  if (c->path_rgb)
    for (int k = 0; k < 3; ++k)
      c->path_rgb[3 * ((uint64_t)e->k0 * c->cfg->max_depth + (depth - 1)) + k] += contrib[k];
  double l = lum3(contrib);
  for (int r = 0; r < MAXREC; ++r)
    if (e->rec[r] >= 0 && c->rec_acc) c->rec_acc[e->rec[r]] += l;
}

/* Trace + shade one depth.  Fills v[i].q (q_orig, or 0 for inactive entries). */
static void extend_and_shade(rctx* c, entry* Q, vstate* V, uint64_t n, uint32_t depth, uint32_t pass,
                             or_stats* st) {
  const or_scene* s = c->s;
  const or_cfg* cfg = c->cfg;
  const uint32_t D = cfg->max_depth;
  const double tau = cfg->tau;
  uint64_t rays = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : rays)
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    vstate* v = &V[i];
    v->fragile = 0;
    v->q = 0.0;
    v->q32 = 0.0f;
    v->perr = 0.0;
    v->kq = 0.0;
    v->has_nee = 0;
    v->nee_fragile = 0;
    if (Q[i].dead) { v->prim = MISS; continue; }
    rays++;
    double gerr = 0.0;
    v->fragile = trace_one(s, Q[i].o, Q[i].d, Q[i].excl, s->nodes != NULL, tau, Q[i].perr, Q[i].derr, &v->prim,
                           &v->thit, &v->b1, &v->b2, &gerr);
    v->perr = gerr;
  }
  st->rays += rays;
  /* shading, in slot order (FP64 image sums in a fixed order) */
  /* Mix-Depth (Sec. 4.3): the method is chosen per bounce; the network only where the table says */
  int fixed = cfg->mode != OR_MODE_OFF && depth <= 64 && ((cfg->fixed_depths >> (depth - 1)) & 1u);
  int net = !fixed && cfg->mode == OR_MODE_NET && depth <= 64 && ((cfg->net_depths >> (depth - 1)) & 1u) &&
            c->params != NULL;
  int nrrs = !fixed && (cfg->mode == OR_MODE_NRRS || cfg->mode == OR_MODE_AID) && depth <= 64 &&
             ((cfg->net_depths >> (depth - 1)) & 1u) && c->params != NULL && cfg->hash_log2 > 0;
  const int aid = cfg->mode == OR_MODE_AID;
  for (uint64_t i = 0; i < n; ++i) {
    entry* e = &Q[i];
    vstate* v = &V[i];
    if (e->dead) continue;
    if (v->fragile) mark_fragile(c, e, depth);
    /* beyond KERR_COMPARED the throughput's float32 error bound is too large for the radiance
     * from this depth on (misses included) to be compared */
    if (tau > 0.0 && e->kerr > KERR_COMPARED) mark_fragile(c, e, depth);
    if (v->prim == MISS) {
      add_emission(c, e, s->env, depth);
      continue;
    }
    const double* tv = s->tri + 9 * (uint64_t)v->prim;
    double e1[3], e2[3], ng[3];
    sub3(tv + 3, tv, e1);
    sub3(tv + 6, tv, e2);
    cross3(e1, e2, ng);
    normalize3(ng);
    double w0 = 1.0 - v->b1 - v->b2;
    for (int k = 0; k < 3; ++k) v->p[k] = w0 * tv[k] + v->b1 * tv[3 + k] + v->b2 * tv[6 + k];
    for (int k = 0; k < 3; ++k) v->wo[k] = -e->d[k];
    double cos_o = dot3(ng, v->wo);
    if (tau > 0.0 && fabs(cos_o) < tau) mark_fragile(c, e, depth);
    /* float32 error of the hit point: the ray's error spread along the surface, plus the
     * rounding of its coordinates */
    v->perr = v->perr / fmax(fabs(cos_o), 1e-12) +
              8.0 * F32_UNIT * fmax(fabs(v->p[0]), fmax(fabs(v->p[1]), fabs(v->p[2])));
    /* beyond a quarter of the typical triangle the traversal's flags would need wider box
     * paddings than it gives: stop comparing the path from the children on (the bound is then
     * held there) */
    if (v->perr > s->perr_max) {
      if (tau > 0.0) mark_fragile(c, e, depth + 1);
      v->perr = s->perr_max;
    }
    v->kq = e->kerr + 8.0 * F32_UNIT;
    int front = cos_o > 0.0;
    for (int k = 0; k < 3; ++k) v->n[k] = front ? ng[k] : -ng[k];
    v->mat = s->tmat[v->prim];
    const double* mp = s->mpar + 7 * (uint64_t)v->mat;
    if (front && (mp[4] != 0.0 || mp[5] != 0.0 || mp[6] != 0.0)) {
      if (cfg->nee && depth > 1 && e->pdfb > 0.0) {
        /* a BSDF-sampled hit on a light: power-heuristic weight against light sampling */
        const double pl = s->lpdf[v->prim] * v->thit * v->thit / cos_o;
        const double w = e->pdfb * e->pdfb / (e->pdfb * e->pdfb + pl * pl);
        const double le[3] = {w * mp[4], w * mp[5], w * mp[6]};
        add_emission(c, e, le, depth);
      } else {
        add_emission(c, e, mp + 4, depth);
      }
    }
    if (depth >= D || s->mtype[v->mat] == 2) continue; /* last vertex or pure emitter: terminate */
    if (cfg->mode == OR_MODE_OFF) {
      v->q = 1.0;
    } else {
      double tr[3] = {e->t[0] * mp[0], e->t[1] * mp[1], e->t[2] * mp[2]};
      v->q = lum3(tr); /* heuristic: luminance of throughput x albedo */
      /* Mix-Depth's fixed rate (Sec. 4.3): one raw factor for every vertex that continues, so the
       * normalization gives all of them the same expected number of children */
      if (fixed) v->q = v->q > 0.0 ? 1.0 : 0.0;
    }
    /* training record (vertex reflected radiance target, descendants add to it) */
    if (cfg->mode != OR_MODE_OFF && e->train && depth <= (uint32_t)cfg->net_max_depth && depth <= MAXREC &&
        c->nrec < cfg->rec_cap && c->rec_feat) {
      uint64_t r = c->nrec++;
      features(s, e, v, depth, D, c->rec_feat + 20 * r);
      c->rec_lumt[r] = lum3(e->t);
      c->rec_acc[r] = 0.0;
      c->rec_depth[r] = depth;
      c->rec_pix[r] = e->pix;
      c->rec_id[r] = ((uint64_t)e->id_hi << 32) | e->id_lo;
      e->rec[depth - 1] = (int32_t)r;
    }
  }
  if (cfg->nee && s->nl > 0) {
    /* next-event estimation at every vertex that may continue (d < D, not a pure emitter): one
     * light sample, a shadow ray from the offset hit point, power-heuristic weight against the
     * BSDF's sampling of the same direction */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
      entry* e = &Q[i];
      vstate* v = &V[i];
      if (e->dead || v->prim == MISS || depth >= D || s->mtype[v->mat] == 2) continue;
      uint32_t r[4];
      rng_block(cfg->seed, e->id_lo, e->id_hi, PURPOSE_NEE, depth, 0, r);
      const double u0 = u01(r[0]), u1 = u01(r[1]), u2 = u01(r[2]);
      uint32_t lo = 0, hi = s->nl - 1; /* smallest k with cdf[k + 1] > u0 */
      while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if (s->light_cdf[mid + 1] > u0) hi = mid; else lo = mid + 1;
      }
      int frag = 0;
      /* the float32 CDF may put a boundary this close to u0 on the other side */
      if (tau > 0.0 && ((lo > 0 && u0 - s->light_cdf[lo] < 1e-6) || s->light_cdf[lo + 1] - u0 < 1e-6)) frag = 1;
      const uint32_t lt = s->light_tri[lo];
      const double* tv = s->tri + 9 * (uint64_t)lt;
      double e1[3], e2[3], ng[3], y[3];
      sub3(tv + 3, tv, e1);
      sub3(tv + 6, tv, e2);
      cross3(e1, e2, ng);
      normalize3(ng);
      const double su = sqrt(u1);
      const double b1 = su * (1.0 - u2), b2 = su * u2;
      for (int k = 0; k < 3; ++k) y[k] = tv[k] + b1 * e1[k] + b2 * e2[k];
      double o[3], d[3];
      for (int k = 0; k < 3; ++k) o[k] = v->p[k] + s->offset * v->n[k];
      sub3(y, o, d);
      const double dist = sqrt(dot3(d, d));
      if (!(dist > 0.0)) continue;
      for (int k = 0; k < 3; ++k) d[k] /= dist;
      const double cos_x = dot3(v->n, d), cos_l = -dot3(ng, d);
      if (tau > 0.0 && (fabs(cos_x) < tau || fabs(cos_l) < tau)) frag = 1;
      /* a light point this close to the vertex: the float32 direction (from two rounded points)
       * carries a relative error beyond the comparison's reach */
      if (tau > 0.0 && (v->perr + 2.0 * F32_UNIT * s->extent) / dist > 2e-5) frag = 1;
      v->nee_fragile = (uint8_t)frag;
      if (cos_x <= 0.0 || cos_l <= 0.0) continue;
      /* BSDF value (times cos) and sampling pdf of d at the vertex */
      const double* mp = s->mpar + 7 * (uint64_t)v->mat;
      double tb[3], bb[3];
      onb(v->n, tb, bb);
      const double wol[3] = {dot3(v->wo, tb), dot3(v->wo, bb), dot3(v->wo, v->n)};
      const double wil[3] = {dot3(d, tb), dot3(d, bb), cos_x};
      double fc[3], pb;
      if (s->mtype[v->mat] == 1) {
        for (int k = 0; k < 3; ++k) fc[k] = or_ggx_eval_cos(mp[3], mp[k], wol, wil);
        pb = ggx_pdf(mp[3], wol, wil);
      } else {
        for (int k = 0; k < 3; ++k) fc[k] = mp[k] / M_PI * cos_x;
        pb = cos_x / M_PI;
      }
      const double pl = s->lpdf[lt] * dist * dist / cos_l;
      const double w = pl * pl / (pl * pl + pb * pb);
      /* visibility: nothing closer than the light point (shortened by 1e-4 of the distance) */
      uint32_t prim;
      double th, hb1, hb2, gerr;
      const double derr = 2.0 * v->perr / dist + 16.0 * F32_UNIT;
      int tf = trace_one(s, o, d, v->prim, s->nodes != NULL, tau, v->perr, derr, &prim, &th, &hb1, &hb2, &gerr);
      const double tmax = dist * (1.0 - 1e-4);
      /* the light's own hit lies 1e-4 dist beyond tmax, as far as the general near-tie margin tau:
       * this comparison takes the margin of its float32 error instead (origin and direction
       * errors plus a few units in the last place of t and tmax, far below 1e-5 t) */
      const double tol_t = fmin(tau, 1e-5) * tmax + v->perr + derr * th;
      if (tau > 0.0 && (tf || (prim != MISS && fabs(th - tmax) < tol_t))) frag = 1;
      v->nee_fragile = (uint8_t)frag;
      if (prim != MISS && th < tmax) continue; /* occluded */
      const double* le = s->mpar + 7 * (uint64_t)s->tmat[lt] + 4;
      for (int k = 0; k < 3; ++k) v->nee[k] = fc[k] * le[k] * w / pl;
      v->has_nee = 1;
    }
    /* in slot order: the radiance (with the vertex's throughput) to the image, the path and the
     * records of the vertex's ancestors (its own record does not see its own light sample) */
    for (uint64_t i = 0; i < n; ++i) {
      entry* e = &Q[i];
      vstate* v = &V[i];
      if (v->nee_fragile) mark_fragile(c, e, depth);
      if (!v->has_nee) continue;
      entry anc = *e;
      if (depth <= MAXREC) anc.rec[depth - 1] = -1;
      add_emission(c, &anc, v->nee, depth);
    }
  }
  if (net) {
    /* ADRRS ratio with the network's reflected-radiance estimate (Sec. 2.2, Sec. 5 "Compromise"). */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
      entry* e = &Q[i];
      vstate* v = &V[i];
      if (e->dead || v->q <= 0.0 || v->prim == MISS) continue;
      double g = c->guide ? c->guide[e->pix] : -1.0;
      if (!(g >= 0.0)) continue; /* no pixel history: keep the heuristic */
      double f[20], y, z;
      features(s, e, v, depth, D, f);
      or_mlp_forward(c->params, f, 1, &y, &z);
      if (!isfinite(y)) continue;
      /* the ADRRS ratio, held within [q_h / 8, 64 q_h] of the heuristic factor q_h of the vertex */
      const double qr = lum3(e->t) * y / (g + 0.01);
      if (!isfinite(qr)) continue;
      v->q = fmin(fmax(qr, 0.125 * v->q), 64.0 * v->q);
      /* the inputs carry the hit point's error (the sine encoding scales it by 16 pi / extent) */
      v->kq += 64.0 * v->perr / s->extent;
    }
  }
  if (nrrs) {
    /* NRRS (Sec. 4.2): StatNet's statistics of the vertex, then RRSNet's factor, with the pixel's
     * previous mean as I_px; AID-NRRS: the AID RRSNet alone (params = its MLP and hash grid); no
     * pixel history keeps the heuristic */
    const double* Ps = c->params;
    const double* Pr = Ps + OR_STAT_NPARAM;
    const double* Tb = Pr + OR_RRS_NPARAM;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
      entry* e = &Q[i];
      vstate* v = &V[i];
      if (e->dead || v->q <= 0.0 || v->prim == MISS) continue;
      double g = c->guide ? c->guide[e->pix] : -1.0;
      if (!(g >= 0.0)) continue;
      const double* mp = s->mpar + 7 * (uint64_t)v->mat;
      double raw[7];
      for (int k = 0; k < 3; ++k) raw[k] = (v->p[k] - s->amin[k]) / s->extent;
      for (int k = 0; k < 3; ++k) raw[3 + k] = v->wo[k];
      raw[6] = 1.0 - exp(-(s->mtype[v->mat] == 1 ? mp[3] : 1.0));
#define FACTOR(RAW, T) (aid ? or_aid_factor(Ps, Ps + OR_AID_NPARAM, cfg->hash_log2, RAW, T, g, NULL) \
                            : or_nrrs_factor(Ps, Pr, Tb, cfg->hash_log2, RAW, T, g, NULL, NULL))
      const double q = FACTOR(raw, e->t);
      if (!(q >= 1e-20 && q < 3e38)) continue; /* a factor out of range keeps the heuristic */
      /* float32 error of the factor from its inputs' errors: the change of q when the position
       * moves by twice its error bound, the direction by twice its bound, the throughput by
       * twice its relative bound (central differences, summed: about four times the linear
       * estimate) */
      double dq = 0.0;
      for (int k = 0; k < 6; ++k) {
        const double h = k < 3 ? 2.0 * v->perr / s->extent : 2.0 * e->derr;
        double rp[7], rm[7];
        memcpy(rp, raw, sizeof(rp));
        memcpy(rm, raw, sizeof(rm));
        rp[k] += h;
        rm[k] -= h;
        dq += fabs(FACTOR(rp, e->t) - FACTOR(rm, e->t));
      }
      double tp[3], tm[3];
      for (int k = 0; k < 3; ++k) {
        tp[k] = e->t[k] * (1.0 + 2.0 * e->kerr);
        tm[k] = e->t[k] * (1.0 - 2.0 * e->kerr);
      }
      dq += fabs(FACTOR(raw, tp) - FACTOR(raw, tm));
#undef FACTOR
      v->q = q;
      v->kq += dq / q;
    }
  }
  (void)pass;
}

static void expand_children(rctx* c, const entry* Q, const vstate* V, uint64_t n, const uint32_t* X,
                            const uint64_t* off, entry* Qn, uint32_t depth) {
  const or_scene* s = c->s;
  const or_cfg* cfg = c->cfg;
  const double tau = cfg->tau;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    if (X[i] == 0) continue;
    const entry* e = &Q[i];
    const vstate* v = &V[i];
    const double* mp = s->mpar + 7 * (uint64_t)v->mat;
    double tb[3], bb[3];
    onb(v->n, tb, bb);
    /* the local frame switches sign convention at n_z = 0: a nonzero n_z this close to the
     * switch may have the other sign in float32, a near-tie (an exact zero is exact there too) */
    if (tau > 0.0 && v->n[2] != 0.0 && fabs(v->n[2]) < tau) mark_fragile(c, e, depth + 1);
    double wol[3] = {dot3(v->wo, tb), dot3(v->wo, bb), dot3(v->wo, v->n)};
    for (uint32_t j = 0; j < X[i]; ++j) {
      uint32_t r[4];
      rng_block(cfg->seed, e->id_lo, e->id_hi, PURPOSE_CHILD, depth, cfg->frozen ? 0u : j, r);
      double u2 = u01(r[0]), u3 = u01(r[1]);
      double wil[3], w[3], pdf;
      int alive = 1;
      if (s->mtype[v->mat] == 1) {
        double a = mp[3];
        for (int k = 0; k < 3; ++k) {
          double wk;
          alive = or_ggx_sample(a, mp[k], wol, u2, u3, wil, &wk, &pdf);
          w[k] = wk;
        }
        if (tau > 0.0 && fabs(wil[2]) < tau) mark_fragile(c, e, depth + 1);
      } else {
        or_lambert_sample(u2, u3, wil, &pdf);
        for (int k = 0; k < 3; ++k) w[k] = mp[k];
      }
      entry* ch = &Qn[off[i] + j];
      ch->pdfb = pdf;
      double wi[3];
      for (int k = 0; k < 3; ++k) wi[k] = wil[0] * tb[k] + wil[1] * bb[k] + wil[2] * v->n[k];
      normalize3(wi);
      for (int k = 0; k < 3; ++k) {
        ch->o[k] = v->p[k] + s->offset * v->n[k];
        ch->d[k] = wi[k];
        ch->t[k] = alive ? e->t[k] * w[k] / (double)v->q32 : 0.0;
      }
      /* float32 error bounds of the child: the hit point's (and the offset's rounding); a cosine
       * sample takes a fresh direction in the triangle's frame, a GGX sample carries the incoming
       * direction's error through the visible-normal map (stretched by up to 1 / alpha) and into
       * the Smith terms (growing as 1 / |cos|) */
      ch->perr = v->perr + 4.0 * F32_UNIT * fmax(fabs(v->p[0]), fmax(fabs(v->p[1]), fabs(v->p[2])));
      if (s->mtype[v->mat] == 1) {
        /* reflection keeps an angular error; the visible-normal sample moves with the incoming
         * direction by at most about alpha times its change */
        ch->derr = e->derr * (1.0 + 2.0 * mp[3]) + 16.0 * F32_UNIT;
        ch->kerr = e->kerr + 8.0 * F32_UNIT + e->derr * (2.0 / fmax(fabs(wol[2]), 1e-12) + 2.0 / fmax(fabs(wil[2]), 1e-12));
      } else {
        ch->derr = 16.0 * F32_UNIT;
        ch->kerr = e->kerr + 8.0 * F32_UNIT;
      }
      if (ch->derr * s->diag > s->perr_max) {
        if (tau > 0.0) mark_fragile(c, e, depth + 1);
        ch->derr = s->perr_max / s->diag;
      }
      ch->pix = e->pix;
      ch->k0 = e->k0;
      ch->excl = v->prim;
      ch->id_lo = r[2];
      ch->id_hi = r[3];
      for (int k = 0; k < MAXREC; ++k) ch->rec[k] = e->rec[k];
      ch->train = e->train;
      ch->dead = alive ? 0 : 1;
    }
  }
}

int32_t or_render(const or_scene* s, or_cfg* cfg, const double* params, double* guide, double* image,
                  uint8_t* fragile, or_stats* stats, double* rec_feat, double* rec_lumt, double* rec_acc,
                  uint32_t* rec_depth, uint32_t* rec_pix, uint64_t* rec_id, double* path_rgb,
                  uint8_t* path_first) {
  if (!s || !cfg || cfg->width == 0 || cfg->height == 0 || cfg->s_batch == 0 || cfg->max_depth == 0 ||
      cfg->max_depth > OR_MAXD)
    return -1;
  memset(stats, 0, sizeof(*stats));
  const uint64_t npx = (uint64_t)cfg->width * cfg->height;
  const uint64_t nprim = npx * cfg->s_batch;
  const uint64_t cap = (uint64_t)floor(cfg->cap_factor * (double)nprim);
  const uint64_t qcap = cap > nprim ? cap : nprim;
  entry* Q = (entry*)malloc(sizeof(entry) * qcap);
  entry* Qn = (entry*)malloc(sizeof(entry) * qcap);
  vstate* V = (vstate*)malloc(sizeof(vstate) * qcap);
  double* qv = (double*)malloc(sizeof(double) * qcap);
  double* uv = (double*)malloc(sizeof(double) * qcap);
  uint32_t* X = (uint32_t*)malloc(sizeof(uint32_t) * qcap);
  uint64_t* off = (uint64_t*)malloc(sizeof(uint64_t) * qcap);
  float* q32 = (float*)malloc(sizeof(float) * qcap);
  rctx c = {s, cfg, params, guide, image, fragile, rec_feat, rec_lumt, rec_acc, rec_depth, rec_pix, rec_id, 0, 1.0,
            path_rgb, path_first};
  if (path_first)
    for (uint64_t k = 0; k < nprim; ++k) path_first[k] = (uint8_t)(cfg->max_depth + 1);
  int32_t status = 0;
  for (uint32_t pp = 0; pp < cfg->n_passes && status == 0; ++pp) {
    uint32_t pass = cfg->pass_begin + pp;
    /* camera: primary path k is sample k mod s_batch of pixel floor(k / s_batch) */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)nprim; ++k) {
      entry* e = &Q[k];
      uint32_t pix = (uint32_t)(k / cfg->s_batch);
      uint32_t r[4];
      rng_block(cfg->seed, (uint32_t)k, pass, PURPOSE_CAMERA, 0, 0, r);
      camera_ray(s, cfg->width, cfg->height, pix % cfg->width, pix / cfg->width, u01(r[0]), u01(r[1]), e->o, e->d);
      e->t[0] = e->t[1] = e->t[2] = 1.0;
      e->perr = F32_UNIT * fmax(fabs(e->o[0]), fmax(fabs(e->o[1]), fabs(e->o[2])));
      e->derr = 16.0 * F32_UNIT;
      e->kerr = 0.0;
      e->pdfb = 0.0;
      e->pix = pix;
      e->k0 = (uint32_t)k;
      e->excl = MISS;
      e->id_lo = (uint32_t)k;
      e->id_hi = pass;
      for (int j = 0; j < MAXREC; ++j) e->rec[j] = -1;
      e->dead = 0;
      rng_block(cfg->seed, (uint32_t)k, pass, PURPOSE_TRAIN, 0, 0, r);
      e->train = u01(r[0]) < cfg->p_train ? 1 : 0;
    }
    uint64_t n = nprim;
    for (uint32_t depth = 1; depth <= cfg->max_depth && n > 0; ++depth) {
      stats->n[depth] += n;
      extend_and_shade(&c, Q, V, n, depth, pass, stats);
      if (depth == cfg->max_depth) break;
      uint64_t act = 0;
      for (uint64_t i = 0; i < n; ++i) {
        qv[i] = V[i].q;
        if (V[i].q > 0.0) act++;
        uint32_t r[4];
        rng_block(cfg->seed, Q[i].id_lo, Q[i].id_hi, PURPOSE_ROULETTE, depth, 0, r);
        uv[i] = u01(r[0]);
      }
      stats->active[depth] += act;
      uint64_t S;
      double F;
      uint32_t retries;
      int32_t mode = cfg->mode == OR_MODE_OFF ? 2 : cfg->norm_mode;
      status = or_rrs_expand(qv, uv, n, (double)nprim, cfg->f_rate, &cfg->alpha, mode, cap, X, off, NULL, &S, &F,
                             q32, &retries);
      if (status != 0) break;
      stats->sumq[depth] = 0.0;
      for (uint64_t i = 0; i < n; ++i) stats->sumq[depth] += qv[i];
      stats->F[depth] = F;
      stats->S[depth] += S;
      stats->retries[depth] += retries;
      for (uint64_t i = 0; i < n; ++i) {
        V[i].q32 = q32[i];
        if (V[i].q > 0.0 && cfg->tau > 0.0) {
          float r = q32[i] - floorf(q32[i]);
          /* within the decision margin, or within the float32 error bound of the factor */
          if (fabs(uv[i] - (double)r) < (cfg->tau + V[i].kq) * (double)q32[i]) mark_fragile(&c, &Q[i], depth + 1);
        }
      }
      expand_children(&c, Q, V, n, X, off, Qn, depth);
      entry* tmp = Q; Q = Qn; Qn = tmp;
      n = S;
    }
    if (guide && cfg->update_guide && image) {
      double spp = (double)(pass + 1) * (double)cfg->s_batch;
      for (uint64_t p = 0; p < npx; ++p) guide[p] = lum3(image + 3 * p) / spp;
    }
  }
  stats->n_records = c.nrec;
  stats->status = status;
  free(Q); free(Qn); free(V); free(qv); free(uv); free(X); free(off); free(q32);
  return status;
}

/* ------------------------------------------------------------ enumeration */
typedef struct {
  const or_scene* s;
  or_cfg cfg;
  uint64_t nprim, cap;
  double* image;
  uint64_t max_S, branches;
  double* pmf;      /* optional [(max_depth + 1) * (cap + 2)]: probability of S children at depth d
                       (bucket cap + 1 collects S > cap) */
  double* live;     /* optional [max_depth + 1]: probability that depth d normalizes a positive sum */
  float* qn1;       /* optional [nprim]: the normalized factors of depth 1 */
} ectx;

static void enum_depth(ectx* ec, entry* Q, uint64_t n, uint32_t depth, double prob) {
  vstate* V = (vstate*)malloc(sizeof(vstate) * (n ? n : 1));
  rctx c = {ec->s, &ec->cfg, NULL, NULL, ec->image, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0, prob};
  or_stats st;
  memset(&st, 0, sizeof(st));
  extend_and_shade(&c, Q, V, n, depth, 0, &st);
  if (depth == ec->cfg.max_depth || n == 0) {
    ec->branches++;
    free(V);
    return;
  }
  double sum = 0.0;
  for (uint64_t i = 0; i < n; ++i) sum += V[i].q;
  if (sum == 0.0) { ec->branches++; free(V); return; }
  if (ec->live) ec->live[depth] += prob;
  double F = ec->cfg.f_rate * ec->cfg.alpha * (double)ec->nprim / sum;
  if (ec->cfg.norm_mode == OR_NORM_DOWNSCALE && F > 1.0) F = 1.0;
  uint32_t* k = (uint32_t*)malloc(sizeof(uint32_t) * n);
  double* r = (double*)malloc(sizeof(double) * n);
  uint64_t* fi = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t nf = 0;
  for (uint64_t i = 0; i < n; ++i) {
    float q = (float)(F * V[i].q);
    V[i].q32 = q;
    k[i] = (uint32_t)floorf(q);
    r[i] = (double)(q - floorf(q));
    if (r[i] > 0.0) fi[nf++] = i;
    if (depth == 1 && ec->qn1) ec->qn1[i] = q;
  }
  uint32_t* X = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint64_t* off = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (uint64_t mask = 0; mask < (1ull << nf); ++mask) {
    double p = prob;
    for (uint64_t i = 0; i < n; ++i) X[i] = k[i];
    for (uint64_t b = 0; b < nf; ++b) {
      uint64_t i = fi[b];
      if ((mask >> b) & 1ull) { X[i] += 1; p *= r[i]; }
      else p *= 1.0 - r[i];
    }
    uint64_t S = 0;
    for (uint64_t i = 0; i < n; ++i) { off[i] = S; S += X[i]; }
    if (S > ec->max_S) ec->max_S = S;
    if (ec->pmf) ec->pmf[(uint64_t)depth * (ec->cap + 2) + (S <= ec->cap ? S : ec->cap + 1)] += p;
    if (p == 0.0) continue;
    entry* Qn = (entry*)malloc(sizeof(entry) * (S ? S : 1));
    rctx cc = {ec->s, &ec->cfg, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0, 1.0};
    expand_children(&cc, Q, V, n, X, off, Qn, depth);
    enum_depth(ec, Qn, S, depth + 1, p);
    free(Qn);
  }
  free(k); free(r); free(fi); free(X); free(off); free(V);
}

int32_t or_enumerate(const or_scene* s, const or_cfg* cfg, double* image_expect, double* image_off,
                     uint64_t* max_S, uint64_t* branches, double* pmf_S, double* live, float* q_norm1) {
  const uint64_t npx = (uint64_t)cfg->width * cfg->height;
  const uint64_t nprim = npx * cfg->s_batch;
  if (nprim > 16 || cfg->max_depth > 6) return -1;
  ectx ec;
  ec.s = s;
  ec.cfg = *cfg;
  ec.cfg.frozen = 1;
  ec.cfg.tau = 0.0;
  ec.cfg.mode = OR_MODE_HEUR;
  ec.nprim = nprim;
  ec.cap = (uint64_t)floor(cfg->cap_factor * (double)nprim);
  ec.image = image_expect;
  ec.max_S = 0;
  ec.branches = 0;
  ec.pmf = pmf_S;
  ec.live = live;
  ec.qn1 = q_norm1;
  if (pmf_S) memset(pmf_S, 0, sizeof(double) * (cfg->max_depth + 1) * (ec.cap + 2));
  if (live) memset(live, 0, sizeof(double) * (cfg->max_depth + 1));
  memset(image_expect, 0, sizeof(double) * 3 * npx);
  entry* Q = (entry*)malloc(sizeof(entry) * nprim);
  uint32_t pass = cfg->pass_begin;
  for (uint64_t k = 0; k < nprim; ++k) {
    entry* e = &Q[k];
    uint32_t pix = (uint32_t)(k / cfg->s_batch);
    uint32_t r[4];
    rng_block(cfg->seed, (uint32_t)k, pass, PURPOSE_CAMERA, 0, 0, r);
    camera_ray(s, cfg->width, cfg->height, pix % cfg->width, pix / cfg->width, u01(r[0]), u01(r[1]), e->o, e->d);
    e->t[0] = e->t[1] = e->t[2] = 1.0;
    e->perr = e->derr = e->kerr = 0.0;
    e->pdfb = 0.0;
    e->pix = pix; e->k0 = (uint32_t)k; e->excl = MISS; e->id_lo = (uint32_t)k; e->id_hi = pass;
    for (int j = 0; j < MAXREC; ++j) e->rec[j] = -1;
    e->dead = 0; e->train = 0;
  }
  enum_depth(&ec, Q, nprim, 1, 1.0);
  free(Q);
  *max_S = ec.max_S;
  *branches = ec.branches;
  /* plain path tracing on the same (child-0) samples */
  or_cfg oc = *cfg;
  oc.mode = OR_MODE_OFF;
  oc.frozen = 1;
  oc.tau = 0.0;
  oc.n_passes = 1;
  oc.rec_cap = 0;
  oc.alpha = 1.0;
  memset(image_off, 0, sizeof(double) * 3 * npx);
  or_stats st;
  return or_render(s, &oc, NULL, NULL, image_off, NULL, &st, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL);
}

int32_t or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
