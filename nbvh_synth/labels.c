/*
 * Ground-truth labels for the seeded synthetic scenes: closest ray/triangle
 * intersection with the Moller-Trumbore test, in double precision, over the
 * whole mesh. The N-BVH paper (Sec. 4, "Encoding, inference & training")
 * trains against the intersection with the actual geometry; these labels are
 * INPUTS to the training step and to the accuracy reports, not part of the
 * neural ray query itself.
 *
 * Two entry points answer the same question:
 *   tb_closest        -- a triangle BVH (median split on centroids) prunes the
 *                        search; boxes are tested conservatively (expanded), so
 *                        the set of triangles that could be the answer is never
 *                        culled and the result equals the brute-force one.
 *   tb_closest_brute  -- every triangle, used to pin the BVH version.
 *
 * Rules (shared by both): a triangle is hit when |det| >= 1e-12*|e1||e2|,
 * barycentrics u >= 0, v >= 0, u + v <= 1 (inclusive) and t0 <= t <= t1
 * (inclusive). Among hits the smallest t wins; equal t goes to the lowest
 * triangle id.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double lo[3], hi[3];
  int64_t a, b; /* internal: children a, b; leaf: a = first prim, b = -(count) */
} tb_node;

typedef struct {
  const double* v;  /* [nv][3] */
  const int32_t* t; /* [nt][3] */
  int64_t nt;
  tb_node* nodes;
  int64_t n_nodes;
  int64_t* prim; /* permutation of triangle ids */
  double* cen;   /* [nt][3] centroids */
} tb_bvh;

static int less_cen(const double* cen, int axis, int64_t a, int64_t b) {
  double ca = cen[3 * a + axis], cb = cen[3 * b + axis];
  return ca < cb || (ca == cb && a < b);
}

/* quickselect: afterwards p[k] holds the k-th prim in (centroid, id) order,
 * with smaller ones before it and larger ones after it */
static void select_kth(int64_t* p, int64_t n, int64_t k, const double* cen, int axis) {
  int64_t lo = 0, hi = n - 1;
  while (hi > lo) {
    int64_t mid = lo + (hi - lo) / 2;
    /* median of three moved to hi as the pivot */
    if (less_cen(cen, axis, p[mid], p[lo])) { int64_t s = p[mid]; p[mid] = p[lo]; p[lo] = s; }
    if (less_cen(cen, axis, p[hi], p[lo])) { int64_t s = p[hi]; p[hi] = p[lo]; p[lo] = s; }
    if (less_cen(cen, axis, p[mid], p[hi])) { int64_t s = p[mid]; p[mid] = p[hi]; p[hi] = s; }
    int64_t pivot = p[hi], store = lo;
    for (int64_t i = lo; i < hi; ++i)
      if (less_cen(cen, axis, p[i], pivot)) { int64_t s = p[i]; p[i] = p[store]; p[store] = s; ++store; }
    p[hi] = p[store];
    p[store] = pivot;
    if (store == k) return;
    if (store < k) lo = store + 1; else hi = store - 1;
  }
}

static void tri_bounds(const tb_bvh* B, int64_t tri, double lo[3], double hi[3]) {
  for (int k = 0; k < 3; ++k) {
    const double* p = B->v + 3 * (int64_t)B->t[3 * tri + k];
    for (int a = 0; a < 3; ++a) {
      if (k == 0 || p[a] < lo[a]) lo[a] = p[a];
      if (k == 0 || p[a] > hi[a]) hi[a] = p[a];
    }
  }
}

static int64_t build_rec(tb_bvh* B, int64_t first, int64_t count) {
  int64_t id = B->n_nodes++;
  tb_node* n = &B->nodes[id];
  double lo[3], hi[3], clo[3], chi[3];
  for (int64_t i = 0; i < count; ++i) {
    double tl[3], th[3];
    int64_t p = B->prim[first + i];
    tri_bounds(B, p, tl, th);
    for (int a = 0; a < 3; ++a) {
      double c = B->cen[3 * p + a];
      if (i == 0 || tl[a] < lo[a]) lo[a] = tl[a];
      if (i == 0 || th[a] > hi[a]) hi[a] = th[a];
      if (i == 0 || c < clo[a]) clo[a] = c;
      if (i == 0 || c > chi[a]) chi[a] = c;
    }
  }
  /* conservative expansion: rounding in the slab test can never cull a
   * triangle that the exact-arithmetic ray passes through */
  for (int a = 0; a < 3; ++a) {
    double pad = 1e-9 * (1.0 + fabs(lo[a]) + fabs(hi[a]));
    n->lo[a] = lo[a] - pad;
    n->hi[a] = hi[a] + pad;
  }
  if (count <= 4) {
    n->a = first;
    n->b = -count;
    return id;
  }
  int axis = 0;
  double ext = chi[0] - clo[0];
  for (int a = 1; a < 3; ++a)
    if (chi[a] - clo[a] > ext) { ext = chi[a] - clo[a]; axis = a; }
  int64_t half = count / 2;
  select_kth(B->prim + first, count, half, B->cen, axis);
  int64_t l = build_rec(B, first, half);
  int64_t r = build_rec(B, first + half, count - half);
  B->nodes[id].a = l;
  B->nodes[id].b = r;
  return id;
}

void* tb_build(const double* verts, int64_t nv, const int32_t* tris, int64_t nt) {
  (void)nv;
  tb_bvh* B = (tb_bvh*)calloc(1, sizeof(tb_bvh));
  B->v = verts;
  B->t = tris;
  B->nt = nt;
  B->prim = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nt > 0 ? nt : 1));
  B->cen = (double*)malloc(sizeof(double) * 3 * (size_t)(nt > 0 ? nt : 1));
  B->nodes = (tb_node*)malloc(sizeof(tb_node) * (size_t)(2 * nt + 1));
  for (int64_t i = 0; i < nt; ++i) {
    B->prim[i] = i;
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += verts[3 * (int64_t)tris[3 * i + k] + a];
      B->cen[3 * i + a] = s / 3.0;
    }
  }
  if (nt > 0) build_rec(B, 0, nt);
  return B;
}

void tb_free(void* p) {
  tb_bvh* B = (tb_bvh*)p;
  if (!B) return;
  free(B->prim);
  free(B->cen);
  free(B->nodes);
  free(B);
}

/* Moller-Trumbore; returns 1 on a hit inside [t0, t1] and writes t, u, v. */
static int mt_hit(const double* v0, const double* v1, const double* v2, const double o[3],
                  const double d[3], double t0, double t1, double* t, double* u, double* v) {
  double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
  double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
  double pv[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2],
                  d[0] * e2[1] - d[1] * e2[0]};
  double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
  double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  double n2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
  if (fabs(det) < 1e-12 * n1 * n2) return 0;
  double inv = 1.0 / det;
  double tv[3] = {o[0] - v0[0], o[1] - v0[1], o[2] - v0[2]};
  double uu = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
  if (uu < 0.0 || uu > 1.0) return 0;
  double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2],
                  tv[0] * e1[1] - tv[1] * e1[0]};
  double vv = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
  if (vv < 0.0 || uu + vv > 1.0) return 0;
  double tt = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
  if (!(tt >= t0 && tt <= t1)) return 0;
  *t = tt;
  *u = uu;
  *v = vv;
  return 1;
}

/* conservative slab test against [tmin, tmax]; zero direction components are
 * handled explicitly so no 0*inf appears */
static int box_hit(const tb_node* n, const double o[3], const double d[3], double tmin,
                   double tmax) {
  double tn = tmin, tf = tmax;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (o[a] < n->lo[a] || o[a] > n->hi[a]) return 0;
      continue;
    }
    double ta = (n->lo[a] - o[a]) / d[a], tb = (n->hi[a] - o[a]) / d[a];
    if (ta > tb) { double s = ta; ta = tb; tb = s; }
    if (ta > tn) tn = ta;
    if (tb < tf) tf = tb;
  }
  double slack = 1e-9 * (1.0 + fabs(tn) + fabs(tf));
  return tn <= tf + slack;
}

static void consider(int64_t tri, double t, double u, double v, double* bt, int64_t* bi,
                     double* bu, double* bv) {
  if (*bi < 0 || t < *bt || (t == *bt && tri < *bi)) {
    *bt = t;
    *bi = tri;
    *bu = u;
    *bv = v;
  }
}

void tb_closest(void* p, const double* o, const double* d, const double* t0, const double* t1,
                int64_t n, double* t_out, int64_t* tri_out, double* u_out, double* v_out) {
  const tb_bvh* B = (const tb_bvh*)p;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t r = 0; r < n; ++r) {
    const double* ro = o + 3 * r;
    const double* rd = d + 3 * r;
    double bt = 0.0, bu = 0.0, bv = 0.0;
    int64_t bi = -1;
    int64_t stack[128];
    int sp = 0;
    if (B->nt > 0) stack[sp++] = 0;
    while (sp > 0) {
      const tb_node* nd = &B->nodes[stack[--sp]];
      double tmax = (bi >= 0) ? bt : t1[r];
      double lo_t = t0[r] - 1e-9 * (1.0 + fabs(t0[r]));
      if (!box_hit(nd, ro, rd, lo_t, tmax)) continue;
      if (nd->b < 0) {
        for (int64_t k = 0; k < -nd->b; ++k) {
          int64_t tri = B->prim[nd->a + k];
          double t, u, v;
          if (mt_hit(B->v + 3 * (int64_t)B->t[3 * tri], B->v + 3 * (int64_t)B->t[3 * tri + 1],
                     B->v + 3 * (int64_t)B->t[3 * tri + 2], ro, rd, t0[r], t1[r], &t, &u, &v))
            consider(tri, t, u, v, &bt, &bi, &bu, &bv);
        }
      } else {
        stack[sp++] = nd->a;
        stack[sp++] = nd->b;
      }
    }
    t_out[r] = bt;
    tri_out[r] = bi;
    u_out[r] = bu;
    v_out[r] = bv;
  }
}

void tb_closest_brute(const double* verts, const int32_t* tris, int64_t nt, const double* o,
                      const double* d, const double* t0, const double* t1, int64_t n,
                      double* t_out, int64_t* tri_out, double* u_out, double* v_out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < n; ++r) {
    double bt = 0.0, bu = 0.0, bv = 0.0;
    int64_t bi = -1;
    for (int64_t tri = 0; tri < nt; ++tri) {
      double t, u, v;
      if (mt_hit(verts + 3 * (int64_t)tris[3 * tri], verts + 3 * (int64_t)tris[3 * tri + 1],
                 verts + 3 * (int64_t)tris[3 * tri + 2], o + 3 * r, d + 3 * r, t0[r], t1[r], &t,
                 &u, &v))
        consider(tri, t, u, v, &bt, &bi, &bu, &bv);
    }
    t_out[r] = bt;
    tri_out[r] = bi;
    u_out[r] = bu;
    v_out[r] = bv;
  }
}

/* ------------------------------------------------------------------------ */
/* Number of boxes each ray crosses (double precision, inclusive), used only */
/* to shape the segment-count mix of generated ray sets. A median-split BVH  */
/* over the boxes prunes the search.                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  double lo[3], hi[3];
  int64_t a, b; /* inner: children; leaf: a = box index, b = -1 */
} bx_node;

static const double* g_bx;
static int64_t bx_build_rec(bx_node* nodes, int64_t* n_nodes, int64_t* idx, int64_t first, int64_t count,
                            double* cen) {
  int64_t id = (*n_nodes)++;
  bx_node* n = &nodes[id];
  for (int a = 0; a < 3; ++a) {
    n->lo[a] = INFINITY;
    n->hi[a] = -INFINITY;
  }
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < count; ++i) {
    const double* bb = g_bx + 6 * idx[first + i];
    for (int a = 0; a < 3; ++a) {
      if (bb[a] < n->lo[a]) n->lo[a] = bb[a];
      if (bb[3 + a] > n->hi[a]) n->hi[a] = bb[3 + a];
      double c = cen[3 * idx[first + i] + a];
      if (c < clo[a]) clo[a] = c;
      if (c > chi[a]) chi[a] = c;
    }
  }
  if (count == 1) {
    n->a = idx[first];
    n->b = -1;
    return id;
  }
  int axis = 0;
  for (int a = 1; a < 3; ++a)
    if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
  int64_t half = count / 2;
  select_kth(idx + first, count, half, cen, axis);
  int64_t l = bx_build_rec(nodes, n_nodes, idx, first, half, cen);
  int64_t r = bx_build_rec(nodes, n_nodes, idx, first + half, count - half, cen);
  nodes[id].a = l;
  nodes[id].b = r;
  return id;
}

static int bx_hit(const double lo[3], const double hi[3], const double* o, const double* d) {
  double tn = 0.0, tf = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (o[a] < lo[a] || o[a] > hi[a]) return 0;
      continue;
    }
    double ta = (lo[a] - o[a]) / d[a], tb = (hi[a] - o[a]) / d[a];
    if (ta > tb) { double s = ta; ta = tb; tb = s; }
    if (ta > tn) tn = ta;
    if (tb < tf) tf = tb;
  }
  return tn <= tf;
}

void bx_count(const double* boxes, int64_t n_boxes, const double* o, const double* d, int64_t n_rays,
              int32_t* counts) {
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_boxes);
  double* cen = (double*)malloc(sizeof(double) * 3 * (size_t)n_boxes);
  bx_node* nodes = (bx_node*)malloc(sizeof(bx_node) * (size_t)(2 * n_boxes));
  for (int64_t i = 0; i < n_boxes; ++i) {
    idx[i] = i;
    for (int a = 0; a < 3; ++a) cen[3 * i + a] = 0.5 * (boxes[6 * i + a] + boxes[6 * i + 3 + a]);
  }
  int64_t nn = 0;
  g_bx = boxes;
  bx_build_rec(nodes, &nn, idx, 0, n_boxes, cen);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < n_rays; ++r) {
    int64_t stack[128];
    int sp = 0, c = 0;
    stack[sp++] = 0;
    while (sp) {
      const bx_node* nd = &nodes[stack[--sp]];
      if (!bx_hit(nd->lo, nd->hi, o + 3 * r, d + 3 * r)) continue;
      if (nd->b < 0) {
        ++c;
      } else {
        stack[sp++] = nd->a;
        stack[sp++] = nd->b;
      }
    }
    counts[r] = c;
  }
  free(idx);
  free(cen);
  free(nodes);
}
