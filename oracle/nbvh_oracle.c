/*
 * N-BVH neural ray query and training step: plain CPU ORACLE.
 *
 * This file is TEST INFRASTRUCTURE. It is the slow, obviously-correct
 * reference that the GPU library is checked against; nothing in the product
 * path may call it. It shares no code, header or table with the GPU library.
 *
 * Arithmetic is IEEE binary64 except where a floating-point result decides an
 * integer, which both implementations must take in the same precision:
 *   - the ray/box slab test (which leaves a ray visits), and
 *   - the sample positions whose floor picks the hash-grid cell.
 * Those two are defined in binary32, one rounding per operation, no fused
 * multiply-add (build with -ffp-contract=off). Everything after the cell
 * choice (interpolation weights, features, MLP, losses, gradients, Adam) is
 * binary64.
 *
 * Paper: "N-BVH: Neural ray queries with bounding volume hierarchies"
 * (SIGGRAPH 2024). Section names below refer to it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Network description (own copy; the GPU library has its own). */
typedef struct {
  int32_t n_levels, n_features, log2_T, n_samples;
  int32_t level_res[32];
  int32_t mlp_width, mlp_hidden, n_out;
  float scene_lo[3];
  float scene_side;
} oc_cfg;

/* ------------------------------------------------------------------------ */
/* Ray / box slab test in binary32 (Sec. 5: traversal of the N-BVH; the       */
/* visited leaves are those whose box the ray crosses inside [tmin, tmax]).   */
/* Per axis: a zero direction component only keeps rays whose origin lies in  */
/* the slab; otherwise the two plane distances use the correctly rounded      */
/* reciprocal of the direction, the near/far pair is ordered by the sign of   */
/* that reciprocal, and the interval shrinks by max/min. Hit iff tn <= tf.    */
/* *entry (if not NULL) receives where the ray's line enters the box: the     */
/* largest near-plane distance, without tmin (-inf if no axis constrains).    */
/* ------------------------------------------------------------------------ */
static int oc_slab_entry(const float* ray, const float* box, float* t0, float* t1, float* entry) {
  float tn = ray[3], tf = ray[7], te = -INFINITY;
  for (int a = 0; a < 3; ++a) {
    float o = ray[a], d = ray[4 + a];
    float lo = box[a], hi = box[3 + a];
    if (d == 0.0f) {
      if (o < lo || o > hi) return 0;
      continue;
    }
    float inv = 1.0f / d;
    float ta = (lo - o) * inv;
    float tb = (hi - o) * inv;
    if (inv < 0.0f) {
      float s = ta;
      ta = tb;
      tb = s;
    }
    tn = fmaxf(tn, ta);
    te = fmaxf(te, ta);
    tf = fminf(tf, tb);
  }
  *t0 = tn;
  *t1 = tf;
  if (entry) *entry = te;
  return tn <= tf;
}

static int oc_slab(const float* ray, const float* box, float* t0, float* t1) {
  return oc_slab_entry(ray, box, t0, t1, NULL);
}

int oc_slab_one(const float* ray, const float* box, float* t01) {
  return oc_slab(ray, box, &t01[0], &t01[1]);
}

/* Number of leaves each ray crosses (every leaf is tested; no tree). */
void oc_traverse_count(const float* rays, int64_t n_rays, const float* boxes, int64_t n_boxes,
                       uint32_t* counts) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < n_rays; ++r) {
    uint32_t c = 0;
    for (int64_t b = 0; b < n_boxes; ++b) {
      float t0, t1;
      c += (uint32_t)oc_slab(rays + 8 * r, boxes + 6 * b, &t0, &t1);
    }
    counts[r] = c;
  }
}

/* Segment list of each ray in front-to-back order: sorted by entry distance,
 * equal entries by leaf id. offsets = exclusive prefix sum of the counts.
 * reverse != 0 (queries from inside a leaf, the commented-out "Depth
 * estimation" passage of Sec. 6): a box whose chord starts before tmin holds
 * the ray origin; its segment is the whole chord [entry, t1] and its leaf id
 * carries the tag bit 2^31, so that it is queried backwards. */
#define OC_INSIDE_TAG 0x80000000u
void oc_traverse_fill(const float* rays, int64_t n_rays, const float* boxes, int64_t n_boxes,
                      const uint64_t* offsets, uint32_t* seg_ray, uint32_t* seg_leaf,
                      float* seg_t0, float* seg_t1, int reverse) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < n_rays; ++r) {
    uint64_t k = offsets[r];
    for (int64_t b = 0; b < n_boxes; ++b) {
      float t0, t1, entry;
      if (!oc_slab_entry(rays + 8 * r, boxes + 6 * b, &t0, &t1, &entry)) continue;
      uint32_t id = (uint32_t)b;
      if (reverse && entry < rays[8 * r + 3]) {
        t0 = entry;
        id |= OC_INSIDE_TAG;
      }
      /* insertion into the sorted run [offsets[r], k) */
      uint64_t j = k;
      while (j > offsets[r] && (seg_t0[j - 1] > t0 || (seg_t0[j - 1] == t0 && seg_leaf[j - 1] > id))) {
        seg_ray[j] = seg_ray[j - 1];
        seg_leaf[j] = seg_leaf[j - 1];
        seg_t0[j] = seg_t0[j - 1];
        seg_t1[j] = seg_t1[j - 1];
        --j;
      }
      seg_ray[j] = (uint32_t)r;
      seg_leaf[j] = id;
      seg_t0[j] = t0;
      seg_t1[j] = t1;
      ++k;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Sampling along the segment (Fig. "neural ray query pipeline"; Sec. 4      */
/* "Sampling & reconstruction quality"): S points spread uniformly over      */
/* [t0, t1] at the stratum midpoints t0 + (s + 1/2)/S (t1 - t0), then mapped */
/* into the unit cube of the scene and clamped. binary32, as explained above.*/
/* Segment rows are [o.xyz, t0, d.xyz, t1].                                  */
/* ------------------------------------------------------------------------ */
static void oc_sample_x(const oc_cfg* c, const float* seg, int s, float x[3]) {
  float t0 = seg[3], t1 = seg[7];
  float frac = ((float)s + 0.5f) / (float)c->n_samples;
  float span = t1 - t0;
  float step = frac * span;
  float ts = t0 + step;
  float inv_side = 1.0f / c->scene_side;
  for (int a = 0; a < 3; ++a) {
    float dp = ts * seg[4 + a];
    float p = seg[a] + dp;
    float rel = p - c->scene_lo[a];
    float xa = rel * inv_side;
    xa = xa < 0.0f ? 0.0f : xa;
    xa = xa > 1.0f ? 1.0f : xa;
    x[a] = xa;
  }
}

void oc_sample_positions(const oc_cfg* c, const float* segs, int64_t n, float* x_out) {
  for (int64_t i = 0; i < n; ++i)
    for (int s = 0; s < c->n_samples; ++s) oc_sample_x(c, segs + 8 * i, s, x_out + 3 * (i * c->n_samples + s));
}

/* ------------------------------------------------------------------------ */
/* Multiresolution hash encoding (Sec. 3 and Sec. 6 cite Mueller et al.      */
/* 2022 for it): level l has resolution N_l; its table holds (N_l+1)^3       */
/* entries indexed directly when that fits in T, else T entries addressed by  */
/* the spatial hash (x * 1) xor (y * 2654435761) xor (z * 805459861) mod T.   */
/* A point's feature is the trilinear blend of its cell's 8 corner entries.  */
/* Features of sample s, level l, feature f sit at s*L*F + l*F + f: samples  */
/* in ray order, which is what carries the direction (Sec. 4, "Encoding,     */
/* inference & training").                                                   */
/* ------------------------------------------------------------------------ */
static int64_t oc_level_entries(const oc_cfg* c, int l) {
  int64_t r1 = (int64_t)c->level_res[l] + 1;
  int64_t T = (int64_t)1 << c->log2_T;
  int64_t dense = r1 * r1 * r1;
  return dense <= T ? dense : T;
}

static int oc_level_is_dense(const oc_cfg* c, int l) {
  int64_t r1 = (int64_t)c->level_res[l] + 1;
  return r1 * r1 * r1 <= ((int64_t)1 << c->log2_T);
}

int64_t oc_table_params(const oc_cfg* c) {
  int64_t s = 0;
  for (int l = 0; l < c->n_levels; ++l) s += oc_level_entries(c, l) * c->n_features;
  return s;
}

static int64_t oc_level_offset(const oc_cfg* c, int l) {
  int64_t s = 0;
  for (int j = 0; j < l; ++j) s += oc_level_entries(c, j) * c->n_features;
  return s;
}

static uint32_t oc_corner_index(const oc_cfg* c, int l, const int64_t v[3]) {
  if (oc_level_is_dense(c, l)) {
    int64_t r1 = (int64_t)c->level_res[l] + 1;
    return (uint32_t)(v[0] + r1 * (v[1] + r1 * v[2]));
  }
  uint32_t h = ((uint32_t)v[0] * 1u) ^ ((uint32_t)v[1] * 2654435761u) ^ ((uint32_t)v[2] * 805459861u);
  return h & (uint32_t)((1u << c->log2_T) - 1u);
}

/* cell and weights of one point at one level: cell = floor(x N), kept
 * inside [0, N-1]; weights = x N - cell (exact in binary64) */
static void oc_cell(const oc_cfg* c, int l, const float x[3], int64_t cell[3], double w[3]) {
  int N = c->level_res[l];
  for (int a = 0; a < 3; ++a) {
    double y = (double)x[a] * (double)N;
    double fl = floor(y);
    if (fl > (double)(N - 1)) fl = (double)(N - 1);
    cell[a] = (int64_t)fl;
    w[a] = y - fl;
  }
}

static void oc_visit_corners(const oc_cfg* c, int l, const float x[3], double* wts, int64_t* idx) {
  int64_t cell[3];
  double w[3];
  oc_cell(c, l, x, cell, w);
  int64_t off = oc_level_offset(c, l);
  for (int k = 0; k < 8; ++k) {
    int64_t v[3];
    double wk = 1.0;
    for (int a = 0; a < 3; ++a) {
      int bit = (k >> a) & 1;
      v[a] = cell[a] + bit;
      wk *= bit ? w[a] : (1.0 - w[a]);
    }
    wts[k] = wk;
    idx[k] = off + (int64_t)oc_corner_index(c, l, v) * c->n_features;
  }
}

static void oc_encode_one(const oc_cfg* c, const double* table, const float* seg, double* u) {
  int L = c->n_levels, F = c->n_features;
  for (int s = 0; s < c->n_samples; ++s) {
    float x[3];
    oc_sample_x(c, seg, s, x);
    for (int l = 0; l < L; ++l) {
      double wts[8];
      int64_t idx[8];
      oc_visit_corners(c, l, x, wts, idx);
      for (int f = 0; f < F; ++f) {
        double acc = 0.0;
        for (int k = 0; k < 8; ++k) acc += wts[k] * table[idx[k] + f];
        u[s * L * F + l * F + f] = acc;
      }
    }
  }
}

static int oc_n_in(const oc_cfg* c) { return c->n_samples * c->n_levels * c->n_features; }

void oc_encode(const oc_cfg* c, const double* table, const float* segs, int64_t n, double* u) {
  int n_in = oc_n_in(c);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) oc_encode_one(c, table, segs + 8 * i, u + (int64_t)n_in * i);
}

/* ------------------------------------------------------------------------ */
/* MLP (Sec. 6, "Neural model & training"): ReLU hidden layers, no biases;   */
/* the last layer is linear here and the output activations (sigmoid for     */
/* hit and distance, identity for the normal) are applied by the consumers.  */
/* Weights: W_0 [width][n_in], W_1..W_{H-1} [width][width], W_H             */
/* [n_out][width], row-major, concatenated.                                  */
/* ------------------------------------------------------------------------ */
static void oc_layer_dims(const oc_cfg* c, int k, int* fan_in, int* fan_out) {
  int H = c->mlp_hidden;
  *fan_in = (k == 0) ? oc_n_in(c) : c->mlp_width;
  *fan_out = (k == H) ? c->n_out : c->mlp_width;
}

int64_t oc_mlp_params(const oc_cfg* c) {
  int64_t s = 0;
  for (int k = 0; k <= c->mlp_hidden; ++k) {
    int a, b;
    oc_layer_dims(c, k, &a, &b);
    s += (int64_t)a * b;
  }
  return s;
}

/* acts (optional): per segment, the pre-activations of each hidden layer,
 * [H][width] */
static void oc_mlp_one(const oc_cfg* c, const double* W, const double* u, double* z, double* pre_all,
                       double* h_buf /* 2*max_width */) {
  int H = c->mlp_hidden, width = c->mlp_width, n_in = oc_n_in(c);
  int maxw = n_in > width ? n_in : width;
  double* h = h_buf;
  double* hn = h_buf + maxw;
  memcpy(h, u, sizeof(double) * (size_t)n_in);
  const double* Wk = W;
  for (int k = 0; k <= H; ++k) {
    int fi, fo;
    oc_layer_dims(c, k, &fi, &fo);
    for (int o = 0; o < fo; ++o) {
      double acc = 0.0;
      for (int i = 0; i < fi; ++i) acc += Wk[(int64_t)o * fi + i] * h[i];
      if (k < H) {
        if (pre_all) pre_all[k * width + o] = acc;
        hn[o] = acc > 0.0 ? acc : 0.0;
      } else {
        z[o] = acc;
      }
    }
    Wk += (int64_t)fi * fo;
    double* t = h;
    h = hn;
    hn = t;
  }
}

void oc_mlp_forward(const oc_cfg* c, const double* W, const double* u, int64_t n, double* z) {
  int n_in = oc_n_in(c);
  int maxw = n_in > c->mlp_width ? n_in : c->mlp_width;
#pragma omp parallel
  {
    double* buf = (double*)malloc(sizeof(double) * 2 * (size_t)maxw);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      oc_mlp_one(c, W, u + (int64_t)n_in * i, z + (int64_t)c->n_out * i, NULL, buf);
    free(buf);
  }
}

/* Smallest |pre-activation| over the hidden units of each segment: where it
 * is within rounding of 0 the ReLU derivative (a 0/1 decision) is not fixed
 * by the arithmetic, so gradient comparisons leave such segments out. */
void oc_min_abs_preact(const oc_cfg* c, const double* params, const float* segs, int64_t n, double* out) {
  int64_t n_tab = oc_table_params(c);
  int n_in = oc_n_in(c), width = c->mlp_width, H = c->mlp_hidden;
  int maxw = n_in > width ? n_in : width;
#pragma omp parallel
  {
    double* u = (double*)malloc(sizeof(double) * (size_t)n_in);
    double* pre = (double*)malloc(sizeof(double) * (size_t)H * width);
    double* buf = (double*)malloc(sizeof(double) * 2 * (size_t)maxw);
    double* z = (double*)malloc(sizeof(double) * (size_t)c->n_out);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      oc_encode_one(c, params, segs + 8 * i, u);
      oc_mlp_one(c, params + n_tab, u, z, pre, buf);
      double m = INFINITY;
      for (int j = 0; j < H * width; ++j) m = fabs(pre[j]) < m ? fabs(pre[j]) : m;
      out[i] = m;
    }
    free(u);
    free(pre);
    free(buf);
    free(z);
  }
}

/* Largest magnitude of each layer's input over a batch: amax[0] = max |u|
 * over the encoded features, amax[k] = max h_k over the ReLU outputs of
 * hidden layer k (k = 1..H). These fix the per-layer scales of 8-bit
 * inference (value range of the format / amax). */
void oc_layer_amax(const oc_cfg* c, const double* params, const float* segs, int64_t n, double* amax) {
  int64_t n_tab = oc_table_params(c);
  int n_in = oc_n_in(c), width = c->mlp_width, H = c->mlp_hidden;
  int maxw = n_in > width ? n_in : width;
  for (int k = 0; k <= H; ++k) amax[k] = 0.0;
#pragma omp parallel
  {
    double* u = (double*)malloc(sizeof(double) * (size_t)n_in);
    double* pre = (double*)malloc(sizeof(double) * (size_t)H * width);
    double* buf = (double*)malloc(sizeof(double) * 2 * (size_t)maxw);
    double* z = (double*)malloc(sizeof(double) * (size_t)c->n_out);
    double* local = (double*)calloc((size_t)H + 1, sizeof(double));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      oc_encode_one(c, params, segs + 8 * i, u);
      oc_mlp_one(c, params + n_tab, u, z, pre, buf);
      for (int j = 0; j < n_in; ++j) local[0] = fabs(u[j]) > local[0] ? fabs(u[j]) : local[0];
      for (int k = 1; k <= H; ++k)
        for (int j = 0; j < width; ++j) {
          double h = pre[(size_t)(k - 1) * width + j] > 0.0 ? pre[(size_t)(k - 1) * width + j] : 0.0;
          local[k] = h > local[k] ? h : local[k];
        }
    }
#pragma omp critical
    for (int k = 0; k <= H; ++k) amax[k] = local[k] > amax[k] ? local[k] : amax[k];
    free(local);
    free(u);
    free(pre);
    free(buf);
    free(z);
  }
}

/* ------------------------------------------------------------------------ */
/* Losses (Sec. 5.2): visibility is a binary cross-entropy on a sigmoid;     */
/* the local distance (distance along the segment relative to its length,    */
/* in [0,1]) takes an L1 loss on a sigmoid output; the normal an L1 loss on  */
/* a linear output; the albedo (n_out >= 8: outputs 5..7 through a sigmoid) */
/* a relative L2 loss; all but visibility only where the label says the     */
/* segment is hit. Combined with weights 2, 2, 1, 1 ("Combined loss").      */
/* Means over the batch B. labels rows: [tau, n.xyz, hit, albedo.rgb].      */
/* loss_out: total, bce, dist, normal (the last three unweighted; the       */
/* albedo term only enters the total). dz (optional) = dL/dz.               */
/* Relative L2 of one channel: (a_hat - a)^2 / (a_hat^2 + 0.01), mean over  */
/* the three channels; the denominator only normalises the error and is     */
/* held constant in the derivative, as in relative L2 losses generally.     */
/* ------------------------------------------------------------------------ */
static double oc_sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }
static double oc_sgn(double v) { return (v > 0.0) - (v < 0.0); }
static const double kRelEps = 0.01;

static double oc_albedo_term(const double* zi, const float* lb, double* dterm /* [3] or NULL */) {
  double s = 0.0;
  for (int ch = 0; ch < 3; ++ch) {
    double ah = oc_sigmoid(zi[5 + ch]), a = (double)lb[5 + ch];
    double den = ah * ah + kRelEps;
    s += (ah - a) * (ah - a) / den;
    if (dterm) {
      /* 2 (a_hat - a) / (a_hat^2 + eps), the denominator held constant,   */
      /* times d a_hat / dz                                                 */
      double d = 2.0 * (ah - a) / den;
      dterm[ch] = d * ah * (1.0 - ah) / 3.0;
    }
  }
  return s / 3.0;
}

void oc_loss(const oc_cfg* c, const double* z, const float* labels, int64_t n, double w_hit, double w_t,
             double w_n, double w_a, double* loss_out, double* dz) {
  int no = c->n_out;
  double B = (double)n;
  double s_bce = 0.0, s_t = 0.0, s_n = 0.0, s_a = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double* zi = z + (int64_t)no * i;
    const float* lb = labels + 8 * i;
    double h = (double)lb[4];
    double tau = (double)lb[0];
    double z0 = zi[0];
    double bce = (z0 > 0.0 ? z0 : 0.0) - z0 * h + log1p(exp(-fabs(z0)));
    double st = oc_sigmoid(zi[1]);
    double lt = fabs(st - tau);
    double ln = 0.0;
    for (int a = 0; a < 3; ++a) ln += fabs(zi[2 + a] - (double)lb[1 + a]);
    ln /= 3.0;
    double da[3] = {0.0, 0.0, 0.0};
    double la = no >= 8 ? oc_albedo_term(zi, lb, da) : 0.0;
    s_bce += bce;
    s_t += h * lt;
    s_n += h * ln;
    s_a += h * la;
    if (dz) {
      double* g = dz + (int64_t)no * i;
      for (int o = 0; o < no; ++o) g[o] = 0.0;
      g[0] = w_hit * (oc_sigmoid(z0) - h) / B;
      g[1] = h * w_t * oc_sgn(st - tau) * st * (1.0 - st) / B;
      for (int a = 0; a < 3; ++a) g[2 + a] = h * w_n * oc_sgn(zi[2 + a] - (double)lb[1 + a]) / (3.0 * B);
      if (no >= 8)
        for (int ch = 0; ch < 3; ++ch) g[5 + ch] = h * w_a * da[ch] / B;
    }
  }
  loss_out[1] = s_bce / B;
  loss_out[2] = s_t / B;
  loss_out[3] = s_n / B;
  loss_out[0] = w_hit * loss_out[1] + w_t * loss_out[2] + w_n * loss_out[3] + w_a * s_a / B;
}

/* Combined loss of each segment on its own (Sec. 5.1, "Node error": the
 * training loss q of a node is taken over the segments that train it):
 * out[i] = w_hit BCE + h (w_t |sigma(z1) - tau| + w_n (1/3) sum |n_hat - n|
 * + w_a relative L2 of the albedo), not divided by the batch size. */
void oc_segment_loss(const oc_cfg* c, const double* z, const float* labels, int64_t n, double w_hit, double w_t,
                     double w_n, double w_a, double* out) {
  int no = c->n_out;
  for (int64_t i = 0; i < n; ++i) {
    const double* zi = z + (int64_t)no * i;
    const float* lb = labels + 8 * i;
    double h = (double)lb[4];
    double z0 = zi[0];
    double bce = (z0 > 0.0 ? z0 : 0.0) - z0 * h + log1p(exp(-fabs(z0)));
    double lt = fabs(oc_sigmoid(zi[1]) - (double)lb[0]);
    double ln = 0.0;
    for (int a = 0; a < 3; ++a) ln += fabs(zi[2 + a] - (double)lb[1 + a]);
    double la = no >= 8 ? oc_albedo_term(zi, lb, NULL) : 0.0;
    out[i] = w_hit * bce + h * (w_t * lt + w_n * ln / 3.0 + w_a * la);
  }
}

/* ------------------------------------------------------------------------ */
/* Back-propagation of dL/dz into every parameter (Sec. 4: the loss is       */
/* back-propagated to the learnable parameters): through the MLP layers      */
/* (ReLU derivative taken as 0 at 0), then into the hash-table entries with  */
/* the same trilinear weights as the forward pass. Encodings and activations */
/* are recomputed from the segments. grad has the parameter layout          */
/* [table | W_0 .. W_H] and is overwritten.                                  */
/* ------------------------------------------------------------------------ */
void oc_backward(const oc_cfg* c, const double* params, const float* segs, int64_t n, const double* dz,
                 double* grad) {
  int64_t n_tab = oc_table_params(c), n_mlp = oc_mlp_params(c);
  const double* W = params + n_tab;
  int H = c->mlp_hidden, width = c->mlp_width, n_in = oc_n_in(c), no = c->n_out;
  int L = c->n_levels, F = c->n_features, S = c->n_samples;
  int maxw = n_in > width ? n_in : width;
  memset(grad, 0, sizeof(double) * (size_t)(n_tab + n_mlp));
  double* du_all = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)n_in);
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  double* gW_part = (double*)calloc((size_t)nthreads * (size_t)n_mlp, sizeof(double));
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* gW = gW_part + (int64_t)tid * n_mlp;
    double* u = (double*)malloc(sizeof(double) * (size_t)n_in);
    double* pre = (double*)malloc(sizeof(double) * (size_t)H * width);
    double* buf = (double*)malloc(sizeof(double) * 2 * (size_t)maxw);
    double* z = (double*)malloc(sizeof(double) * (size_t)no);
    double* g = (double*)malloc(sizeof(double) * (size_t)maxw);
    double* gn = (double*)malloc(sizeof(double) * (size_t)maxw);
    double* hk = (double*)malloc(sizeof(double) * (size_t)maxw);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      oc_encode_one(c, params, segs + 8 * i, u);
      oc_mlp_one(c, W, u, z, pre, buf);
      /* offsets of each W_k */
      int64_t offs[34];
      offs[0] = 0;
      for (int k = 0; k <= H; ++k) {
        int fi, fo;
        oc_layer_dims(c, k, &fi, &fo);
        offs[k + 1] = offs[k] + (int64_t)fi * fo;
      }
      for (int o = 0; o < no; ++o) g[o] = dz[(int64_t)no * i + o];
      for (int k = H; k >= 0; --k) {
        int fi, fo;
        oc_layer_dims(c, k, &fi, &fo);
        /* input of layer k */
        if (k == 0) {
          memcpy(hk, u, sizeof(double) * (size_t)n_in);
        } else {
          for (int j = 0; j < fi; ++j) {
            double p = pre[(k - 1) * width + j];
            hk[j] = p > 0.0 ? p : 0.0;
          }
        }
        const double* Wk = W + offs[k];
        double* gWk = gW + offs[k];
        for (int o = 0; o < fo; ++o) {
          double go = g[o];
          if (go == 0.0) continue;
          for (int j = 0; j < fi; ++j) gWk[(int64_t)o * fi + j] += go * hk[j];
        }
        for (int j = 0; j < fi; ++j) {
          double acc = 0.0;
          for (int o = 0; o < fo; ++o) acc += Wk[(int64_t)o * fi + j] * g[o];
          if (k > 0) acc = pre[(k - 1) * width + j] > 0.0 ? acc : 0.0;
          gn[j] = acc;
        }
        double* t = g;
        g = gn;
        gn = t;
      }
      memcpy(du_all + (int64_t)n_in * i, g, sizeof(double) * (size_t)n_in);
    }
    free(u);
    free(pre);
    free(buf);
    free(z);
    free(g);
    free(gn);
    free(hk);
  }
  for (int t = 0; t < nthreads; ++t)
    for (int64_t j = 0; j < n_mlp; ++j) grad[n_tab + j] += gW_part[(int64_t)t * n_mlp + j];
  free(gW_part);
  /* table: sequential in segment order, so the sum order is fixed */
  for (int64_t i = 0; i < n; ++i) {
    const double* du = du_all + (int64_t)n_in * i;
    for (int s = 0; s < S; ++s) {
      float x[3];
      oc_sample_x(c, segs + 8 * i, s, x);
      for (int l = 0; l < L; ++l) {
        double wts[8];
        int64_t idx[8];
        oc_visit_corners(c, l, x, wts, idx);
        for (int k = 0; k < 8; ++k)
          for (int f = 0; f < F; ++f) grad[idx[k] + f] += wts[k] * du[s * L * F + l * F + f];
      }
    }
  }
  free(du_all);
}

/* ------------------------------------------------------------------------ */
/* Adam (Sec. 6: Adam, learning rate 0.01; Kingma & Ba 2015): dense update   */
/* of every parameter with bias-corrected moments. step = 1 for the first   */
/* update. grad is multiplied by inv_scale first (loss-scale removal).       */
/* ------------------------------------------------------------------------ */
void oc_adam(int64_t n, double* params, const double* grad, double* m, double* v, int64_t step, double lr,
             double beta1, double beta2, double eps, double inv_scale) {
  double c1 = 1.0 - pow(beta1, (double)step);
  double c2 = 1.0 - pow(beta2, (double)step);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double g = grad[i] * inv_scale;
    m[i] = beta1 * m[i] + (1.0 - beta1) * g;
    v[i] = beta2 * v[i] + (1.0 - beta2) * g * g;
    double mh = m[i] / c1, vh = v[i] / c2;
    params[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ------------------------------------------------------------------------ */
/* Resolve (Sec. 5: front-to-back queries of the leaves a ray reaches; Sec.  */
/* 5.2 "Visibility": the segment is hit when the sigmoid output exceeds 0.5, */
/* i.e. z0 > 0; "Intersection point": distance local to the segment). The    */
/* ray's hit is the smallest t0 + sigmoid(z1) (t1 - t0) over its hit         */
/* segments; equal t keeps the earlier segment. A tagged (inside) segment   */
/* was queried backwards from t1, so its local distance counts from t1:      */
/* t = t1 - sigmoid(z1) (t1 - t0), and it is a hit only in front of the      */
/* origin, t > tmin. out rows: [t, n.xyz, leaf (untagged, as double, -1 =    */
/* miss), seg index (-1), albedo.rgb].                                       */
/* ------------------------------------------------------------------------ */
void oc_resolve(int64_t n_rays, const uint64_t* offsets, const uint32_t* seg_leaf, const float* seg_t0,
                const float* seg_t1, const double* z, int n_out, const float* ray_tmin, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n_rays; ++r) {
    double best = INFINITY;
    int64_t bs = -1;
    for (uint64_t k = offsets[r]; k < offsets[r + 1]; ++k) {
      const double* zk = z + (int64_t)n_out * (int64_t)k;
      if (!(zk[0] > 0.0)) continue;
      const double a = (double)seg_t0[k], b = (double)seg_t1[k], tau = oc_sigmoid(zk[1]);
      double t;
      if (seg_leaf[k] & OC_INSIDE_TAG) {
        t = b - tau * (b - a);
        if (!(t > (double)ray_tmin[r])) continue;
      } else {
        t = a + tau * (b - a);
      }
      if (t < best) {
        best = t;
        bs = (int64_t)k;
      }
    }
    double* o = out + 9 * r;
    for (int j = 0; j < 9; ++j) o[j] = 0.0;
    if (bs < 0) {
      o[4] = -1.0;
      o[5] = -1.0;
      continue;
    }
    const double* zk = z + (int64_t)n_out * bs;
    o[0] = best;
    o[1] = zk[2];
    o[2] = zk[3];
    o[3] = zk[4];
    o[4] = (double)(seg_leaf[bs] & ~OC_INSIDE_TAG);
    o[5] = (double)bs;
    if (n_out >= 8)
      for (int a = 0; a < 3; ++a) o[6 + a] = oc_sigmoid(zk[5 + a]);
  }
}

/* ------------------------------------------------------------------------ */
/* Node error rank (Sec. 5.1, "Node error"): r = 2 log q + log p, where q is  */
/* the leaf's mean combined training loss (loss_sum / count over the          */
/* first-hit segments it received) and p the fraction of the n_rays sampled  */
/* rays that cross it (hits / n_rays). No segment, no crossing or a zero loss */
/* gives r = -inf.                                                            */
/* ------------------------------------------------------------------------ */
void oc_node_rank(int64_t n, const double* loss_sum, const int64_t* count, const int64_t* hits, int64_t n_rays,
                  double* r) {
  for (int64_t i = 0; i < n; ++i) {
    if (count[i] <= 0 || hits[i] <= 0 || n_rays <= 0) {
      r[i] = -INFINITY;
      continue;
    }
    const double q = loss_sum[i] / (double)count[i];
    const double p = (double)hits[i] / (double)n_rays;
    r[i] = 2.0 * log(q) + log(p);
  }
}

/* Acceptance probability of a leaf's first-hit training rays (Sec. 5.2, "Ray */
/* distribution"), read in linear space: a = max(exp(r - r_max), floor) over  */
/* the finite ranks, the floor for r = -inf, and 1 everywhere when no rank is */
/* finite.                                                                    */
void oc_acceptance(int64_t n, const double* r, double floor_, double* a) {
  double rmax = -INFINITY;
  for (int64_t i = 0; i < n; ++i)
    if (isfinite(r[i]) && r[i] > rmax) rmax = r[i];
  for (int64_t i = 0; i < n; ++i) {
    if (!isfinite(rmax)) {
      a[i] = 1.0;
      continue;
    }
    const double e = isfinite(r[i]) ? exp(r[i] - rmax) : 0.0;
    a[i] = e > floor_ ? e : floor_;
  }
}

int oc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
