/*
 * nbvh.h -- C ABI of the MI355X (gfx950) N-BVH library: neural ray queries
 * through a shallow BVH whose leaves are neural nodes, and the training step
 * of that network.
 *
 * Paper: "N-BVH: Neural ray queries with bounding volume hierarchies"
 * (Weier et al., SIGGRAPH 2024). Section references below are to it.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Pointers named *_dev are device (HBM) pointers; *_host are host
 *    pointers. The caller allocates and owns ALL device memory: nodes,
 *    parameters, optimiser state, workspace, inputs and outputs. The library
 *    keeps pointers and host metadata in its context and never frees caller
 *    memory.
 *  - `stream` is a hipStream_t (NULL = the null stream). Every call except
 *    nbvh_build and nbvh_read_state only enqueues work on that stream and
 *    returns; none of them synchronises the host, so the sequences are
 *    capturable in a HIP graph.
 *  - Return value: NBVH_OK or an error code. Argument errors are detected on
 *    the host before anything is enqueued; nbvh_last_error() then holds a
 *    message (per thread). Launch failures return NBVH_ERR_HIP.
 *  - Device-side conditions (segment capacity exceeded, non-finite
 *    gradients) set bits in the state block; nbvh_read_state reports them.
 *  - Structs are plain 4-byte-aligned records, laid out exactly as declared.
 */
#ifndef NBVH_H
#define NBVH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NBVH_OK = 0,
  NBVH_ERR_INVALID_ARG = 1, /* bad pointer, size or configuration */
  NBVH_ERR_CAPACITY = 2,    /* a caller buffer is too small */
  NBVH_ERR_NOT_BOUND = 3,   /* parameters not bound (nbvh_bind_params) */
  NBVH_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
  NBVH_ERR_UNSUPPORTED = 5  /* valid but not implemented shape/precision */
} nbvh_status;

/* Arithmetic of the MLP and of the feature reads in queries and training.
 * FP32: FP32 table reads and FP32 matrix-core products.
 * BF16: BF16 table shadow, BF16 activations and weights, FP32 accumulation.
 * FP8 : inference only (queries and nbvh_forward): BF16 table shadow, OCP
 *       E4M3 weights and activations (largest value 448) with one scale per
 *       layer, FP32 accumulation; set up by nbvh_calibrate_fp8. Training
 *       calls return NBVH_ERR_UNSUPPORTED. */
typedef enum { NBVH_FP32 = 0, NBVH_BF16 = 1, NBVH_FP8 = 2 } nbvh_precision;

/* Device-state flag bits (nbvh_state_host.flags). */
#define NBVH_FLAG_CAPACITY 1u  /* a traversal produced more segments than seg_capacity */
#define NBVH_FLAG_NONFINITE 2u /* a training step saw a non-finite loss/gradient and was skipped */

#define NBVH_MAX_LEVELS 32
#define NBVH_MISS 0xFFFFFFFFu

/* How a leaf that contains the ray origin (the ray's line enters the box
 * before tmin and leaves it after) is queried; nbvh_config.inside_rule.
 * CLIP   : the segment is the part of the box after tmin, [tmin, exit],
 *          sampled and encoded in ray order like any other.
 * REVERSE: the whole chord [entry, exit] of the box is queried in reverse,
 *          as the ray (o, -d) crossing it from the exit point, so the
 *          features are concatenated in the opposite order (the reversal
 *          rule of Sec. 6, a commented-out "Depth estimation" passage, and
 *          the convexity assumption of Sec. 9, "Limitations"). The reversed query
 *          predicts the last surface crossing of the chord; the leaf is hit
 *          only if that point lies in front of the origin (t > tmin). Such
 *          segments carry NBVH_SEG_INSIDE in their leaf field and store the
 *          chord [entry, exit] with entry < tmin. */
typedef enum { NBVH_INSIDE_CLIP = 0, NBVH_INSIDE_REVERSE = 1 } nbvh_inside_rule;
#define NBVH_SEG_INSIDE 0x80000000u

/* A ray: origin, [tmin, tmax], direction (not necessarily unit length).
 * Direction components must be 0 or normal floats. 32 bytes. */
typedef struct {
  float o[3];
  float tmin;
  float d[3];
  float tmax;
} nbvh_ray;

/* One ray/leaf crossing: [t0, t1] is the part of the ray's [tmin, tmax]
 * inside the leaf box (Sec. 5: inference queries the model on each leaf a
 * ray reaches). Under NBVH_INSIDE_REVERSE a leaf containing the origin has
 * leaf = id | NBVH_SEG_INSIDE and [t0, t1] = the whole chord (t0 < tmin).
 * Runs are sorted by (t0, leaf). 16 bytes. */
typedef struct {
  uint32_t ray;
  uint32_t leaf;
  float t0;
  float t1;
} nbvh_segment;

/* A training/forward segment: ray origin o, direction d and the leaf
 * interval [t0, t1] to sample (Sec. 4, "Encoding, inference & training").
 * 32 bytes. */
typedef struct {
  float o[3];
  float t0;
  float d[3];
  float t1;
} nbvh_probe;

/* Ground truth of a probe (Sec. 5.2): tau = (t_hit - t0)/(t1 - t0) in [0,1]
 * (local distance), unit normal n, hit = 1.0f if the geometry is hit inside
 * the segment else 0.0f, albedo (unused unless n_out >= 8). 32 bytes. */
typedef struct {
  float tau;
  float n[3];
  float hit;
  float albedo[3];
} nbvh_label;

/* Result of a neural ray query: the closest predicted hit over the leaves
 * the ray crosses. t is along the ray; n is the raw (linear) normal output;
 * albedo is the sigmoid output when n_out >= 8, else 0; leaf = NBVH_MISS
 * when no segment is predicted hit (then the other fields are 0). 32 bytes. */
typedef struct {
  float t;
  float n[3];
  float albedo[3];
  uint32_t leaf;
} nbvh_hit;

/* Network and training description (Sec. 3, Sec. 6). Level l has
 * resolution level_res[l] (N_l); a level whose (N_l+1)^3 entries fit in
 * T = 2^log2_T is indexed densely, otherwise by the spatial hash
 * (x*1 xor y*2654435761 xor z*805459861) mod T. Each segment is sampled at
 * n_samples stratum midpoints; the MLP input is the concatenation
 * n_in = n_samples * n_levels * n_features (sample-major, then level, then
 * feature), followed by mlp_hidden ReLU layers of mlp_width and a linear
 * output layer of n_out (hit logit, local-distance logit, normal xyz
 * [, albedo logits rgb]). Sample positions are mapped into the cube
 * [scene_lo, scene_lo + scene_side]^3 and clamped to it.
 * Supported: n_features in {2, 4}; n_in % 32 == 0; mlp_width in
 * {32, 64, 128, 256}; 1 <= mlp_hidden <= 8; 5 <= n_out <= 16;
 * 1 <= n_levels <= 32; 1 <= n_samples <= 16; 1 <= log2_T <= 24.
 * Loss weights w_* (Sec. 5.2 "Combined loss": 2, 2, 1, 1) and Adam
 * hyper-parameters (Sec. 6: learning rate 0.01) drive nbvh_train_step;
 * loss_scale multiplies dL/dz before back-propagation and is divided out
 * in the optimiser. */
typedef struct {
  int32_t n_levels, n_features, log2_T, n_samples;
  int32_t level_res[NBVH_MAX_LEVELS];
  int32_t mlp_width, mlp_hidden, n_out;
  int32_t precision; /* nbvh_precision */
  float scene_lo[3];
  float scene_side;
  float w_hit, w_t, w_normal, w_albedo; /* loss weights (Sec. 5.2: 2, 2, 1, 1); albedo only with n_out >= 8 */
  float lr, beta1, beta2, eps, loss_scale;
  int32_t inside_rule; /* nbvh_inside_rule: queries and training-ray selection (NBVH_INSIDE_CLIP) */
} nbvh_config;

/* Caller-owned device buffers of the learnable state. All FP32 arrays have
 * n_params = n_table + n_mlp entries laid out as [hash table | W_0 | ... |
 * W_H]: the table level-major, then entry, then feature; each W_k row-major
 * [fan_out][fan_in] (no biases); each block starts on a 64-element
 * boundary and the gaps are zero (nbvh_param_layout gives the offsets).
 * params_lp is the BF16 shadow of params in
 * the same layout (written by nbvh_sync_shadow and by every Adam step);
 * it may be NULL only if precision is FP32. grad accumulates dL/dparams
 * (times loss_scale) and is cleared by each optimiser step. state_dev is
 * nbvh_state_bytes() bytes. Every buffer must be 16-byte aligned
 * (nbvh_bind_params returns NBVH_ERR_INVALID_ARG otherwise). */
typedef struct {
  float* params_dev;
  void* params_lp_dev;
  float* adam_m_dev;
  float* adam_v_dev;
  float* grad_dev;
  void* state_dev;
  void* aux_dev; /* nbvh_aux_bytes(cfg) bytes: transposed weight copies read by back-propagation,
                    then the FP8 weights and scales */
} nbvh_params;

/* Host copy of the device state block. */
typedef struct {
  int64_t step;        /* optimiser steps applied */
  int64_t skipped;     /* steps skipped because of non-finite gradients */
  float loss_scale;    /* current loss scale */
  uint32_t flags;      /* NBVH_FLAG_* bits, sticky until nbvh_clear_flags */
  float last_loss[4];  /* last train step: total, BCE, distance L1, normal L1 (unweighted; the
                          albedo term only enters the total) */
  uint64_t last_n_segments; /* segments produced by the last traversal */
  uint64_t n_evaluated;     /* segments evaluated by queries since the last nbvh_reset_optimizer */
} nbvh_state_host;

typedef struct nbvh_ctx nbvh_ctx; /* opaque host handle */

/* Launch-shape knobs (defaults shown). Results do not depend on them beyond
 * floating-point summation order; an autotuner may search them. Changing
 * wgrad_splits, scatter_lds_kb, scatter_binned or scatter_hash_levels changes
 * nbvh_workspace_bytes. */
typedef struct {
  int32_t query_waves;      /* waves per query workgroup: 4 or 8 (8) */
  int32_t query_unroll;     /* (sample, level) pairs gathered together: 2, 3, 4; 0 = 2, or 3 with pair
                               loads of 4-byte entries (0) */
  int32_t query_wgs_per_cu; /* persistent query workgroups per compute unit; 0 = as many as LDS allows (0) */
  int32_t train_waves;      /* waves per training-tile workgroup: 4 or 8 (8) */
  int32_t wgrad_splits;     /* batch splits of the weight-gradient GEMMs: 1..256 (64) */
  int32_t scatter_lds_kb;   /* LDS budget for coarse dense levels held whole per compute unit in the
                               table-gradient scatter: 0..144 (0) */
  int32_t scatter_binned;   /* levels after the LDS and hash levels: 1 = counting sort by 64 KiB table
                               chunk, then per-chunk LDS accumulation (no global atomics); 0 = coalesced
                               global atomics (1) */
  int32_t scatter_hash_levels; /* levels after the LDS ones whose gradient is summed per 256-probe tile in
                                  an LDS hash table before the global atomics: 0..32 (8) */
  int32_t query_pairs;      /* 1 = fetch the x-neighbour corners of a cell with one load where they are
                               adjacent in the table; 0 = one load per corner (0) */
  int32_t query_lds_kb;     /* LDS per query workgroup for the table's leading (coarse) levels, copied
                               there whole once per workgroup and gathered from LDS; as many leading
                               levels as fit, none if the first does not; ignored with query_pairs
                               and by grouped queries: 0..64 (0) */
  int32_t traverse_mode;    /* how a wave walks the tree: 0 = each lane its own ray (per-lane stacks),
                               1 = the wave together over the union of its rays' nodes (one node load
                               per wave), 2 = the wave together when its rays are coherent (directions
                               and origins close), else each lane alone (2) */
  int32_t query_order;      /* the order the rays are traversed and evaluated in (a stable radix sort
                               of the rays by a Morton key before the traversal; every ray keeps its
                               index): 0 = the caller's; 1 = by the origin's cell (8 bits per axis of
                               the box of the ray origins), so that rays leaving one region of the
                               scene share a wave whatever the caller's order (bounce rays of several
                               samples per pixel); 2 = by the origin's cell (6 bits per axis) and the
                               direction's cell (6 bits per axis of its octahedral map), for
                               incoherent rays. Results do not change; 1 and 2 enlarge the query
                               workspace by about 16 bytes per ray; grouped queries follow the first
                               object's setting, with one order for all objects (0) */
} nbvh_tuning;

/* Read / replace the context's launch knobs (validated). */
nbvh_status nbvh_get_tuning(const nbvh_ctx* ctx, nbvh_tuning* out);
nbvh_status nbvh_set_tuning(nbvh_ctx* ctx, const nbvh_tuning* t);

/* Parameter counts for a configuration (no context needed). Returns
 * NBVH_ERR_INVALID_ARG for unsupported configurations. */
nbvh_status nbvh_param_count(const nbvh_config* cfg, uint64_t* n_table, uint64_t* n_mlp);

/* Offsets (elements) of the parameter blocks: offsets[0] = 0 is the hash
 * table, offsets[1 + k] the start of W_k (k = 0..mlp_hidden), and
 * offsets[mlp_hidden + 2] the total n_params. `offsets` must hold
 * mlp_hidden + 3 entries. */
nbvh_status nbvh_param_layout(const nbvh_config* cfg, uint64_t* offsets);

/* Bytes of the auxiliary buffer: transposed FP32 and BF16 weight copies
 * (rewritten by nbvh_sync_shadow and every optimiser step), then E4M3
 * weights and per-layer scales (written by nbvh_calibrate_fp8). */
size_t nbvh_aux_bytes(const nbvh_config* cfg);

/* Bytes of the node buffer nbvh_build writes for n_leaves leaves:
 * max(1, n_leaves - 1) nodes of 64 bytes, node 0 the root. A node holds the
 * boxes of its two children and their indices: float lo0[3], hi0[3],
 * lo1[3], hi1[3]; int32 c0, c1; int32 pad[2]. A child index c >= 0 is the
 * inner node c (always after its parent), c < 0 the leaf ~c; c1 = 0x7fffffff
 * marks the missing second child of a single-leaf tree. The layout is fixed
 * so that callers may read the tree (for instance to count the nodes a ray
 * visits); the library only reads the buffer after nbvh_build. */
size_t nbvh_nodes_bytes(uint32_t n_leaves);

/* Bytes of the device state block. */
size_t nbvh_state_bytes(void);

/* Build the N-BVH over the neural leaves (Sec. 5, Fig. "pipeline": a
 * shallow BVH whose leaves are hollow boxes). leaf_boxes_host is
 * [n_leaves][6] floats (lo.xyz, hi.xyz), leaf ids are row indices. The
 * tree is a median split of leaf centroids on the widest axis; every inner
 * box is the exact min/max union of its children, so the tree visits
 * exactly the leaves an every-leaf slab test would. Nodes are copied to
 * nodes_dev (nbvh_nodes_bytes(n_leaves) bytes, caller-owned) and the call
 * synchronises `stream` once. *out receives a new context (nbvh_destroy). */
nbvh_status nbvh_build(const nbvh_config* cfg, const float* leaf_boxes_host, uint32_t n_leaves,
                       void* nodes_dev, size_t nodes_bytes, void* stream, nbvh_ctx** out);

/* Attach the learnable state. Pointers are kept until the next bind. */
nbvh_status nbvh_bind_params(nbvh_ctx* ctx, const nbvh_params* p);

/* Reset optimiser state: m = v = grad = 0, step = 0, loss scale =
 * cfg.loss_scale, flags cleared; and write the BF16 shadow of params. */
nbvh_status nbvh_reset_optimizer(nbvh_ctx* ctx, void* stream);

/* Rewrite the BF16 shadow from the FP32 params (after the caller edits
 * params directly). */
nbvh_status nbvh_sync_shadow(nbvh_ctx* ctx, void* stream);

/* FP8 inference set-up (precision FP8 only; the MLP of Sec. 4 run at 8 bits).
 * Weight scale of layer k: sw_k = 448 / max|W_k| over the FP32 master
 * weights. Activation scale of layer k's input: sa_k = 448 / max|h_k|, the
 * maximum taken over an FP32 forward (BF16 table reads, FP32 weights) of the
 * n calibration segments probes_dev (device, [n]); a zero maximum gives
 * scale 1. Writes E4M3 weights fp8(W_k * sw_k) and the scales into aux.
 * A query then stores fp8(h_k * sa_k) in LDS, multiplies on the FP8 matrix
 * cores with FP32 accumulation and divides by sw_k * sa_k; values beyond the
 * calibrated range saturate at +-448. Must be called again after any change
 * of the parameters (nbvh_bind_params, nbvh_sync_shadow,
 * nbvh_reset_optimizer and nbvh_optimizer_step invalidate it); until then
 * FP8 queries and nbvh_forward return NBVH_ERR_NOT_BOUND. Asynchronous on
 * `stream`; NBVH_ERR_INVALID_ARG for n = 0, a NULL buffer or a non-FP8 context. */
nbvh_status nbvh_calibrate_fp8(nbvh_ctx* ctx, const nbvh_probe* probes_dev, uint64_t n, void* stream);

/* Workspace bytes for queries of up to max_rays rays producing up to
 * max_segments segments, and for training/forward/backward batches of up to
 * max_batch probes. One workspace may serve all calls (not concurrently). */
size_t nbvh_workspace_bytes(const nbvh_ctx* ctx, uint64_t max_rays, uint64_t max_segments,
                            uint64_t max_batch);

/* Traversal only (Sec. 5: front-to-back N-BVH traversal with empty-space
 * skipping): writes seg_offsets_dev[n_rays + 1] (exclusive prefix sum of
 * per-ray counts) and, if the total fits seg_capacity, segs_dev[total] with
 * each ray's run sorted by (t0, leaf id). Slab tests are binary32, one
 * rounding per operation, correctly rounded reciprocals. On overflow the
 * offsets are still complete, segments are not written and
 * NBVH_FLAG_CAPACITY is set. */
nbvh_status nbvh_traverse(nbvh_ctx* ctx, const nbvh_ray* rays_dev, uint64_t n_rays,
                          uint32_t* seg_offsets_dev, nbvh_segment* segs_dev, uint64_t seg_capacity,
                          void* ws_dev, size_t ws_bytes, void* stream);

/* Neural ray query (Sec. 5; Fig. "neural ray query pipeline"): traversal,
 * then for each ray its segments front to back: sample, encode, MLP,
 * predicted hit when the hit logit z0 > 0 at t = t0 + sigmoid(z1)(t1 - t0).
 * The ray's answer is the smallest such t (ties: earlier segment); a ray
 * stops evaluating once its next segment starts at or after its best t,
 * which cannot change the answer. seg_capacity bounds the segment queue in
 * the workspace (see nbvh_traverse for overflow). Writes hits_dev[n_rays]. */
nbvh_status nbvh_query(nbvh_ctx* ctx, const nbvh_ray* rays_dev, uint64_t n_rays, nbvh_hit* hits_dev,
                       uint64_t seg_capacity, void* ws_dev, size_t ws_bytes, void* stream);

/* nbvh_query for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, with the query's workspace taken from a
 * library-owned static device buffer of 64 MiB instead of a caller workspace.
 * Each GPU the library runs on holds its own copy until the process ends.
 * The workspace of a query is 16 bytes per ray for offsets, counts, the
 * active list and its positions, 192 bytes per ray of traversal staging, 16 bytes per segment
 * of capacity, plus a few hundred bytes of counters and scan partials,
 * each part rounded up to 256 bytes; a query needing more than 64 MiB returns
 * NBVH_ERR_CAPACITY before enqueuing anything (about 200,000 rays at 8
 * segments of capacity per ray fit). The call allocates nothing. Every call
 * on one GPU shares that GPU's buffer, whatever the context: calls that may
 * overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller. Each call clears the counters it uses; the
 * buffer otherwise keeps the last call's contents. */
nbvh_status nbvh_query_noalloc(nbvh_ctx* ctx, const nbvh_ray* rays_dev, uint64_t n_rays, nbvh_hit* hits_dev,
                               uint64_t seg_capacity, void* stream);

/* Optional outputs of nbvh_query_traced (each pointer nullable, device):
 * seg_offsets_dev [n_rays + 1] and segs_dev [seg_capacity] receive the
 * segment queue the traversal built (as nbvh_traverse writes them; the
 * segments only if they fit); z_dev [seg_capacity][n_out] receives the raw
 * network outputs of every segment the query evaluates and u_dev
 * [seg_capacity][n_in] the encoded features the MLP read for it (FP32 copies
 * of the values in the kernel's feature tile: BF16-rounded under BF16; not
 * available under FP8), both at the segment's position in the queue. Rows of
 * segments skipped by early termination are left untouched, so a caller that
 * fills them with NaN first can tell which segments were evaluated. */
typedef struct {
  uint32_t* seg_offsets_dev;
  nbvh_segment* segs_dev;
  float* z_dev;
  float* u_dev;
} nbvh_query_trace;

/* nbvh_query with the same kernels and launch shapes, also writing the
 * outputs `trace` asks for (Sec. 5; Fig. "neural ray query pipeline": the
 * per-leaf network queries behind each hit record). For checking a query
 * against a reference segment by segment; `trace` must not be NULL.
 * NBVH_ERR_UNSUPPORTED for a feature trace under FP8. */
nbvh_status nbvh_query_traced(nbvh_ctx* ctx, const nbvh_ray* rays_dev, uint64_t n_rays, nbvh_hit* hits_dev,
                              uint64_t seg_capacity, void* ws_dev, size_t ws_bytes,
                              const nbvh_query_trace* trace, void* stream);

/* Query over a caller-given segment queue (offsets/segments as written by
 * nbvh_traverse): evaluation and resolve only. */
nbvh_status nbvh_query_segments(nbvh_ctx* ctx, const nbvh_ray* rays_dev, uint64_t n_rays,
                                const uint32_t* seg_offsets_dev, const nbvh_segment* segs_dev,
                                nbvh_hit* hits_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Training-ray selection for the error-driven construction (Sec. 5.2, "Ray
 * distribution" and "Node error"). For each of the n_rays rays (device,
 * typically sampled uniformly in the inflated root box) the N-BVH is
 * traversed as by nbvh_traverse; the first leaf crossed (smallest t0, ties
 * to the lower leaf id) is kept iff u_dev[r] < accept_dev[leaf] (u_dev:
 * [n_rays] caller-drawn uniforms in [0, 1); accept_dev: [n_leaves]
 * acceptance probabilities). Kept segments are written to probes_dev as
 * (o, t0, d, t1) (under NBVH_INSIDE_REVERSE a first leaf that contains the
 * origin gives the reversed chord (o, -exit, -d, -entry), the probe such a
 * leaf is queried with) with their leaf id in leaf_ids_dev, in an unspecified
 * order; both need room for n_rays entries. *n_out_dev (device) receives the
 * number kept (cleared by the call). If leaf_hits_dev is not NULL, every
 * leaf crossed by a ray has its counter incremented (the caller clears it),
 * the numerator of the node's hit-probability estimate. Asynchronous. */
nbvh_status nbvh_first_hits(nbvh_ctx* ctx, const nbvh_ray* rays_dev, uint64_t n_rays, const float* u_dev,
                            const float* accept_dev, nbvh_probe* probes_dev, uint32_t* leaf_ids_dev,
                            uint32_t* n_out_dev, uint32_t* leaf_hits_dev, void* stream);

/* Training probes grouped by leaf (Sec. 5.2: each training ray trains the
 * first leaf it crosses, so a batch mixes leaves in ray order). Writes the n
 * probes of probes_dev to probes_out_dev ordered by their leaf ids
 * (leaf_ids_dev, as written by nbvh_first_hits), increasing, keeping the
 * input order among probes of one leaf; the sorted ids go to leaf_ids_out_dev
 * if it is not NULL (it may be leaf_ids_dev). Ids are compared on the bits
 * that ids below the context's leaf count use; higher bits are carried
 * along. The training kernels then find a leaf's probes side by side, which
 * keeps their table lines in one die's L2 and lets the per-tile gradient
 * sums merge a leaf's entries. probes_out_dev must not alias probes_dev.
 * ws_dev: nbvh_group_ws_bytes(n) bytes (nbvh_workspace_bytes with
 * max_batch >= n covers it). Deterministic. Asynchronous. */
size_t      nbvh_group_ws_bytes(uint64_t n);
nbvh_status nbvh_group_by_leaf(nbvh_ctx* ctx, const nbvh_probe* probes_dev, const uint32_t* leaf_ids_dev,
                               uint64_t n, nbvh_probe* probes_out_dev, uint32_t* leaf_ids_out_dev, void* ws_dev,
                               size_t ws_bytes, void* stream);

/* Per-leaf training loss (Sec. 5.1, "Node error"): runs the network on the n
 * segments probes_dev with labels_dev and adds each segment's combined loss
 * (weights w_hit, w_t, w_normal, w_albedo; not divided by the batch size) to
 * leaf_loss_dev[leaf_ids_dev[i]] (float, [n_leaves]) and one to
 * leaf_count_dev[...] (uint32). The caller clears both. Needs n * n_out
 * floats of workspace. Asynchronous; atomics make the sums' rounding order
 * unspecified. */
nbvh_status nbvh_leaf_loss(nbvh_ctx* ctx, const nbvh_probe* probes_dev, const nbvh_label* labels_dev,
                           const uint32_t* leaf_ids_dev, uint64_t n, float* leaf_loss_dev,
                           uint32_t* leaf_count_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Node error rank of each leaf for the error-driven construction (Sec. 5.1,
 * "Node error"): rank_dev[i] = 2 log q + log p with q = leaf_loss_dev[i] /
 * leaf_count_dev[i] (the mean combined loss of the leaf's first-hit training
 * segments, as nbvh_leaf_loss sums them) and p = leaf_hits_dev[i] / n_rays
 * (the fraction of the n_rays sampled rays crossing the leaf, as
 * nbvh_first_hits counts them); -inf where the count, the crossings or the
 * loss is zero. Binary32, all arrays [n_leaves] on the device. No context
 * needed. Asynchronous. */
nbvh_status nbvh_node_rank(const float* leaf_loss_dev, const uint32_t* leaf_count_dev, const uint32_t* leaf_hits_dev,
                           uint32_t n_leaves, uint64_t n_rays, float* rank_dev, void* stream);

/* Per-leaf acceptance probability of first-hit training rays (Sec. 5.2,
 * "Ray distribution"): accept_dev[i] = max(exp(r_i - r_max), min_accept)
 * over the finite ranks of rank_dev, min_accept where r_i = -inf, and 1 for
 * every leaf when no rank is finite. The paper writes max(r / r_max, 0.005);
 * with r a sum of logarithms of numbers below one that ratio inverts the
 * order, so it is taken in linear space (q^2 p relative to its maximum).
 * min_accept in [0, 1]. One workgroup; asynchronous. */
nbvh_status nbvh_acceptance(const float* rank_dev, uint32_t n_leaves, float min_accept, float* accept_dev,
                            void* stream);

/* Encoding only (Sec. 3/4): u_dev[n][n_in] FP32 features of each probe's
 * samples, read from the FP32 table (precision FP32) or the BF16 shadow. */
nbvh_status nbvh_encode(nbvh_ctx* ctx, const nbvh_probe* probes_dev, uint64_t n, float* u_dev,
                        void* stream);

/* Network outputs z_dev[n][n_out] (raw: logits and linear normal) for
 * probe segments, in the configured precision. */
nbvh_status nbvh_forward(nbvh_ctx* ctx, const nbvh_probe* probes_dev, uint64_t n, float* z_dev,
                         void* ws_dev, size_t ws_bytes, void* stream);

/* Back-propagate dz_dev[n][n_out] (= dL/dz) into grad_dev (ADDED to it,
 * scaled by the current loss scale), recomputing encodings and activations
 * instead of storing them (Sec. 4: the loss is back-propagated into the
 * MLP weights and the hash-table features). */
nbvh_status nbvh_backward(nbvh_ctx* ctx, const nbvh_probe* probes_dev, uint64_t n,
                          const float* dz_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Adam step over all parameters from grad_dev (Sec. 6: Adam, lr 0.01):
 * unscale by the loss scale, bias-corrected moments, update params, write
 * the BF16 shadow, clear grad. If the gradient holds a non-finite value
 * the update is skipped, the loss scale halves and NBVH_FLAG_NONFINITE is
 * set. */
nbvh_status nbvh_optimizer_step(nbvh_ctx* ctx, void* stream);

/* One training step (Sec. 4, Sec. 5.2): forward on the probes, combined
 * loss L = (1/B) sum [w_hit BCE(z0, hit) + hit (w_t |sigmoid(z1) - tau| +
 * w_normal/3 sum |z2..4 - n| + w_albedo/3 sum_c (a_c - alb_c)^2 / (a_c^2 + 0.01))]
 * with a_c = sigmoid(z_{5+c}) (the relative-L2 albedo term only when
 * n_out >= 8), back-propagation into grad and an optimiser step. loss_dev
 * (nullable) receives [total, bce, dist, normal] as FP32 (unweighted terms;
 * total weighted, albedo included). Here and in nbvh_backward, a batch
 * whose binned table-gradient pass would need more than 2^32 records
 * (n * binned levels * n_samples * 8) returns NBVH_ERR_UNSUPPORTED before
 * any launch; split such batches. Both calls run the table gradient's
 * hash-route levels and the weight-gradient kernels on a second stream that
 * the context owns, forked from `stream` after the training tile and joined
 * back into it after the other table-gradient kernels, so work the caller
 * enqueues on `stream` afterwards sees all of them; while `stream` is being
 * captured into a graph they use `stream` alone. */
nbvh_status nbvh_train_step(nbvh_ctx* ctx, const nbvh_probe* probes_dev, const nbvh_label* labels_dev,
                            uint64_t n, float* loss_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Loss and dL/dz only (no back-propagation): dz_dev may be NULL. */
nbvh_status nbvh_loss(nbvh_ctx* ctx, const float* z_dev, const nbvh_label* labels_dev, uint64_t n,
                      float* loss_dev, float* dz_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* ---- Several N-BVH objects in one scene --------------------------------
 * Objects that share the network shape (levels, features, samples, level
 * resolutions, MLP, precision; table sizes may differ) are grouped so that a
 * ray batch is answered in one evaluation launch: each object is traversed,
 * one persistent kernel drains every object's ray queue (a workgroup's tile
 * always holds segments of a single object, so the MLP runs on that object's
 * weights), and a merge keeps each ray's closest predicted hit across
 * objects (ties: lower object index). In batch hit records
 * leaf = (object << 24) | leaf id. At most 16 objects of fewer than 2^24
 * leaves each. The contexts must stay alive while the batch is used. */
typedef struct nbvh_batch nbvh_batch;

/* Device bytes of the per-object descriptor table. */
size_t nbvh_batch_desc_bytes(uint32_t n_objects);

/* Validate and group the objects; uploads their descriptors into
 * descs_dev (caller-owned) and synchronises `stream` once. */
nbvh_status nbvh_batch_create(nbvh_ctx* const* ctxs, uint32_t n_objects, void* descs_dev, size_t descs_bytes,
                              void* stream, nbvh_batch** out);

/* Workspace bytes for batch queries of up to max_rays rays with up to
 * seg_capacity segments per object. */
size_t nbvh_batch_workspace_bytes(const nbvh_batch* b, uint64_t max_rays, uint64_t seg_capacity);

/* Neural ray query against all objects of the batch (see nbvh_query for the
 * per-object semantics). */
nbvh_status nbvh_batch_query(nbvh_batch* b, const nbvh_ray* rays_dev, uint64_t n_rays, nbvh_hit* hits_dev,
                             uint64_t seg_capacity, void* ws_dev, size_t ws_bytes, void* stream);

void nbvh_batch_destroy(nbvh_batch* b);

/* Kernel groups reported by the profiler. */
typedef enum {
  NBVH_K_TRAVERSE = 0,   /* count + scan + fill */
  NBVH_K_QUERY_EVAL = 1, /* fused encode + MLP + resolve */
  NBVH_K_FORWARD = 2,    /* forward tile kernel */
  NBVH_K_TRAIN_TILE = 3, /* fused encode + forward + loss + dgrad */
  NBVH_K_WGRAD = 4,      /* weight-gradient GEMMs + reduction */
  NBVH_K_SCATTER = 5,    /* table-gradient scatter: LDS levels, per-tile hash levels, direct atomics */
  NBVH_K_OPTIMIZER = 6,  /* finite check + Adam */
  NBVH_K_SCATTER_SORT = 7,   /* binned scatter: count + scan + record write */
  NBVH_K_SCATTER_REDUCE = 8, /* binned scatter: per-chunk accumulation */
  NBVH_K_COUNT = 9
} nbvh_kernel_id;

typedef struct {
  double ms[NBVH_K_COUNT];     /* summed device time between the group's start and end events */
  int64_t calls[NBVH_K_COUNT]; /* launches of the group */
} nbvh_profile;

/* Start recording a HIP event pair around every kernel group launched
 * through this context (on the caller's stream) until nbvh_profile_end,
 * which synchronises on the events and returns the sums. At most 16384
 * groups are recorded per window; later ones are not timed. */
nbvh_status nbvh_profile_begin(nbvh_ctx* ctx);
nbvh_status nbvh_profile_end(nbvh_ctx* ctx, nbvh_profile* out);

/* Copy the device state block to the host (synchronises `stream`). */
nbvh_status nbvh_read_state(nbvh_ctx* ctx, nbvh_state_host* out, void* stream);

/* The state block's sticky NBVH_FLAG_* bits alone (synchronises `stream`):
 * whether a query overflowed its segment capacity or a training step saw a
 * non-finite gradient and was skipped. */
nbvh_status nbvh_device_status(nbvh_ctx* ctx, uint32_t* flags_host, void* stream);

/* Caller-owned buffers of a context, by role (nbvh_param_bytes). */
typedef enum {
  NBVH_BUF_PARAMS = 0,    /* FP32 master parameters: table and MLP weights */
  NBVH_BUF_PARAMS_LP = 1, /* BF16 shadow of the parameters */
  NBVH_BUF_ADAM_M = 2,    /* Adam first moments (FP32) */
  NBVH_BUF_ADAM_V = 3,    /* Adam second moments (FP32) */
  NBVH_BUF_GRAD = 4,      /* gradient accumulator (FP32, times the loss scale) */
  NBVH_BUF_STATE = 5,     /* device state block */
  NBVH_BUF_AUX = 6        /* transposed weights, E4M3 weights and scales */
} nbvh_buffer;

/* Bytes the caller allocates for buffer `which` (nbvh_buffer) of this
 * context's network (Sec. 3 hash grid and Sec. 6 MLP sizes, padded to the
 * layout of nbvh_param_layout); 0 for an unknown role or a NULL context. */
size_t nbvh_param_bytes(const nbvh_ctx* ctx, int which);

/* dL/dparams as the last back-propagation left it in grad_dev, divided by
 * the current loss scale (the training step's loss scaling undone on the
 * device), written to out_dev ([n_params] FP32, same layout; may be
 * grad_dev itself). clear != 0 also zeroes grad_dev. Asynchronous. */
nbvh_status nbvh_unscaled_grad(nbvh_ctx* ctx, float* out_dev, int clear, void* stream);

/* Clear the sticky flag bits. */
nbvh_status nbvh_clear_flags(nbvh_ctx* ctx, void* stream);

/* Message of the last error on this thread ("" if none). */
const char* nbvh_last_error(void);

/* Library version string. */
const char* nbvh_version(void);

void nbvh_destroy(nbvh_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* NBVH_H */
