// C ABI of the library (include/nbvh.h): argument checking, the N-BVH build
// on the host, parameter layout, workspace carve-up and kernel sequencing.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>
#include <vector>

#include "launch.h"

struct nbvh_ctx {
  nbvh_config cfg;
  nbvh::DevCfg dev;
  uint32_t n_leaves;
  nbvh::Node* nodes;
  nbvh_params p;
  bool bound;
  int n_cu;
  nbvh::Profiler* prof;
  nbvh_tuning tune;
  bool fp8_ready;  // FP8 weights and scales in aux match the current parameters
  int tree_depth;  // inner levels of the N-BVH (traversal stack entries)
  // a second stream of the context: the training step's weight-gradient GEMMs
  // run on it beside the table-gradient scatter (fork and join by events)
  hipStream_t side;
  hipEvent_t ev_fork, ev_join;
};

namespace nbvh {

static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

nbvh_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return NBVH_ERR_HIP;
  }
  return NBVH_OK;
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

__global__ void k_zero_f32(float* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

static uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Validates cfg and fills the device description (no context needed).
static nbvh_status make_devcfg(const nbvh_config* c, DevCfg* d) {
  if (!c) {
    set_error("cfg is NULL");
    return NBVH_ERR_INVALID_ARG;
  }
  const int L = c->n_levels, F = c->n_features, S = c->n_samples;
  if (L < 1 || L > NBVH_MAX_LEVELS) return set_error("n_levels %d not in [1, 32]", L), NBVH_ERR_INVALID_ARG;
  if (F != 2 && F != 4) return set_error("n_features %d not in {2, 4}", F), NBVH_ERR_INVALID_ARG;
  if (S < 1 || S > 16) return set_error("n_samples %d not in [1, 16]", S), NBVH_ERR_INVALID_ARG;
  if (c->log2_T < 1 || c->log2_T > 24) return set_error("log2_T %d not in [1, 24]", c->log2_T), NBVH_ERR_INVALID_ARG;
  const int n_in = S * L * F;
  if (n_in % 32 != 0) return set_error("n_in = %d is not a multiple of 32", n_in), NBVH_ERR_INVALID_ARG;
  if (n_in > 512) return set_error("n_in = %d exceeds 512", n_in), NBVH_ERR_UNSUPPORTED;
  const int W = c->mlp_width;
  if (W != 32 && W != 64 && W != 128 && W != 256) return set_error("mlp_width %d not in {32,64,128,256}", W), NBVH_ERR_INVALID_ARG;
  if (c->mlp_hidden < 1 || c->mlp_hidden > 8) return set_error("mlp_hidden %d not in [1, 8]", c->mlp_hidden), NBVH_ERR_INVALID_ARG;
  if (c->n_out < 5 || c->n_out > 16) return set_error("n_out %d not in [5, 16]", c->n_out), NBVH_ERR_INVALID_ARG;
  if (c->precision != NBVH_FP32 && c->precision != NBVH_BF16 && c->precision != NBVH_FP8)
    return set_error("precision %d unknown", c->precision), NBVH_ERR_INVALID_ARG;
  if (c->inside_rule != NBVH_INSIDE_CLIP && c->inside_rule != NBVH_INSIDE_REVERSE)
    return set_error("inside_rule %d unknown", c->inside_rule), NBVH_ERR_INVALID_ARG;
  if (!(c->scene_side > 0.0f) || !std::isfinite(c->scene_side))
    return set_error("scene_side must be positive and finite"), NBVH_ERR_INVALID_ARG;
  memset(d, 0, sizeof(*d));
  d->n_levels = L;
  d->n_features = F;
  d->log2_T = c->log2_T;
  d->n_samples = S;
  d->n_in = n_in;
  d->width = W;
  d->hidden = c->mlp_hidden;
  d->n_out = c->n_out;
  d->inside_reverse = c->inside_rule == NBVH_INSIDE_REVERSE;
  const uint64_t T = 1ull << c->log2_T;
  uint64_t off = 0;
  for (int l = 0; l < L; ++l) {
    const int N = c->level_res[l];
    if (N < 1 || N > (1 << 24)) return set_error("level_res[%d] = %d invalid", l, N), NBVH_ERR_INVALID_ARG;
    const uint64_t r1 = (uint64_t)N + 1;
    const bool dense = r1 * r1 * r1 <= T;
    d->level_res[l] = N;
    if (dense) d->dense_mask |= 1u << l;
    d->level_off[l] = (uint32_t)off;
    off += (dense ? r1 * r1 * r1 : T) * (uint64_t)F;
    if (off > 0xffffffffull) return set_error("hash table exceeds 2^32 parameters"), NBVH_ERR_UNSUPPORTED;
  }
  d->n_table = off;
  for (int a = 0; a < 3; ++a) d->scene_lo[a] = c->scene_lo[a];
  d->inv_side = 1.0f / c->scene_side;
  for (int s = 0; s < S; ++s) d->frac[s] = ((float)s + 0.5f) / (float)S;
  uint64_t p = round_up(off, kAlign), wt = 0, nm = 0;
  for (int k = 0; k <= d->hidden; ++k) {
    d->fan_in[k] = (k == 0) ? n_in : W;
    d->fan_out[k] = (k == d->hidden) ? c->n_out : W;
    d->w_off[k] = p;
    const uint64_t sz = (uint64_t)d->fan_in[k] * d->fan_out[k];
    nm += sz;
    p = round_up(p + sz, kAlign);
    d->wt_off[k] = wt;
    const int fo_pad = (k == d->hidden) ? 32 : d->fan_out[k];
    wt = round_up(wt + (uint64_t)d->fan_in[k] * fo_pad, kAlign);
  }
  d->n_mlp = nm;
  d->n_params = p;
  d->n_wt = wt;
  return NBVH_OK;
}

// ---------------------------------------------------------------------------
// N-BVH over the leaves: median split of leaf centroids on the widest axis
// (ties by leaf id); inner boxes are exact min/max unions.
struct Box {
  float lo[3], hi[3];
};

static Box unite(const Box& a, const Box& b) {
  Box r;
  for (int k = 0; k < 3; ++k) {
    r.lo[k] = std::min(a.lo[k], b.lo[k]);
    r.hi[k] = std::max(a.hi[k], b.hi[k]);
  }
  return r;
}

struct Builder {
  const Box* leaves;
  std::vector<Node> nodes;
  int max_depth = 0;

  // returns (child code, box) for the subset idx[b, e)
  int32_t build(std::vector<uint32_t>& idx, size_t b, size_t e, Box& box, int depth) {
    if (e - b == 1) {
      box = leaves[idx[b]];
      return ~(int32_t)idx[b];
    }
    max_depth = std::max(max_depth, depth + 1);
    float clo[3], chi[3];
    for (int k = 0; k < 3; ++k) {
      clo[k] = INFINITY;
      chi[k] = -INFINITY;
    }
    for (size_t i = b; i < e; ++i) {
      const Box& l = leaves[idx[i]];
      for (int k = 0; k < 3; ++k) {
        const float cc = 0.5f * (l.lo[k] + l.hi[k]);
        clo[k] = std::min(clo[k], cc);
        chi[k] = std::max(chi[k], cc);
      }
    }
    int axis = 0;
    for (int k = 1; k < 3; ++k)
      if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
    std::sort(idx.begin() + b, idx.begin() + e, [&](uint32_t x, uint32_t y) {
      const float cx = 0.5f * (leaves[x].lo[axis] + leaves[x].hi[axis]);
      const float cy = 0.5f * (leaves[y].lo[axis] + leaves[y].hi[axis]);
      return cx < cy || (cx == cy && x < y);
    });
    const size_t mid = b + (e - b) / 2;
    const int32_t me = (int32_t)nodes.size();
    nodes.emplace_back();
    Box b0, b1;
    const int32_t c0 = build(idx, b, mid, b0, depth + 1);
    const int32_t c1 = build(idx, mid, e, b1, depth + 1);
    Node& n = nodes[me];
    memset(&n, 0, sizeof(n));
    for (int k = 0; k < 3; ++k) {
      n.lo0[k] = b0.lo[k];
      n.hi0[k] = b0.hi[k];
      n.lo1[k] = b1.lo[k];
      n.hi1[k] = b1.hi[k];
    }
    n.c0 = c0;
    n.c1 = c1;
    box = unite(b0, b1);
    return me;
  }
};

static nbvh_status require_bound(const nbvh_ctx* ctx) {
  if (!ctx) return set_error("ctx is NULL"), NBVH_ERR_INVALID_ARG;
  if (!ctx->bound) return set_error("parameters not bound (nbvh_bind_params)"), NBVH_ERR_NOT_BOUND;
  return NBVH_OK;
}

static nbvh_status require_fp8_ready(const nbvh_ctx* ctx) {
  if (ctx->cfg.precision == NBVH_FP8 && !ctx->fp8_ready)
    return set_error("FP8 weights are stale or missing: call nbvh_calibrate_fp8 after setting parameters"),
           NBVH_ERR_NOT_BOUND;
  return NBVH_OK;
}

static LaunchCtx make_launch(const nbvh_ctx* ctx, void* stream) {
  LaunchCtx L;
  memset(&L, 0, sizeof(L));
  L.stream = (hipStream_t)stream;
  L.side = ctx->side;
  L.ev_fork = ctx->ev_fork;
  L.ev_join = ctx->ev_join;
  L.nodes = ctx->nodes;
  L.state = (DevState*)ctx->p.state_dev;
  L.cfg = ctx->dev;
  L.precision = ctx->cfg.precision == NBVH_FP8 ? NBVH_BF16 : ctx->cfg.precision;
  L.params = ctx->p.params_dev;
  L.params_lp = ctx->p.params_lp_dev;
  L.adam_m = ctx->p.adam_m_dev;
  L.adam_v = ctx->p.adam_v_dev;
  L.grad = ctx->p.grad_dev;
  L.aux = ctx->p.aux_dev;
  L.fp8 = ctx->cfg.precision == NBVH_FP8;
  L.stack_depth = ctx->tree_depth > 0 ? ctx->tree_depth : 1;
  L.n_cu = ctx->n_cu;
  L.w_hit = ctx->cfg.w_hit;
  L.w_t = ctx->cfg.w_t;
  L.w_normal = ctx->cfg.w_normal;
  L.w_albedo = ctx->cfg.w_albedo;
  L.lr = ctx->cfg.lr;
  L.beta1 = ctx->cfg.beta1;
  L.beta2 = ctx->cfg.beta2;
  L.eps = ctx->cfg.eps;
  L.loss_scale = ctx->cfg.loss_scale;
  L.prof = (ctx->prof && ctx->prof->on) ? ctx->prof : nullptr;
  L.tune = ctx->tune;
  return L;
}

// query workspace carve-up
struct QueryLayout {
  size_t offsets, counts, active, pos, sums, sums2, misc, staging, segs, order, total;
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// `ordered`: room for sorting the active rays by origin (tuning query_order)
static QueryLayout query_layout(uint64_t n_rays, uint64_t cap, bool ordered = false) {
  QueryLayout Q;
  size_t off = 0;
  Q.offsets = off;
  off = a256(off + (n_rays + 1) * 4);
  Q.counts = off;
  off = a256(off + n_rays * 4);
  Q.active = off;
  off = a256(off + n_rays * 4);
  Q.pos = off;
  off = a256(off + (n_rays + 1) * 4);
  Q.sums = off;
  off = a256(off + (n_rays / 1024 + 2) * 4);
  Q.sums2 = off;
  off = a256(off + (n_rays / 1024 + 2) * 4);
  Q.misc = off;
  off = a256(off + 16 * 4);
  Q.staging = off;
  off = a256(off + traverse_staging_bytes(n_rays));
  Q.segs = off;
  off = a256(off + cap * sizeof(nbvh_segment));
  Q.order = off;
  if (ordered) off = a256(off + ray_order_bytes(n_rays));
  Q.total = off;
  return Q;
}

// Device memory of nbvh_query_noalloc: one query's workspace (segment
// offsets and counts, active-ray list, scan partials, counters, traversal
// staging, segment queue), at most kNoAllocBytes. A file-scope array, so each
// GPU the library runs on holds its own copy until the process ends; its
// address on a device comes from hipGetSymbolAddress with that device
// current, and host code uses only that address.
constexpr size_t kNoAllocBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// The current device's address of `scratch`, looked up once per device.
static nbvh_status scratch_for_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return set_error("no usable current device for the no-allocation query"), NBVH_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e)),
             NBVH_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NBVH_OK;
}

}  // namespace nbvh

using namespace nbvh;

extern "C" {

const char* nbvh_last_error(void) { return g_err; }

const char* nbvh_version(void) { return "nbvh-gfx950 0.1"; }

nbvh_status nbvh_param_count(const nbvh_config* cfg, uint64_t* n_table, uint64_t* n_mlp) {
  DevCfg d;
  nbvh_status s = make_devcfg(cfg, &d);
  if (s != NBVH_OK) return s;
  if (n_table) *n_table = d.n_table;
  if (n_mlp) *n_mlp = d.n_mlp;
  return NBVH_OK;
}

nbvh_status nbvh_param_layout(const nbvh_config* cfg, uint64_t* offsets) {
  DevCfg d;
  nbvh_status s = make_devcfg(cfg, &d);
  if (s != NBVH_OK) return s;
  if (!offsets) return set_error("offsets is NULL"), NBVH_ERR_INVALID_ARG;
  offsets[0] = 0;
  for (int k = 0; k <= d.hidden; ++k) offsets[1 + k] = d.w_off[k];
  offsets[d.hidden + 2] = d.n_params;
  return NBVH_OK;
}

size_t nbvh_aux_bytes(const nbvh_config* cfg) {
  DevCfg d;
  if (make_devcfg(cfg, &d) != NBVH_OK) return 0;
  return (size_t)aux_total_bytes(d);
}

size_t nbvh_nodes_bytes(uint32_t n_leaves) { return (size_t)(n_leaves > 1 ? n_leaves - 1 : 1) * sizeof(Node); }

size_t nbvh_state_bytes(void) { return sizeof(DevState); }

nbvh_status nbvh_build(const nbvh_config* cfg, const float* leaf_boxes_host, uint32_t n_leaves, void* nodes_dev,
                       size_t nodes_bytes, void* stream, nbvh_ctx** out) {
  if (!out) return set_error("out is NULL"), NBVH_ERR_INVALID_ARG;
  *out = nullptr;
  DevCfg d;
  nbvh_status s = make_devcfg(cfg, &d);
  if (s != NBVH_OK) return s;
  if (!leaf_boxes_host || n_leaves == 0) return set_error("no leaves"), NBVH_ERR_INVALID_ARG;
  if (n_leaves > (1u << 30)) return set_error("too many leaves"), NBVH_ERR_UNSUPPORTED;
  if (!nodes_dev) return set_error("nodes_dev is NULL"), NBVH_ERR_INVALID_ARG;
  if (nodes_bytes < nbvh_nodes_bytes(n_leaves))
    return set_error("nodes buffer too small: need %zu", nbvh_nodes_bytes(n_leaves)), NBVH_ERR_CAPACITY;
  const Box* boxes = (const Box*)leaf_boxes_host;
  for (uint32_t i = 0; i < n_leaves; ++i)
    for (int k = 0; k < 3; ++k)
      if (!(boxes[i].lo[k] <= boxes[i].hi[k]) || !std::isfinite(boxes[i].lo[k]) || !std::isfinite(boxes[i].hi[k]))
        return set_error("leaf %u has an invalid box", i), NBVH_ERR_INVALID_ARG;
  Builder B;
  B.leaves = boxes;
  std::vector<Node> host;
  if (n_leaves == 1) {
    Node n;
    memset(&n, 0, sizeof(n));
    for (int k = 0; k < 3; ++k) {
      n.lo0[k] = boxes[0].lo[k];
      n.hi0[k] = boxes[0].hi[k];
    }
    n.c0 = ~0;
    n.c1 = kEmptyChild;
    host.push_back(n);
  } else {
    std::vector<uint32_t> idx(n_leaves);
    std::iota(idx.begin(), idx.end(), 0u);
    Box root;
    B.nodes.reserve(n_leaves);
    B.build(idx, 0, n_leaves, root, 0);
    if (B.max_depth >= kMaxDepth) return set_error("tree depth %d too large", B.max_depth), NBVH_ERR_UNSUPPORTED;
    host.swap(B.nodes);
  }
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(nodes_dev, host.data(), host.size() * sizeof(Node), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    set_error("copying nodes: %s", hipGetErrorString(hipGetLastError()));
    return NBVH_ERR_HIP;
  }
  nbvh_ctx* ctx = new nbvh_ctx;
  memset(ctx, 0, sizeof(*ctx));
  ctx->tree_depth = B.max_depth;
  ctx->cfg = *cfg;
  ctx->dev = d;
  ctx->n_leaves = n_leaves;
  ctx->nodes = (Node*)nodes_dev;
  int dev = 0;
  hipGetDevice(&dev);
  hipDeviceProp_t prop;
  ctx->n_cu = (hipGetDeviceProperties(&prop, dev) == hipSuccess) ? prop.multiProcessorCount : 256;
  if (ctx->n_cu <= 0) ctx->n_cu = 256;
  ctx->tune = nbvh_tuning{8, 0, 0, 8, 64, 0, 1, 8, 0, 0, 2, 0};
  if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess) {
    set_error("creating the context's stream and events failed");
    nbvh_destroy(ctx);
    return NBVH_ERR_HIP;
  }
  void* sp = nullptr;
  s = scratch_for_current_device(&sp);  // set-up of the no-allocation query on this device
  if (s != NBVH_OK) {
    nbvh_destroy(ctx);
    return s;
  }
  *out = ctx;
  return NBVH_OK;
}

nbvh_status nbvh_bind_params(nbvh_ctx* ctx, const nbvh_params* p) {
  if (!ctx || !p) return set_error("ctx or params NULL"), NBVH_ERR_INVALID_ARG;
  if (!p->params_dev || !p->adam_m_dev || !p->adam_v_dev || !p->grad_dev || !p->state_dev || !p->aux_dev)
    return set_error("a parameter buffer is NULL"), NBVH_ERR_INVALID_ARG;
  if (ctx->cfg.precision != NBVH_FP32 && !p->params_lp_dev)
    return set_error("params_lp_dev is required for BF16/FP8 precision"), NBVH_ERR_INVALID_ARG;
  if (((uintptr_t)p->params_dev | (uintptr_t)p->params_lp_dev | (uintptr_t)p->aux_dev | (uintptr_t)p->adam_m_dev |
       (uintptr_t)p->adam_v_dev | (uintptr_t)p->grad_dev) & 15)
    return set_error("parameter buffers must be 16-byte aligned"), NBVH_ERR_INVALID_ARG;
  ctx->p = *p;
  ctx->bound = true;
  ctx->fp8_ready = false;
  return NBVH_OK;
}

nbvh_status nbvh_reset_optimizer(nbvh_ctx* ctx, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  LaunchCtx L = make_launch(ctx, stream);
  const uint64_t n = ctx->dev.n_params;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 4096);
  k_zero_f32<<<grid, 256, 0, L.stream>>>(L.adam_m, n);
  k_zero_f32<<<grid, 256, 0, L.stream>>>(L.adam_v, n);
  k_zero_f32<<<grid, 256, 0, L.stream>>>(L.grad, n);
  k_zero_f32<<<grid, 256, 0, L.stream>>>((float*)L.aux, aux_total_bytes(ctx->dev) / 4);
  ctx->fp8_ready = false;
  return launch_optimizer(L, true, true);
}

nbvh_status nbvh_sync_shadow(nbvh_ctx* ctx, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  LaunchCtx L = make_launch(ctx, stream);
  ctx->fp8_ready = false;
  return launch_optimizer(L, false, true);
}

nbvh_status nbvh_calibrate_fp8(nbvh_ctx* ctx, const nbvh_probe* probes, uint64_t n, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  if (ctx->cfg.precision != NBVH_FP8) return set_error("context precision is not FP8"), NBVH_ERR_INVALID_ARG;
  if (n == 0 || !probes) return set_error("calibration needs at least one segment"), NBVH_ERR_INVALID_ARG;
  if (n > 0x7fffffffull) return set_error("batch too large"), NBVH_ERR_UNSUPPORTED;
  s = launch_calibrate_fp8(make_launch(ctx, stream), probes, (uint32_t)n);
  if (s == NBVH_OK) ctx->fp8_ready = true;
  return s;
}

size_t nbvh_workspace_bytes(const nbvh_ctx* ctx, uint64_t max_rays, uint64_t max_segments, uint64_t max_batch) {
  if (!ctx) return 0;
  size_t q = query_layout(max_rays, max_segments, ctx->tune.query_order != 0).total;
  const int prec = ctx->cfg.precision == NBVH_FP8 ? NBVH_BF16 : ctx->cfg.precision;
  size_t t = train_ws_bytes(ctx->dev, prec, max_batch, ctx->tune);
  size_t l = std::max(a256((max_batch / 256 + 2) * 16), group_ws_bytes(max_batch));
  return std::max(q, std::max(t, l));
}

nbvh_status nbvh_traverse(nbvh_ctx* ctx, const nbvh_ray* rays, uint64_t n_rays, uint32_t* seg_offsets,
                          nbvh_segment* segs, uint64_t seg_capacity, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return set_error("ctx is NULL"), NBVH_ERR_INVALID_ARG;
  if (!ctx->p.state_dev) return set_error("state buffer not bound"), NBVH_ERR_NOT_BOUND;
  if (n_rays > 0xfffffff0ull) return set_error("too many rays"), NBVH_ERR_UNSUPPORTED;
  if ((n_rays && !rays) || !seg_offsets || (seg_capacity && !segs) || !ws)
    return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  const QueryLayout Q = query_layout(n_rays, 0);
  if (ws_bytes < Q.segs) return set_error("workspace too small: need %zu", Q.segs), NBVH_ERR_CAPACITY;
  LaunchCtx L = make_launch(ctx, stream);
  char* w = (char*)ws;
  uint32_t* misc = (uint32_t*)(w + Q.misc);
  return launch_traverse(L, rays, (uint32_t)n_rays, seg_offsets, segs, seg_capacity, nullptr, nullptr, nullptr,
                         (uint32_t*)(w + Q.counts), (uint32_t*)(w + Q.sums), misc + 12, (float*)(w + Q.staging));
}

nbvh_status nbvh_query(nbvh_ctx* ctx, const nbvh_ray* rays, uint64_t n_rays, nbvh_hit* hits, uint64_t seg_capacity,
                       void* ws, size_t ws_bytes, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  s = require_fp8_ready(ctx);
  if (s != NBVH_OK) return s;
  if (n_rays > 0xfffffff0ull) return set_error("too many rays"), NBVH_ERR_UNSUPPORTED;
  if ((n_rays && (!rays || !hits)) || !ws) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (seg_capacity > 0xffffffffull) seg_capacity = 0xffffffffull;
  const bool ordered = ctx->tune.query_order != 0;
  const QueryLayout Q = query_layout(n_rays, seg_capacity, ordered);
  if (ws_bytes < Q.total) return set_error("workspace too small: need %zu, got %zu", Q.total, ws_bytes), NBVH_ERR_CAPACITY;
  if (n_rays == 0) return NBVH_OK;
  LaunchCtx L = make_launch(ctx, stream);
  char* w = (char*)ws;
  uint32_t* offsets = (uint32_t*)(w + Q.offsets);
  uint32_t* misc = (uint32_t*)(w + Q.misc);
  nbvh_segment* segs = (nbvh_segment*)(w + Q.segs);
  s = launch_traverse(L, rays, (uint32_t)n_rays, offsets, segs, seg_capacity, hits, (uint32_t*)(w + Q.active), misc + 0,
                      (uint32_t*)(w + Q.counts), (uint32_t*)(w + Q.sums), misc + 12, (float*)(w + Q.staging),
                      nullptr, ordered ? w + Q.order : nullptr, (uint32_t*)(w + Q.pos), (uint32_t*)(w + Q.sums2));
  if (s != NBVH_OK) return s;
  return launch_query_eval(L, rays, offsets, segs, (const uint32_t*)(w + Q.active), misc + 0, misc + 1, hits,
                           (uint32_t)n_rays, seg_capacity);
}

nbvh_status nbvh_query_noalloc(nbvh_ctx* ctx, const nbvh_ray* rays, uint64_t n_rays, nbvh_hit* hits,
                               uint64_t seg_capacity, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  if (n_rays > 0xfffffff0ull) return set_error("too many rays"), NBVH_ERR_UNSUPPORTED;
  if (seg_capacity > 0xffffffffull) seg_capacity = 0xffffffffull;
  const size_t need = query_layout(n_rays, seg_capacity, ctx->tune.query_order != 0).total;
  if (need > kNoAllocBytes)
    return set_error("query of %llu rays with %llu segments needs %zu bytes of scratch; the no-allocation query "
                     "holds %zu",
                     (unsigned long long)n_rays, (unsigned long long)seg_capacity, need, kNoAllocBytes),
           NBVH_ERR_CAPACITY;
  void* ws = nullptr;
  s = scratch_for_current_device(&ws);
  if (s != NBVH_OK) return s;
  return nbvh_query(ctx, rays, n_rays, hits, seg_capacity, ws, kNoAllocBytes, stream);
}

nbvh_status nbvh_query_traced(nbvh_ctx* ctx, const nbvh_ray* rays, uint64_t n_rays, nbvh_hit* hits,
                              uint64_t seg_capacity, void* ws, size_t ws_bytes, const nbvh_query_trace* trace,
                              void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  s = require_fp8_ready(ctx);
  if (s != NBVH_OK) return s;
  if (!trace) return set_error("trace is NULL"), NBVH_ERR_INVALID_ARG;
  if (trace->u_dev && ctx->cfg.precision == NBVH_FP8)
    return set_error("FP8 queries keep scaled E4M3 features: no feature trace"), NBVH_ERR_UNSUPPORTED;
  if (n_rays > 0xfffffff0ull) return set_error("too many rays"), NBVH_ERR_UNSUPPORTED;
  if ((n_rays && (!rays || !hits)) || !ws) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (seg_capacity > 0xffffffffull) seg_capacity = 0xffffffffull;
  const bool ordered = ctx->tune.query_order != 0;
  const QueryLayout Q = query_layout(n_rays, seg_capacity, ordered);
  if (ws_bytes < Q.total) return set_error("workspace too small: need %zu, got %zu", Q.total, ws_bytes), NBVH_ERR_CAPACITY;
  if (n_rays == 0) return NBVH_OK;
  LaunchCtx L = make_launch(ctx, stream);
  char* w = (char*)ws;
  uint32_t* offsets = (uint32_t*)(w + Q.offsets);
  uint32_t* misc = (uint32_t*)(w + Q.misc);
  nbvh_segment* segs = (nbvh_segment*)(w + Q.segs);
  s = launch_traverse(L, rays, (uint32_t)n_rays, offsets, segs, seg_capacity, hits, (uint32_t*)(w + Q.active), misc + 0,
                      (uint32_t*)(w + Q.counts), (uint32_t*)(w + Q.sums), misc + 12, (float*)(w + Q.staging),
                      nullptr, ordered ? w + Q.order : nullptr, (uint32_t*)(w + Q.pos), (uint32_t*)(w + Q.sums2));
  if (s != NBVH_OK) return s;
  if (trace->seg_offsets_dev &&
      hipMemcpyAsync(trace->seg_offsets_dev, offsets, (n_rays + 1) * 4, hipMemcpyDeviceToDevice, L.stream) != hipSuccess)
    return set_error("copy of the segment offsets failed"), NBVH_ERR_HIP;
  if (trace->segs_dev && seg_capacity &&
      hipMemcpyAsync(trace->segs_dev, segs, seg_capacity * sizeof(nbvh_segment), hipMemcpyDeviceToDevice, L.stream) !=
          hipSuccess)
    return set_error("copy of the segment queue failed"), NBVH_ERR_HIP;
  return launch_query_eval(L, rays, offsets, segs, (const uint32_t*)(w + Q.active), misc + 0, misc + 1, hits,
                           (uint32_t)n_rays, seg_capacity, trace->z_dev, trace->u_dev);
}

nbvh_status nbvh_query_segments(nbvh_ctx* ctx, const nbvh_ray* rays, uint64_t n_rays, const uint32_t* seg_offsets,
                                const nbvh_segment* segs, nbvh_hit* hits, void* ws, size_t ws_bytes, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  s = require_fp8_ready(ctx);
  if (s != NBVH_OK) return s;
  if (n_rays > 0xfffffff0ull) return set_error("too many rays"), NBVH_ERR_UNSUPPORTED;
  if ((n_rays && (!rays || !hits || !seg_offsets || !segs)) || !ws) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  const QueryLayout Q = query_layout(n_rays, 0);
  if (ws_bytes < Q.segs) return set_error("workspace too small: need %zu", Q.segs), NBVH_ERR_CAPACITY;
  if (n_rays == 0) return NBVH_OK;
  LaunchCtx L = make_launch(ctx, stream);
  char* w = (char*)ws;
  uint32_t* misc = (uint32_t*)(w + Q.misc);
  uint32_t* active = (uint32_t*)(w + Q.active);
  s = launch_active_rays(L, seg_offsets, (uint32_t)n_rays, hits, active, misc);
  if (s != NBVH_OK) return s;
  return launch_query_eval(L, rays, seg_offsets, segs, active, misc + 0, misc + 1, hits, (uint32_t)n_rays,
                           0xffffffffull);
}

nbvh_status nbvh_first_hits(nbvh_ctx* ctx, const nbvh_ray* rays, uint64_t n_rays, const float* u, const float* accept,
                            nbvh_probe* probes, uint32_t* leaf_ids, uint32_t* n_out, uint32_t* leaf_hits,
                            void* stream) {
  if (!ctx) return set_error("ctx is NULL"), NBVH_ERR_INVALID_ARG;
  if (n_rays > 0xfffffff0ull) return set_error("too many rays"), NBVH_ERR_UNSUPPORTED;
  if (!n_out || (n_rays && (!rays || !u || !accept || !probes || !leaf_ids)))
    return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  return launch_first_hits(make_launch(ctx, stream), rays, (uint32_t)n_rays, u, accept, probes, leaf_ids, n_out,
                           leaf_hits);
}

size_t nbvh_group_ws_bytes(uint64_t n) { return group_ws_bytes(n); }

nbvh_status nbvh_group_by_leaf(nbvh_ctx* ctx, const nbvh_probe* probes_in, const uint32_t* leaf_ids_in, uint64_t n,
                               nbvh_probe* probes_out, uint32_t* leaf_ids_out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return set_error("ctx is NULL"), NBVH_ERR_INVALID_ARG;
  if (n > 0xfffffff0ull) return set_error("too many probes"), NBVH_ERR_UNSUPPORTED;
  if (n == 0) return NBVH_OK;
  if (!probes_in || !leaf_ids_in || !probes_out || !ws) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (probes_out == probes_in) return set_error("probes_out must not alias probes_in"), NBVH_ERR_INVALID_ARG;
  const size_t need = group_ws_bytes(n);
  if (ws_bytes < need) return set_error("workspace too small: need %zu, got %zu", need, ws_bytes), NBVH_ERR_CAPACITY;
  return launch_group_by_leaf(make_launch(ctx, stream), ctx->n_leaves, probes_in, leaf_ids_in, (uint32_t)n,
                              probes_out, leaf_ids_out, ws);
}

nbvh_status nbvh_leaf_loss(nbvh_ctx* ctx, const nbvh_probe* probes, const nbvh_label* labels, const uint32_t* leaf_ids,
                           uint64_t n, float* leaf_loss, uint32_t* leaf_count, void* ws, size_t ws_bytes,
                           void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  s = require_fp8_ready(ctx);
  if (s != NBVH_OK) return s;
  if (n > 0x7fffffffull) return set_error("batch too large"), NBVH_ERR_UNSUPPORTED;
  if (n && (!probes || !labels || !leaf_ids || !leaf_loss || !leaf_count || !ws))
    return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  const size_t need = (size_t)n * ctx->cfg.n_out * sizeof(float);
  if (ws_bytes < need) return set_error("workspace too small: need %zu", need), NBVH_ERR_CAPACITY;
  return launch_leaf_loss(make_launch(ctx, stream), probes, labels, leaf_ids, (uint32_t)n, (float*)ws, leaf_loss,
                          leaf_count);
}

nbvh_status nbvh_node_rank(const float* leaf_loss, const uint32_t* leaf_count, const uint32_t* leaf_hits,
                           uint32_t n_leaves, uint64_t n_rays, float* rank, void* stream) {
  if (n_leaves && (!leaf_loss || !leaf_count || !leaf_hits || !rank)) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  return launch_node_rank((hipStream_t)stream, leaf_loss, leaf_count, leaf_hits, n_leaves, n_rays, rank);
}

nbvh_status nbvh_acceptance(const float* rank, uint32_t n_leaves, float min_accept, float* accept, void* stream) {
  if (n_leaves && (!rank || !accept)) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (!(min_accept >= 0.0f && min_accept <= 1.0f)) return set_error("min_accept outside [0, 1]"), NBVH_ERR_INVALID_ARG;
  return launch_acceptance((hipStream_t)stream, rank, n_leaves, min_accept, accept);
}

nbvh_status nbvh_encode(nbvh_ctx* ctx, const nbvh_probe* probes, uint64_t n, float* u, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  if (n && (!probes || !u)) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (n > 0x7fffffffull) return set_error("batch too large"), NBVH_ERR_UNSUPPORTED;
  return launch_encode(make_launch(ctx, stream), probes, (uint32_t)n, u);
}

nbvh_status nbvh_forward(nbvh_ctx* ctx, const nbvh_probe* probes, uint64_t n, float* z, void* ws, size_t ws_bytes,
                         void* stream) {
  (void)ws;
  (void)ws_bytes;
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  s = require_fp8_ready(ctx);
  if (s != NBVH_OK) return s;
  if (n && (!probes || !z)) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (n > 0x7fffffffull) return set_error("batch too large"), NBVH_ERR_UNSUPPORTED;
  return launch_forward(make_launch(ctx, stream), probes, (uint32_t)n, z);
}

nbvh_status nbvh_backward(nbvh_ctx* ctx, const nbvh_probe* probes, uint64_t n, const float* dz, void* ws,
                          size_t ws_bytes, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  if (ctx->cfg.precision == NBVH_FP8) return set_error("FP8 is an inference precision"), NBVH_ERR_UNSUPPORTED;
  if (n && (!probes || !dz || !ws)) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (n > 0x7fffffffull) return set_error("batch too large"), NBVH_ERR_UNSUPPORTED;
  return launch_train_fwd_bwd(make_launch(ctx, stream), probes, nullptr, dz, (uint32_t)n, nullptr, ws, ws_bytes, false);
}

nbvh_status nbvh_optimizer_step(nbvh_ctx* ctx, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  ctx->fp8_ready = false;
  return launch_optimizer(make_launch(ctx, stream), false, false);
}

nbvh_status nbvh_train_step(nbvh_ctx* ctx, const nbvh_probe* probes, const nbvh_label* labels, uint64_t n,
                            float* loss_dev, void* ws, size_t ws_bytes, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  if (ctx->cfg.precision == NBVH_FP8) return set_error("FP8 is an inference precision"), NBVH_ERR_UNSUPPORTED;
  if (n == 0) return set_error("empty batch"), NBVH_ERR_INVALID_ARG;
  if (!probes || !labels || !ws) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (n > 0x7fffffffull) return set_error("batch too large"), NBVH_ERR_UNSUPPORTED;
  LaunchCtx L = make_launch(ctx, stream);
  s = launch_train_fwd_bwd(L, probes, labels, nullptr, (uint32_t)n, loss_dev, ws, ws_bytes, true);
  if (s != NBVH_OK) return s;
  return launch_optimizer(L, false, false);
}

nbvh_status nbvh_loss(nbvh_ctx* ctx, const float* z, const nbvh_label* labels, uint64_t n, float* loss_dev,
                      float* dz, void* ws, size_t ws_bytes, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  if (n == 0) return set_error("empty batch"), NBVH_ERR_INVALID_ARG;
  if (!z || !labels || !ws) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (n > 0x7fffffffull) return set_error("batch too large"), NBVH_ERR_UNSUPPORTED;
  return launch_loss(make_launch(ctx, stream), z, labels, (uint32_t)n, loss_dev, dz, ws, ws_bytes);
}

nbvh_status nbvh_read_state(nbvh_ctx* ctx, nbvh_state_host* out, void* stream) {
  if (!ctx || !out) return set_error("NULL argument"), NBVH_ERR_INVALID_ARG;
  if (!ctx->p.state_dev) return set_error("state buffer not bound"), NBVH_ERR_NOT_BOUND;
  DevState st;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(&st, ctx->p.state_dev, sizeof(st), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("reading state: %s", hipGetErrorString(hipGetLastError()));
    return NBVH_ERR_HIP;
  }
  out->step = st.step;
  out->skipped = st.skipped;
  out->loss_scale = st.loss_scale;
  out->flags = st.flags;
  for (int i = 0; i < 4; ++i) out->last_loss[i] = st.last_loss[i];
  out->last_n_segments = st.last_n_segments;
  out->n_evaluated = st.n_evaluated;
  return NBVH_OK;
}

nbvh_status nbvh_device_status(nbvh_ctx* ctx, uint32_t* flags_host, void* stream) {
  if (!flags_host) return set_error("flags_host is NULL"), NBVH_ERR_INVALID_ARG;
  nbvh_state_host st;
  nbvh_status s = nbvh_read_state(ctx, &st, stream);
  if (s != NBVH_OK) return s;
  *flags_host = st.flags;
  return NBVH_OK;
}

size_t nbvh_param_bytes(const nbvh_ctx* ctx, int which) {
  if (!ctx) return 0;
  const uint64_t n = ctx->dev.n_params;
  switch (which) {
    case NBVH_BUF_PARAMS:
    case NBVH_BUF_ADAM_M:
    case NBVH_BUF_ADAM_V:
    case NBVH_BUF_GRAD:
      return (size_t)n * 4;
    case NBVH_BUF_PARAMS_LP:
      return (size_t)n * 2;
    case NBVH_BUF_STATE:
      return sizeof(DevState);
    case NBVH_BUF_AUX:
      return (size_t)aux_total_bytes(ctx->dev);
    default:
      return 0;
  }
}

nbvh_status nbvh_unscaled_grad(nbvh_ctx* ctx, float* out_dev, int clear, void* stream) {
  nbvh_status s = require_bound(ctx);
  if (s != NBVH_OK) return s;
  if (!out_dev) return set_error("out_dev is NULL"), NBVH_ERR_INVALID_ARG;
  return launch_unscale_grad(make_launch(ctx, stream), out_dev, clear != 0);
}

__global__ void k_clear_flags(DevState* s) {
  if (threadIdx.x == 0) s->flags = 0u;
}

nbvh_status nbvh_clear_flags(nbvh_ctx* ctx, void* stream) {
  if (!ctx || !ctx->p.state_dev) return set_error("state buffer not bound"), NBVH_ERR_NOT_BOUND;
  k_clear_flags<<<1, 64, 0, (hipStream_t)stream>>>((DevState*)ctx->p.state_dev);
  return check_launch("clear_flags");
}

// ---------------------------------------------------------------------------
// batches of objects
}  // extern "C"

struct nbvh_batch {
  std::vector<nbvh_ctx*> ctxs;
  DevCfg* cfgs_dev;
};

static bool same_shape(const nbvh_config& a, const nbvh_config& b) {
  if (a.n_levels != b.n_levels || a.n_features != b.n_features || a.n_samples != b.n_samples ||
      a.mlp_width != b.mlp_width || a.mlp_hidden != b.mlp_hidden || a.n_out != b.n_out || a.precision != b.precision ||
      a.inside_rule != b.inside_rule)
    return false;
  for (int l = 0; l < a.n_levels; ++l)
    if (a.level_res[l] != b.level_res[l]) return false;
  return true;
}

extern "C" {

nbvh_status nbvh_get_tuning(const nbvh_ctx* ctx, nbvh_tuning* out) {
  if (!ctx || !out) return set_error("NULL argument"), NBVH_ERR_INVALID_ARG;
  *out = ctx->tune;
  return NBVH_OK;
}

nbvh_status nbvh_set_tuning(nbvh_ctx* ctx, const nbvh_tuning* t) {
  if (!ctx || !t) return set_error("NULL argument"), NBVH_ERR_INVALID_ARG;
  if (t->query_waves != 4 && t->query_waves != 8) return set_error("query_waves must be 4 or 8"), NBVH_ERR_INVALID_ARG;
  if (t->query_unroll != 0 && (t->query_unroll < 2 || t->query_unroll > 4))
    return set_error("query_unroll must be 0 (default), 2, 3 or 4"), NBVH_ERR_INVALID_ARG;
  if (t->query_wgs_per_cu < 0 || t->query_wgs_per_cu > 4) return set_error("query_wgs_per_cu in 0..4"), NBVH_ERR_INVALID_ARG;
  if (t->train_waves != 4 && t->train_waves != 8) return set_error("train_waves must be 4 or 8"), NBVH_ERR_INVALID_ARG;
  if (t->wgrad_splits < 1 || t->wgrad_splits > 256) return set_error("wgrad_splits in 1..256"), NBVH_ERR_INVALID_ARG;
  if (t->scatter_lds_kb < 0 || t->scatter_lds_kb > 144) return set_error("scatter_lds_kb in 0..144"), NBVH_ERR_INVALID_ARG;
  if (t->scatter_binned != 0 && t->scatter_binned != 1) return set_error("scatter_binned must be 0 or 1"), NBVH_ERR_INVALID_ARG;
  if (t->scatter_hash_levels < 0 || t->scatter_hash_levels > NBVH_MAX_LEVELS)
    return set_error("scatter_hash_levels in 0..32"), NBVH_ERR_INVALID_ARG;
  if (t->query_pairs != 0 && t->query_pairs != 1) return set_error("query_pairs must be 0 or 1"), NBVH_ERR_INVALID_ARG;
  if (t->query_lds_kb < 0 || t->query_lds_kb > 64) return set_error("query_lds_kb in 0..64"), NBVH_ERR_INVALID_ARG;
  if (t->traverse_mode < 0 || t->traverse_mode > 2) return set_error("traverse_mode must be 0, 1 or 2"), NBVH_ERR_INVALID_ARG;
  if (t->query_order < 0 || t->query_order > 2) return set_error("query_order must be 0, 1 or 2"), NBVH_ERR_INVALID_ARG;
  ctx->tune = *t;
  return NBVH_OK;
}

size_t nbvh_batch_desc_bytes(uint32_t n_objects) { return (size_t)n_objects * sizeof(DevCfg); }

nbvh_status nbvh_batch_create(nbvh_ctx* const* ctxs, uint32_t n_objects, void* descs_dev, size_t descs_bytes,
                              void* stream, nbvh_batch** out) {
  if (!out) return set_error("out is NULL"), NBVH_ERR_INVALID_ARG;
  *out = nullptr;
  if (!ctxs || n_objects < 1 || n_objects > 16) return set_error("batch needs 1..16 objects"), NBVH_ERR_INVALID_ARG;
  if (!descs_dev || descs_bytes < nbvh_batch_desc_bytes(n_objects))
    return set_error("descriptor buffer too small"), NBVH_ERR_CAPACITY;
  std::vector<DevCfg> h(n_objects);
  for (uint32_t k = 0; k < n_objects; ++k) {
    nbvh_status s = require_bound(ctxs[k]);
    if (s != NBVH_OK) return s;
    if (!same_shape(ctxs[0]->cfg, ctxs[k]->cfg)) return set_error("object %u has a different network shape", k), NBVH_ERR_INVALID_ARG;
    if (ctxs[k]->n_leaves >= (1u << 24)) return set_error("object %u has too many leaves", k), NBVH_ERR_UNSUPPORTED;
    h[k] = ctxs[k]->dev;
  }
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(descs_dev, h.data(), h.size() * sizeof(DevCfg), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return set_error("uploading batch descriptors failed"), NBVH_ERR_HIP;
  nbvh_batch* b = new nbvh_batch;
  b->ctxs.assign(ctxs, ctxs + n_objects);
  b->cfgs_dev = (DevCfg*)descs_dev;
  *out = b;
  return NBVH_OK;
}

// workspace: one query part per object, then the per-object hit records
// [object][ray] that the merge reads
// the objects' rays are ordered as the first object's knobs ask
static bool batch_ordered(const nbvh_batch* b) { return b->ctxs[0]->tune.query_order != 0; }

static size_t batch_part_bytes(uint64_t n_rays, uint64_t cap) { return query_layout(n_rays, cap).total; }

// per object: a query workspace and hit records; then, with a ray order, one
// ray permutation that every object's traversal follows
static size_t batch_ws_bytes(const nbvh_batch* b, uint64_t n_rays, uint64_t cap) {
  return b->ctxs.size() * (batch_part_bytes(n_rays, cap) + a256(n_rays * sizeof(nbvh_hit))) +
         (batch_ordered(b) ? a256(ray_order_bytes(n_rays)) : 0);
}

size_t nbvh_batch_workspace_bytes(const nbvh_batch* b, uint64_t max_rays, uint64_t seg_capacity) {
  if (!b) return 0;
  return batch_ws_bytes(b, max_rays, seg_capacity);
}

nbvh_status nbvh_batch_query(nbvh_batch* b, const nbvh_ray* rays, uint64_t n_rays, nbvh_hit* hits, uint64_t seg_capacity,
                             void* ws, size_t ws_bytes, void* stream) {
  if (!b) return set_error("batch is NULL"), NBVH_ERR_INVALID_ARG;
  if (n_rays > 0xfffffff0ull) return set_error("too many rays"), NBVH_ERR_UNSUPPORTED;
  if ((n_rays && (!rays || !hits)) || !ws) return set_error("NULL buffer"), NBVH_ERR_INVALID_ARG;
  if (seg_capacity > 0xffffffffull) seg_capacity = 0xffffffffull;
  const int n = (int)b->ctxs.size();
  const size_t part = batch_part_bytes(n_rays, seg_capacity);
  const size_t need = batch_ws_bytes(b, n_rays, seg_capacity);
  if (ws_bytes < need) return set_error("workspace too small: need %zu, got %zu", need, ws_bytes), NBVH_ERR_CAPACITY;
  if (n_rays == 0) return NBVH_OK;
  std::vector<LaunchCtx> Ls(n);
  std::vector<const uint32_t*> offs(n), act(n), nact(n);
  std::vector<const nbvh_segment*> sg(n);
  std::vector<uint32_t*> cnt(n);
  const bool ordered = batch_ordered(b);
  const QueryLayout Q = query_layout(n_rays, seg_capacity);
  nbvh_hit* per_obj = (nbvh_hit*)((char*)ws + n * part);
  RayOrder ord{nullptr, nullptr};
  if (ordered) {
    char* ow = (char*)ws + n * (part + a256(n_rays * sizeof(nbvh_hit)));
    nbvh_status s = launch_ray_order(make_launch(b->ctxs[0], stream), rays, (uint32_t)n_rays,
                                     b->ctxs[0]->tune.query_order, ow, &ord);
    if (s != NBVH_OK) return s;
  }
  for (int k = 0; k < n; ++k) {
    nbvh_status s = require_fp8_ready(b->ctxs[k]);
    if (s != NBVH_OK) return s;
  }
  for (int k = 0; k < n; ++k) {
    Ls[k] = make_launch(b->ctxs[k], stream);
    char* w = (char*)ws + part * k;
    uint32_t* offsets = (uint32_t*)(w + Q.offsets);
    uint32_t* misc = (uint32_t*)(w + Q.misc);
    nbvh_segment* segs = (nbvh_segment*)(w + Q.segs);
    nbvh_status s = launch_traverse(Ls[k], rays, (uint32_t)n_rays, offsets, segs, seg_capacity,
                                    per_obj + (size_t)k * n_rays, (uint32_t*)(w + Q.active), misc + 0,
                                    (uint32_t*)(w + Q.counts), (uint32_t*)(w + Q.sums), misc + 12,
                                    (float*)(w + Q.staging), ordered ? &ord : nullptr, nullptr,
                                    (uint32_t*)(w + Q.pos), (uint32_t*)(w + Q.sums2));
    if (s != NBVH_OK) return s;
    offs[k] = offsets;
    sg[k] = segs;
    act[k] = (const uint32_t*)(w + Q.active);
    nact[k] = misc + 0;
    cnt[k] = misc + 1;
  }
  return launch_query_eval_batch(Ls.data(), n, b->cfgs_dev, offs.data(), sg.data(), act.data(), nact.data(),
                                 cnt.data(), per_obj, hits, rays, (uint32_t)n_rays, seg_capacity);
}

void nbvh_batch_destroy(nbvh_batch* b) { delete b; }

nbvh_status nbvh_profile_begin(nbvh_ctx* ctx) {
  if (!ctx) return set_error("ctx is NULL"), NBVH_ERR_INVALID_ARG;
  if (!ctx->prof) {
    ctx->prof = new Profiler;
    ctx->prof->ev.resize(2 * Profiler::kMax);
    ctx->prof->kid.resize(Profiler::kMax);
    for (auto& e : ctx->prof->ev)
      if (hipEventCreate(&e) != hipSuccess) return set_error("hipEventCreate failed"), NBVH_ERR_HIP;
  }
  ctx->prof->used = 0;
  ctx->prof->on = true;
  return NBVH_OK;
}

nbvh_status nbvh_profile_end(nbvh_ctx* ctx, nbvh_profile* out) {
  if (!ctx || !out) return set_error("NULL argument"), NBVH_ERR_INVALID_ARG;
  memset(out, 0, sizeof(*out));
  if (!ctx->prof || !ctx->prof->on) return set_error("no profiling window open"), NBVH_ERR_INVALID_ARG;
  Profiler* p = ctx->prof;
  p->on = false;
  for (size_t i = 0; i < p->used; ++i) {
    if (hipEventSynchronize(p->ev[2 * i + 1]) != hipSuccess) return set_error("hipEventSynchronize failed"), NBVH_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) != hipSuccess)
      return set_error("hipEventElapsedTime failed"), NBVH_ERR_HIP;
    const int k = p->kid[i];
    if (k >= 0 && k < NBVH_K_COUNT) {
      out->ms[k] += ms;
      out->calls[k] += 1;
    }
  }
  p->used = 0;
  return NBVH_OK;
}

void nbvh_destroy(nbvh_ctx* ctx) {
  if (!ctx) return;
  if (ctx->prof) {
    for (auto& e : ctx->prof->ev) hipEventDestroy(e);
    delete ctx->prof;
  }
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  delete ctx;
}

}  // extern "C"
