// Host-side launch plumbing shared by the kernel translation units.
#pragma once
#include <vector>

#include "nbvh_internal.h"

namespace nbvh {

// HIP event pairs around kernel groups, recorded on the launch stream while a
// profiling window is open (nbvh_profile_begin / nbvh_profile_end).
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> ev;  // 2 per record
  std::vector<int> kid;
  size_t used = 0;
  static constexpr size_t kMax = 16384;
};

class ProfScope {
 public:
  ProfScope(Profiler* p, int kid, hipStream_t s) : p_(p), idx_((size_t)-1), s_(s) {
    if (p_ && p_->on && p_->used < p_->kid.size()) {
      idx_ = p_->used++;
      p_->kid[idx_] = kid;
      (void)hipEventRecord(p_->ev[2 * idx_], s_);
    }
  }
  ~ProfScope() {
    if (idx_ != (size_t)-1) (void)hipEventRecord(p_->ev[2 * idx_ + 1], s_);
  }

 private:
  Profiler* p_;
  size_t idx_;
  hipStream_t s_;
};

// Device state block (nbvh_state_bytes() bytes, caller-owned).
struct DevState {
  int64_t step;
  int64_t skipped;
  float loss_scale;
  uint32_t flags;
  float last_loss[4];
  uint64_t last_n_segments;
  uint32_t nonfinite_pending;  // set by producers of this step's gradient
  uint32_t pad0;
  unsigned long long n_evaluated;  // segments evaluated by queries
  uint32_t pad[4];
};

struct LaunchCtx {
  hipStream_t stream;
  hipStream_t side;                // the context's second stream (nullable)
  hipEvent_t ev_fork, ev_join;     // fork to and join from `side`
  const Node* nodes;
  DevState* state;
  DevCfg cfg;
  int precision;
  float* params;
  void* params_lp;
  float* adam_m;
  float* adam_v;
  float* grad;
  void* aux;  // transposed weight copies: fp32 [n_wt] then bf16 [n_wt]; FP8 block
  bool fp8;   // queries and forward run the MLP in FP8 (weights and scales in aux)
  int stack_depth;  // inner levels of the N-BVH: entries of a traversal stack
  int n_cu;
  // training hyper-parameters
  float w_hit, w_t, w_normal, w_albedo;
  float lr, beta1, beta2, eps, loss_scale;
  Profiler* prof;
  nbvh_tuning tune;
};

nbvh_status check_launch(const char* what);
void set_error(const char* fmt, ...);

__global__ void k_zero_u32(uint32_t* p, uint32_t n);
__global__ void k_zero_f32(float* p, uint64_t n);

// A permutation of the rays (launch_ray_order): the traversal's counting pass
// takes them in perm order; inv[r] is ray r's position in perm.
struct RayOrder {
  const uint32_t* perm;
  const uint32_t* inv;
};
size_t ray_order_bytes(uint64_t n);
// order: tuning query_order (0 leaves both pointers null); ws: ray_order_bytes(n)
nbvh_status launch_ray_order(const LaunchCtx& L, const nbvh_ray* rays, uint32_t n, int order, void* ws,
                             RayOrder* out);

// `staging` (traverse_staging_bytes(n_rays), required with `segs`): sorted
// per-ray runs kept by the counting pass so that the compaction copies them
// instead of walking again. `order` (nullable): a permutation the counting
// pass follows. `active_order_ws` (nullable, ray_order_bytes(n_rays)): with
// an active list and tuning query_order, sort the list by key once it is
// built instead. With `active` (the list of rays with a segment,
// in ray order; its length goes to *n_active), `segs`, scratch_pos
// (n_rays + 1 words) and scratch_sums2 (like scratch_sums) are required.
size_t traverse_staging_bytes(uint64_t n_rays);
nbvh_status launch_traverse(const LaunchCtx& L, const nbvh_ray* rays, uint32_t n_rays, uint32_t* offsets,
                            nbvh_segment* segs, uint64_t capacity, nbvh_hit* hits, uint32_t* active,
                            uint32_t* n_active, uint32_t* scratch_counts, uint32_t* scratch_sums,
                            uint32_t* scratch_total, float* staging, const RayOrder* order = nullptr,
                            void* active_order_ws = nullptr, uint32_t* scratch_pos = nullptr,
                            uint32_t* scratch_sums2 = nullptr);

// z_trace / u_trace (nullable): each evaluated segment's logits [cap][n_out]
// and FP32 copy of its LDS feature row [cap][n_in] (not in FP8), at the
// segment's queue position; rows of segments not evaluated are untouched.
nbvh_status launch_query_eval(const LaunchCtx& L, const nbvh_ray* rays, const uint32_t* offsets,
                              const nbvh_segment* segs, const uint32_t* active, const uint32_t* n_active,
                              uint32_t* counter, nbvh_hit* hits, uint32_t n_rays_bound, uint64_t capacity,
                              float* z_trace = nullptr, float* u_trace = nullptr);

nbvh_status launch_query_eval_batch(const LaunchCtx* Ls, int n_obj, const DevCfg* cfgs_dev, const uint32_t* const* offsets,
                                    const nbvh_segment* const* segs, const uint32_t* const* active,
                                    const uint32_t* const* n_active, uint32_t* const* counters, nbvh_hit* per_obj,
                                    nbvh_hit* hits, const nbvh_ray* rays, uint32_t n_rays, uint64_t capacity);

nbvh_status launch_first_hits(const LaunchCtx& L, const nbvh_ray* rays, uint32_t n, const float* u,
                              const float* accept, nbvh_probe* probes, uint32_t* leaf_out, uint32_t* n_out,
                              uint32_t* leaf_hits);

size_t group_ws_bytes(uint64_t n);
nbvh_status launch_group_by_leaf(const LaunchCtx& L, uint32_t n_leaves, const nbvh_probe* in, const uint32_t* ids,
                                 uint32_t n, nbvh_probe* out, uint32_t* ids_out, void* ws);

nbvh_status launch_leaf_loss(const LaunchCtx& L, const nbvh_probe* probes, const nbvh_label* labels,
                             const uint32_t* leaf_ids, uint32_t n, float* z, float* leaf_loss, uint32_t* leaf_count);

nbvh_status launch_active_rays(const LaunchCtx& L, const uint32_t* offsets, uint32_t n_rays, nbvh_hit* hits,
                               uint32_t* active, uint32_t* misc);

nbvh_status launch_encode(const LaunchCtx& L, const nbvh_probe* probes, uint32_t n, float* u);

nbvh_status launch_forward(const LaunchCtx& L, const nbvh_probe* probes, uint32_t n, float* z);

// FP8 calibration: weight scales from the FP32 master weights, activation
// scales from an FP32 forward of the given segments, then E4M3 weights.
nbvh_status launch_calibrate_fp8(const LaunchCtx& L, const nbvh_probe* probes, uint32_t n);

// training
size_t train_ws_bytes(const DevCfg& c, int precision, uint64_t max_batch, const nbvh_tuning& tune);
// out[0..n] = exclusive prefix sums of in[0..n) (out[n] = total); sums needs
// n / 1024 + 2 words, total_out one word
nbvh_status launch_exclusive_scan(hipStream_t s, const uint32_t* in, uint32_t n, uint32_t* out, uint32_t* sums,
                                  uint32_t* total_out);
nbvh_status launch_train_fwd_bwd(const LaunchCtx& L, const nbvh_probe* probes, const nbvh_label* labels,
                                 const float* dz_in, uint32_t n, float* loss_dev, void* ws, size_t ws_bytes,
                                 bool apply_grad);
nbvh_status launch_loss(const LaunchCtx& L, const float* z, const nbvh_label* labels, uint32_t n, float* loss_dev,
                        float* dz, void* ws, size_t ws_bytes);
nbvh_status launch_optimizer(const LaunchCtx& L, bool reset, bool shadow_only);
nbvh_status launch_unscale_grad(const LaunchCtx& L, float* out, bool clear);
nbvh_status launch_node_rank(hipStream_t s, const float* loss, const uint32_t* count, const uint32_t* hits, uint32_t n,
                             uint64_t n_rays, float* rank);
nbvh_status launch_acceptance(hipStream_t s, const float* rank, uint32_t n, float floor_, float* accept);

}  // namespace nbvh
