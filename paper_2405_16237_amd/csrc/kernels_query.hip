// Neural ray query evaluation (Sec. 5; Fig. "neural ray query pipeline").
//
// One persistent kernel fuses sampling + hash-grid encoding, the MLP and the
// front-to-back resolve. Each workgroup owns 64 ray slots (wave 0, lane =
// slot). Per iteration every live slot evaluates its ray's current segment:
// all four waves gather the features of the 64 segments into an LDS tile
// (lanes = slots, so a wave's 64 lookups share one level and neighbouring
// rays share cache lines), the tile goes through the MLP on the matrix cores,
// and wave 0 updates each ray's best hit. A ray moves on to its next segment
// only while that segment starts before its best t; otherwise its hit record
// is written and the slot takes the next ray from the queue of rays with at
// least one segment. Workgroups exit when the queue is drained and their
// slots are empty.
#include "launch.h"
#include "mlp_tile.h"
#include "encode_tile.h"

namespace nbvh {

constexpr int kQM = 64;      // slots per workgroup
constexpr int kQWaves = 8;   // waves per workgroup
constexpr uint32_t kXcds = 8;  // accelerator complex dies of an MI355X; ray-queue partitions

// Instantiation choice from the precision, feature count and the tuned
// (waves, unroll, pairs) triple; unroll 0 means 2 (3 with pair loads of
// 4-byte table entries).
#define NBVH_DISPATCH_UNROLL(AT, F, LP, NW, UNR, PR, M) \
  do {                                                   \
    if ((UNR) == 2) M(AT, F, LP, NW, 2, PR);              \
    if ((UNR) == 3) M(AT, F, LP, NW, 3, PR);              \
    M(AT, F, LP, NW, 4, PR);                             \
  } while (0)
#define NBVH_DISPATCH_PAIRS(AT, F, LP, NW, Lc, M)                                                    \
  do {                                                                                             \
    const bool pr_ = (Lc).tune.query_pairs != 0;                                                   \
    const int eb_ = (F) * ((LP) ? 2 : 4);                                                          \
    const int unr_ = (Lc).tune.query_unroll > 0 ? (Lc).tune.query_unroll : (pr_ && eb_ == 4 ? 3 : 2);     \
    if (pr_) NBVH_DISPATCH_UNROLL(AT, F, LP, NW, unr_, true, M);                                   \
    NBVH_DISPATCH_UNROLL(AT, F, LP, NW, unr_, false, M);                                           \
  } while (0)
#define NBVH_DISPATCH_WAVES(AT, F, LP, Lc, M)                                     \
  do {                                                                            \
    if ((Lc).tune.query_waves == 4) NBVH_DISPATCH_PAIRS(AT, F, LP, 4, Lc, M);     \
    NBVH_DISPATCH_PAIRS(AT, F, LP, 8, Lc, M);                                     \
  } while (0)
#define NBVH_DISPATCH_QUERY(Lc, M)                                               \
  do {                                                                           \
    if ((Lc).precision == NBVH_FP32) {                                          \
      if ((Lc).cfg.n_features == 2) NBVH_DISPATCH_WAVES(float, 2, false, Lc, M); \
      NBVH_DISPATCH_WAVES(float, 4, false, Lc, M);                              \
    }                                                                           \
    if ((Lc).fp8) {                                                              \
      if ((Lc).cfg.n_features == 2) NBVH_DISPATCH_WAVES(fp8e4, 2, true, Lc, M); \
      NBVH_DISPATCH_WAVES(fp8e4, 4, true, Lc, M);                               \
    }                                                                           \
    if ((Lc).cfg.n_features == 2) NBVH_DISPATCH_WAVES(bf16, 2, true, Lc, M);     \
    NBVH_DISPATCH_WAVES(bf16, 4, true, Lc, M);                                  \
  } while (0)

__device__ inline uint32_t xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u; }

template <typename AT>
__host__ __device__ inline size_t query_lds_bytes(int n_in, int width) {
  const int ld0 = (n_in > width ? n_in : width) + Pad<AT>::v;
  const int ld1 = width + Pad<AT>::v;
  return (size_t)kQM * (ld0 + ld1) * sizeof(AT) + (size_t)kQM * kOutPad * 4 + (size_t)kQM * 32 + kQM * 4 + 16 +
         (size_t)kQM * 4 * 13;
}

// One object's query inputs.
struct QueryJob {
  const void* table;
  const void* W;
  const float* scales;  // FP8: weight scales [kMaxLayers], then activation scales
  const nbvh_ray* rays;
  const uint32_t* offsets;
  const nbvh_segment* segs;
  const uint32_t* active;
  const uint32_t* n_active;
  uint32_t* counters;  // kXcds ray-queue counters
  nbvh_hit* hits;
  const uint32_t* total_segs;
  uint64_t capacity;
  DevState* state;
  uint32_t lds_words;  // 4-byte words of the table's leading levels copied to LDS (0: none)
  int lds_levels;      // levels gathered from that copy
  // optional per-segment outputs (nullptr: not written), indexed by the
  // segment's queue position: logits [cap][n_out] and features [cap][n_in]
  float* z_trace;
  float* u_trace;
};

// LDS bytes of the slot state and tiles, before the staged table levels
template <typename AT>
__host__ __device__ inline size_t query_ltab_offset(int n_in, int width) {
  return (query_lds_bytes<AT>(n_in, width) + 15) & ~(size_t)15;
}

// The persistent slot loop over one object's ray queue (see the file comment).
// Returns with every slot drained, so a workgroup can move on to another
// object afterwards.
template <typename AT, int F, bool LP, int NW, int U, bool PR>
__device__ inline void query_eval_loop(const DevCfg& c, const QueryJob& J, unsigned char* smem) {
  if ((uint64_t)*J.total_segs > J.capacity) return;  // segment queue overflowed: flagged, nothing to read
  const int ld0 = (c.n_in > c.width ? c.n_in : c.width) + Pad<AT>::v;
  const int ld1 = c.width + Pad<AT>::v;
  AT* act0 = (AT*)smem;
  AT* act1 = act0 + (size_t)kQM * ld0;
  float* z = (float*)(act1 + (size_t)kQM * ld1);
  float4* sA = (float4*)(z + kQM * kOutPad);
  float4* sB = sA + kQM;
  int* s_valid = (int*)(sB + kQM);
  int* s_any = s_valid + kQM;
  // slot state (owned by wave 0, lane = slot), kept in LDS to spare VGPRs
  uint32_t* s_ray = (uint32_t*)(s_any + 4);
  uint32_t* s_cur = s_ray + kQM;
  uint32_t* s_end = s_cur + kQM;
  uint32_t* s_leaf = s_end + kQM;
  uint32_t* s_bleaf = s_leaf + kQM;
  float* s_bt = (float*)(s_bleaf + kQM);
  float* s_bn = s_bt + kQM;       // [3][kQM]
  float* s_ba = s_bn + 3 * kQM;   // [3][kQM]
  float* s_tmin = s_ba + 3 * kQM;
  // the table's leading levels, copied once; the slot loop's first barrier
  // orders the copy before any gather from it
  const unsigned char* ltab = smem + query_ltab_offset<AT>(c.n_in, c.width);
  {
    const uint32_t* src = (const uint32_t*)J.table;
    uint32_t* dst = (uint32_t*)(smem + query_ltab_offset<AT>(c.n_in, c.width));
    for (uint32_t i = threadIdx.x; i < J.lds_words; i += blockDim.x) dst[i] = src[i];
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t n_active = *J.n_active;
  bool exhausted = false;
  const uint32_t first_part = xcc_id() % kXcds;
  uint32_t part = first_part;
  uint32_t evaluated = 0;
  if (wave == 0) s_ray[lane] = NBVH_MISS;

  while (true) {
    if (wave == 0) {
      uint32_t ray = s_ray[lane];
      const bool is_free = (ray == NBVH_MISS);
      // free slots take the next rays of this XCD's eighth of the queue
      // (neighbouring rays read the same table lines, which then stay in
      // one L2); an exhausted eighth moves on to the next one
      uint64_t mask = exhausted ? 0ull : __ballot(is_free);
      while (mask) {
        const uint32_t nfree = (uint32_t)__popcll(mask);
        const uint32_t r0 = (uint32_t)(((uint64_t)n_active * part) / kXcds);
        const uint32_t r1 = (uint32_t)(((uint64_t)n_active * (part + 1)) / kXcds);
        const int leader = __ffsll((unsigned long long)mask) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(J.counters + part, nfree);
        base = __shfl(base, leader);
        if ((mask >> lane) & 1ull) {
          const uint32_t idx = r0 + base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
          if (idx < r1) {
            ray = J.active[idx];
            const uint32_t cur = J.offsets[ray];
            s_ray[lane] = ray;
            s_cur[lane] = cur;
            s_end[lane] = J.offsets[ray + 1];
            s_bt[lane] = INFINITY;
            s_bleaf[lane] = NBVH_MISS;
            const float4* rp = (const float4*)(J.rays + ray);
            const float4 ra = rp[0], rb = rp[1];
            const nbvh_segment sg = J.segs[cur];
            s_leaf[lane] = sg.leaf;
            s_tmin[lane] = ra.w;
            // a leaf around the origin (reversed inside rule) is queried as the
            // chord crossed backwards: origin o, direction -d, [-t1, -t0]
            const bool in = (sg.leaf & NBVH_SEG_INSIDE) != 0u;
            sA[lane] = make_float4(ra.x, ra.y, ra.z, in ? -sg.t1 : sg.t0);
            sB[lane] = in ? make_float4(-rb.x, -rb.y, -rb.z, -sg.t0) : make_float4(rb.x, rb.y, rb.z, sg.t1);
          }
        }
        if (r0 + base + nfree < r1) break;  // this eighth still has rays
        part = (part + 1) % kXcds;
        if (part == first_part) {
          exhausted = true;
          break;
        }
        mask = __ballot(ray == NBVH_MISS);
      }
      s_valid[lane] = (ray != NBVH_MISS) ? 1 : 0;
      const uint64_t live = __ballot(ray != NBVH_MISS);
      if (lane == 0) *s_any = live ? 1 : 0;
    }
    __syncthreads();
    if (*s_any == 0) break;

    // wave 0 fetches each live slot's following segment now, so the load
    // overlaps the encoding and the MLP instead of stalling the resolve
    nbvh_segment nxt{0u, 0u, INFINITY, INFINITY};
    if (wave == 0 && s_valid[lane]) {
      const uint32_t c1 = s_cur[lane] + 1;
      if (c1 < s_end[lane]) nxt = J.segs[c1];
    }
    if constexpr (sizeof(AT) == 1) {
      encode_tile<AT, F, LP, NW, U, PR>(c, J.table, sA, sB, s_valid, act0, ld0, kQM, J.scales[kMaxLayers], ltab,
                                        J.lds_levels);
      __syncthreads();
      mlp_forward_tile_fp8<kQM, NW>(c, (const uint8_t*)J.W, J.scales, (uint8_t*)act0, ld0, (uint8_t*)act1, ld1, z,
                                    kOutPad);
    } else if constexpr (sizeof(AT) == 2) {
      // layer 0's first weight fragments travel while the table is gathered
      const PreBf16 pre0 = prefetch_bf16<NW>((const bf16*)J.W + c.w_off[0], c.fan_in[0], c.fan_in[0], c.fan_out[0]);
      encode_tile<AT, F, LP, NW, U, PR>(c, J.table, sA, sB, s_valid, act0, ld0, kQM, 1.0f, ltab, J.lds_levels);
      __syncthreads();
      if (J.u_trace) {
        for (int e = threadIdx.x; e < kQM * c.n_in; e += blockDim.x) {
          const int m = e / c.n_in, k = e - m * c.n_in;
          if (s_valid[m]) J.u_trace[(size_t)s_cur[m] * c.n_in + k] = (float)act0[m * ld0 + k];
        }
        __syncthreads();
      }
      mlp_forward_tile<kQM, NW, AT>(c, (const AT*)J.W, act0, ld0, act1, ld1, z, kOutPad, &pre0);
    } else {
      encode_tile<AT, F, LP, NW, U, PR>(c, J.table, sA, sB, s_valid, act0, ld0, kQM, 1.0f, ltab, J.lds_levels);
      __syncthreads();
      if (J.u_trace) {  // uniform over the launch: the feature tile as the MLP reads it
        for (int e = threadIdx.x; e < kQM * c.n_in; e += blockDim.x) {
          const int m = e / c.n_in, k = e - m * c.n_in;
          if (s_valid[m]) J.u_trace[(size_t)s_cur[m] * c.n_in + k] = (float)act0[m * ld0 + k];
        }
        __syncthreads();
      }
      mlp_forward_tile<kQM, NW, AT>(c, (const AT*)J.W, act0, ld0, act1, ld1, z, kOutPad);
    }

    if (wave == 0 && s_valid[lane]) {
      ++evaluated;
      const uint32_t ray = s_ray[lane];
      const float t0 = sA[lane].w, t1 = sB[lane].w;
      float best_t = s_bt[lane];
      const float* zr = z + lane * kOutPad;
      if (J.z_trace)
        for (int o = 0; o < c.n_out; ++o) J.z_trace[(size_t)s_cur[lane] * c.n_out + o] = zr[o];
      const uint32_t leaf = s_leaf[lane];
      const bool in = (leaf & NBVH_SEG_INSIDE) != 0u;
      if (zr[0] > 0.0f) {
        // distance along the queried direction; a reversed chord's point is
        // mapped back to the ray and counts only in front of the origin
        const float tq = t0 + sigmoidf_(zr[1]) * (t1 - t0);
        const float t = in ? -tq : tq;
        if (t < best_t && (!in || t > s_tmin[lane])) {
          best_t = t;
          s_bt[lane] = t;
          s_bleaf[lane] = leaf & ~NBVH_SEG_INSIDE;
          s_bn[lane] = zr[2];
          s_bn[kQM + lane] = zr[3];
          s_bn[2 * kQM + lane] = zr[4];
          if (c.n_out >= 8) {
            s_ba[lane] = sigmoidf_(zr[5]);
            s_ba[kQM + lane] = sigmoidf_(zr[6]);
            s_ba[2 * kQM + lane] = sigmoidf_(zr[7]);
          }
        }
      }
      const uint32_t cur = s_cur[lane] + 1;
      s_cur[lane] = cur;
      bool more = false;
      if (cur < s_end[lane] && nxt.t0 < best_t) {
        more = true;
        const bool nin = (nxt.leaf & NBVH_SEG_INSIDE) != 0u;
        s_leaf[lane] = nxt.leaf;
        if (nin != in) {
          sB[lane].x = -sB[lane].x;
          sB[lane].y = -sB[lane].y;
          sB[lane].z = -sB[lane].z;
        }
        sA[lane].w = nin ? -nxt.t1 : nxt.t0;
        sB[lane].w = nin ? -nxt.t0 : nxt.t1;
      }
      if (!more) {
        float4* h = (float4*)(J.hits + ray);
        const uint32_t bl = s_bleaf[lane];
        if (bl == NBVH_MISS) {
          h[0] = make_float4(0.f, 0.f, 0.f, 0.f);
          h[1] = make_float4(0.f, 0.f, 0.f, __uint_as_float(NBVH_MISS));
        } else {
          const bool alb = c.n_out >= 8;
          h[0] = make_float4(best_t, s_bn[lane], s_bn[kQM + lane], s_bn[2 * kQM + lane]);
          h[1] = make_float4(alb ? s_ba[lane] : 0.f, alb ? s_ba[kQM + lane] : 0.f, alb ? s_ba[2 * kQM + lane] : 0.f,
                             __uint_as_float(bl));
        }
        s_ray[lane] = NBVH_MISS;
      }
    }
    __syncthreads();
  }
  if (wave == 0) {
    uint32_t e = evaluated;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if (lane == 0 && e) atomicAdd(&J.state->n_evaluated, (unsigned long long)e);
  }
}

template <typename AT, int F, bool LP, int NW, int U, bool PR>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void k_query_eval(DevCfg c, QueryJob J) {
  extern __shared__ __align__(16) unsigned char smem[];
  query_eval_loop<AT, F, LP, NW, U, PR>(c, J, smem);
}

// Several objects (same network shape, own tables and weights) in one
// launch: each workgroup drains the objects' ray queues starting at a
// different object.
constexpr int kMaxBatch = 16;
struct QueryJobs {
  QueryJob j[kMaxBatch];
  int n;
};

template <typename AT, int F, bool LP, int NW, int U, bool PR>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void k_query_eval_batch(
    const DevCfg* __restrict__ cfgs, QueryJobs jobs) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int i = 0; i < jobs.n; ++i) {
    const int k = (int)((blockIdx.x + (uint32_t)i) % (uint32_t)jobs.n);
    query_eval_loop<AT, F, LP, NW, U, PR>(cfgs[k], jobs.j[k], smem);
    __syncthreads();
  }
}

// Rays with at least one segment, appended in wave order (query over a
// caller-given segment queue). Also clears the ray counter of the eval kernel.
__global__ __launch_bounds__(256) void k_active_rays(const uint32_t* __restrict__ offsets, uint32_t n_rays,
                                                     nbvh_hit* __restrict__ hits, uint32_t* __restrict__ active,
                                                     uint32_t* __restrict__ n_active) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = r < n_rays;
  const bool want = valid && offsets[r + 1] > offsets[r];
  if (valid && !want) {
    float4* h = (float4*)(hits + r);
    h[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    h[1] = make_float4(0.f, 0.f, 0.f, __uint_as_float(NBVH_MISS));
  }
  const uint64_t mask = __ballot(want);
  if (mask) {
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(n_active, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (want) active[base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull))] = r;
  }
}

nbvh_status launch_active_rays(const LaunchCtx& L, const uint32_t* offsets, uint32_t n_rays, nbvh_hit* hits,
                               uint32_t* active, uint32_t* misc) {
  k_zero_u32<<<1, 64, 0, L.stream>>>(misc, 1 + kXcds);
  if (n_rays) k_active_rays<<<(n_rays + 255) / 256, 256, 0, L.stream>>>(offsets, n_rays, hits, active, misc);
  return check_launch("active_rays");
}

// Forward of probe segments: tile of 64 probes per workgroup, z -> global.
template <typename AT, int F, bool LP>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_forward(
    DevCfg c, const void* __restrict__ table, const void* __restrict__ W, const float* __restrict__ scales,
    const nbvh_probe* __restrict__ probes, uint32_t n, float* __restrict__ zout) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ld0 = (c.n_in > c.width ? c.n_in : c.width) + Pad<AT>::v;
  const int ld1 = c.width + Pad<AT>::v;
  AT* act0 = (AT*)smem;
  AT* act1 = act0 + (size_t)kQM * ld0;
  float* z = (float*)(act1 + (size_t)kQM * ld1);
  float4* sA = (float4*)(z + kQM * kOutPad);
  float4* sB = sA + kQM;
  int* s_valid = (int*)(sB + kQM);
  const uint32_t base = blockIdx.x * kQM;
  if (threadIdx.x < kQM) {
    const uint32_t i = base + threadIdx.x;
    const bool v = i < n;
    const float4* p = (const float4*)(probes + (v ? i : 0));
    sA[threadIdx.x] = p[0];
    sB[threadIdx.x] = p[1];
    s_valid[threadIdx.x] = v ? 1 : 0;
  }
  __syncthreads();
  if constexpr (sizeof(AT) == 1) {
    encode_tile<AT, F, LP, kQWaves>(c, table, sA, sB, s_valid, act0, ld0, kQM, scales[kMaxLayers]);
    __syncthreads();
    mlp_forward_tile_fp8<kQM, kQWaves>(c, (const uint8_t*)W, scales, (uint8_t*)act0, ld0, (uint8_t*)act1, ld1, z,
                                       kOutPad);
  } else {
    encode_tile<AT, F, LP, kQWaves>(c, table, sA, sB, s_valid, act0, ld0, kQM);
    __syncthreads();
    mlp_forward_tile<kQM, kQWaves, AT>(c, (const AT*)W, act0, ld0, act1, ld1, z, kOutPad);
  }
  for (int e = threadIdx.x; e < kQM * c.n_out; e += blockDim.x) {
    const int m = e / c.n_out, o = e - m * c.n_out;
    if (base + m < n) zout[(size_t)(base + m) * c.n_out + o] = z[m * kOutPad + o];
  }
}

// Encoding only: thread per (probe, sample, level), FP32 output.
template <int F, bool LP>
__global__ __launch_bounds__(256) void k_encode(DevCfg c, const void* __restrict__ table,
                                                const nbvh_probe* __restrict__ probes, uint32_t n,
                                                float* __restrict__ u) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int SL = c.n_samples * c.n_levels;
  if (t >= (uint64_t)n * SL) return;
  const uint32_t i = (uint32_t)(t / SL);
  const int sl = (int)(t - (uint64_t)i * SL);
  const int s = sl / c.n_levels, l = sl - s * c.n_levels;
  const float4* p = (const float4*)(probes + i);
  const float4 a = p[0], b = p[1];
  const float o[3] = {a.x, a.y, a.z}, d[3] = {b.x, b.y, b.z};
  float x[3], v[F];
  sample_position(c, o, d, a.w, b.w, s, x);
  interp_level<F, LP>(c, table, l, x, v);
#pragma unroll
  for (int f = 0; f < F; ++f) u[(size_t)i * c.n_in + s * c.n_levels * F + l * F + f] = v[f];
}

// ---------------------------------------------------------------------------
// A workgroup's LDS cannot exceed the CU's 160 KiB: wide networks in FP32
// (n_in + width > ~600) do not fit the 64-row tiles and are refused.
static nbvh_status lds_fits(size_t bytes, const char* what) {
  if (bytes > 160 * 1024)
    return set_error("%s needs %zu bytes of LDS (> 160 KiB) for this network and precision", what, bytes),
           NBVH_ERR_UNSUPPORTED;
  return NBVH_OK;
}

template <typename K>
static void set_lds(K kernel, size_t bytes) {
  (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// persistent workgroups per CU: as many as LDS allows (at most 4) unless tuned
static int query_per_cu(const LaunchCtx& L, size_t lds) {
  int per_cu = (int)(160 * 1024 / lds);
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 4) per_cu = 4;
  if (L.tune.query_wgs_per_cu > 0 && L.tune.query_wgs_per_cu < per_cu) per_cu = L.tune.query_wgs_per_cu;
  return per_cu;
}

// merge per-object hit records: closest t, ties to the lower object index
__global__ __launch_bounds__(256) void k_merge_hits(const nbvh_hit* __restrict__ per_obj, uint32_t n_obj, uint32_t n_rays,
                                                    nbvh_hit* __restrict__ hits) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  float4 best0 = make_float4(0.f, 0.f, 0.f, 0.f), best1 = make_float4(0.f, 0.f, 0.f, __uint_as_float(NBVH_MISS));
  bool have = false;
  for (uint32_t k = 0; k < n_obj; ++k) {
    const float4* h = (const float4*)(per_obj + (size_t)k * n_rays + r);
    const float4 a = h[0], b = h[1];
    const uint32_t leaf = __float_as_uint(b.w);
    if (leaf == NBVH_MISS) continue;
    if (!have || a.x < best0.x) {
      best0 = a;
      best1 = make_float4(b.x, b.y, b.z, __uint_as_float((k << 24) | leaf));
      have = true;
    }
  }
  float4* o = (float4*)(hits + r);
  o[0] = best0;
  o[1] = best1;
}

template <typename AT, int F, bool LP, int NW, int U, bool PR>
static nbvh_status query_batch_t(const LaunchCtx* Ls, int n_obj, const DevCfg* cfgs_dev, const QueryJob* jobs,
                                 nbvh_hit* per_obj, nbvh_hit* hits, uint32_t n_rays) {
  const LaunchCtx& L = Ls[0];
  const size_t lds = query_lds_bytes<AT>(L.cfg.n_in, L.cfg.width);
  if (lds_fits(lds, "the query") != NBVH_OK) return NBVH_ERR_UNSUPPORTED;
  auto kern = k_query_eval_batch<AT, F, LP, NW, U, PR>;
  set_lds(kern, lds);
  const int per_cu = query_per_cu(L, lds);
  QueryJobs Q;
  Q.n = n_obj;
  for (int k = 0; k < n_obj; ++k) Q.j[k] = jobs[k];
  {
    ProfScope ps(L.prof, NBVH_K_QUERY_EVAL, L.stream);
    kern<<<(uint32_t)L.n_cu * per_cu, 64 * NW, lds, L.stream>>>(cfgs_dev, Q);
  }
  k_merge_hits<<<(n_rays + 255) / 256, 256, 0, L.stream>>>(per_obj, (uint32_t)n_obj, n_rays, hits);
  return check_launch("query_eval_batch");
}

nbvh_status launch_query_eval_batch(const LaunchCtx* Ls, int n_obj, const DevCfg* cfgs_dev, const uint32_t* const* offsets,
                                    const nbvh_segment* const* segs, const uint32_t* const* active,
                                    const uint32_t* const* n_active, uint32_t* const* counters, nbvh_hit* per_obj,
                                    nbvh_hit* hits, const nbvh_ray* rays, uint32_t n_rays, uint64_t capacity) {
  if (n_obj < 1 || n_obj > kMaxBatch) return set_error("batch of %d objects (1..%d)", n_obj, kMaxBatch), NBVH_ERR_INVALID_ARG;
  QueryJob jobs[kMaxBatch];
  for (int k = 0; k < n_obj; ++k) {
    const LaunchCtx& Lk = Ls[k];
    QueryJob& J = jobs[k];
    J.W = Lk.fp8 ? (const void*)((const char*)Lk.aux + fp8_weights_off(Lk.cfg))
                 : (Lk.precision != NBVH_FP32) ? (const void*)Lk.params_lp : (const void*)Lk.params;
    J.scales = (const float*)((const char*)Lk.aux + fp8_scales_off(Lk.cfg));
    J.table = (Lk.precision != NBVH_FP32) ? (const void*)Lk.params_lp : (const void*)Lk.params;
    J.rays = rays;
    J.offsets = offsets[k];
    J.segs = segs[k];
    J.active = active[k];
    J.n_active = n_active[k];
    J.counters = counters[k];
    J.hits = per_obj + (size_t)k * n_rays;
    J.total_segs = offsets[k] + n_rays;
    J.capacity = capacity;
    J.state = Lk.state;
    J.lds_words = 0;  // objects differ in their tables: nothing staged
    J.lds_levels = 0;
    J.z_trace = nullptr;
    J.u_trace = nullptr;
  }
#define NBVH_QB(AT, F, LP, NW, U, PR) \
  return query_batch_t<AT, F, LP, NW, U, PR>(Ls, n_obj, cfgs_dev, jobs, per_obj, hits, n_rays)
  NBVH_DISPATCH_QUERY(Ls[0], NBVH_QB);
#undef NBVH_QB
}

template <typename AT, int F, bool LP, int NW, int U, bool PR>
static nbvh_status query_eval_t(const LaunchCtx& L, const nbvh_ray* rays, const uint32_t* offsets,
                                const nbvh_segment* segs, const uint32_t* active, const uint32_t* n_active,
                                uint32_t* counter, nbvh_hit* hits, uint32_t n_rays_bound, uint64_t capacity,
                                float* z_trace, float* u_trace) {
  const DevCfg& c = L.cfg;
  // leading levels staged in LDS: as many whole levels as the budget holds
  int lds_levels = 0;
  size_t staged = 0;
  if (!PR && L.tune.query_lds_kb > 0) {
    const size_t budget = (size_t)L.tune.query_lds_kb * 1024, pb = LP ? 2 : 4;
    while (lds_levels < c.n_levels) {
      const size_t end = lds_levels + 1 < c.n_levels ? c.level_off[lds_levels + 1] : c.n_table;
      if (end * pb > budget) break;
      ++lds_levels;
      staged = end * pb;
    }
  }
  const size_t lds = staged ? query_ltab_offset<AT>(c.n_in, c.width) + staged : query_lds_bytes<AT>(c.n_in, c.width);
  if (lds_fits(lds, "the query") != NBVH_OK) return NBVH_ERR_UNSUPPORTED;
  auto kern = k_query_eval<AT, F, LP, NW, U, PR>;
  set_lds(kern, lds);
  uint32_t grid = (uint32_t)L.n_cu * query_per_cu(L, lds);
  const uint32_t need = (n_rays_bound + kQM - 1) / kQM;
  if (need < grid) grid = need > 0 ? need : 1;
  QueryJob J;
  J.W = (sizeof(AT) == 1)   ? (const void*)((const char*)L.aux + fp8_weights_off(c))
        : (sizeof(AT) == 2) ? (const void*)L.params_lp
                            : (const void*)L.params;
  J.scales = (const float*)((const char*)L.aux + fp8_scales_off(c));
  J.table = LP ? (const void*)L.params_lp : (const void*)L.params;
  J.rays = rays;
  J.offsets = offsets;
  J.segs = segs;
  J.active = active;
  J.n_active = n_active;
  J.counters = counter;
  J.hits = hits;
  J.total_segs = offsets + n_rays_bound;
  J.capacity = capacity;
  J.state = L.state;
  J.lds_words = (uint32_t)(staged / 4);
  J.lds_levels = lds_levels;
  J.z_trace = z_trace;
  J.u_trace = sizeof(AT) == 1 ? nullptr : u_trace;
  ProfScope ps(L.prof, NBVH_K_QUERY_EVAL, L.stream);
  kern<<<grid, 64 * NW, lds, L.stream>>>(c, J);
  return check_launch("query_eval");
}

nbvh_status launch_query_eval(const LaunchCtx& L, const nbvh_ray* rays, const uint32_t* offsets,
                              const nbvh_segment* segs, const uint32_t* active, const uint32_t* n_active,
                              uint32_t* counter, nbvh_hit* hits, uint32_t n_rays_bound, uint64_t capacity,
                              float* z_trace, float* u_trace) {
#define NBVH_QE(AT, F, LP, NW, U, PR)                                                                          \
  return query_eval_t<AT, F, LP, NW, U, PR>(L, rays, offsets, segs, active, n_active, counter, hits, n_rays_bound, \
                                            capacity, z_trace, u_trace)
  NBVH_DISPATCH_QUERY(L, NBVH_QE);
#undef NBVH_QE
}

template <typename AT, int F, bool LP>
static nbvh_status forward_t(const LaunchCtx& L, const nbvh_probe* probes, uint32_t n, float* z) {
  const DevCfg& c = L.cfg;
  const size_t lds = query_lds_bytes<AT>(c.n_in, c.width);
  if (lds_fits(lds, "the forward pass") != NBVH_OK) return NBVH_ERR_UNSUPPORTED;
  auto kern = k_forward<AT, F, LP>;
  set_lds(kern, lds);
  const void* W = (sizeof(AT) == 1)   ? (const void*)((const char*)L.aux + fp8_weights_off(c))
                  : (sizeof(AT) == 2) ? (const void*)L.params_lp
                                      : (const void*)L.params;
  const float* scales = (const float*)((const char*)L.aux + fp8_scales_off(c));
  const void* table = LP ? (const void*)L.params_lp : (const void*)L.params;
  if (n == 0) return NBVH_OK;
  ProfScope ps(L.prof, NBVH_K_FORWARD, L.stream);
  kern<<<(n + kQM - 1) / kQM, 64 * kQWaves, lds, L.stream>>>(c, table, W, scales, probes, n, z);
  return check_launch("forward");
}

nbvh_status launch_forward(const LaunchCtx& L, const nbvh_probe* probes, uint32_t n, float* z) {
  const int F = L.cfg.n_features;
  if (L.precision == NBVH_FP32) return F == 2 ? forward_t<float, 2, false>(L, probes, n, z) : forward_t<float, 4, false>(L, probes, n, z);
  if (L.fp8) return F == 2 ? forward_t<fp8e4, 2, true>(L, probes, n, z) : forward_t<fp8e4, 4, true>(L, probes, n, z);
  return F == 2 ? forward_t<bf16, 2, true>(L, probes, n, z) : forward_t<bf16, 4, true>(L, probes, n, z);
}

nbvh_status launch_encode(const LaunchCtx& L, const nbvh_probe* probes, uint32_t n, float* u) {
  const DevCfg& c = L.cfg;
  const uint64_t total = (uint64_t)n * c.n_samples * c.n_levels;
  if (total == 0) return NBVH_OK;
  const uint32_t grid = (uint32_t)((total + 255) / 256);
  const bool lp = L.precision != NBVH_FP32;
  const void* table = lp ? (const void*)L.params_lp : (const void*)L.params;
  if (c.n_features == 2) {
    if (lp) k_encode<2, true><<<grid, 256, 0, L.stream>>>(c, table, probes, n, u);
    else k_encode<2, false><<<grid, 256, 0, L.stream>>>(c, table, probes, n, u);
  } else {
    if (lp) k_encode<4, true><<<grid, 256, 0, L.stream>>>(c, table, probes, n, u);
    else k_encode<4, false><<<grid, 256, 0, L.stream>>>(c, table, probes, n, u);
  }
  return check_launch("encode");
}


// ---------------------------------------------------------------------------
// FP8 calibration. Every amax is a maximum of non-negative floats, whose bit
// patterns order like unsigned integers, so it is kept with integer atomicMax.
__device__ inline void amax_lds(float* dst, float v) { atomicMax((unsigned int*)dst, __float_as_uint(v)); }

__device__ inline float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// amax |W_k| per layer: blockIdx.y = layer
__global__ __launch_bounds__(256) void k_weight_amax(DevCfg c, const float* __restrict__ params,
                                                     float* __restrict__ amax_w) {
  const int k = blockIdx.y;
  const float* W = params + c.w_off[k];
  const uint64_t cnt = (uint64_t)c.fan_in[k] * c.fan_out[k];
  float m = 0.0f;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(W[i]));
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) amax_lds(amax_w + k, m);
}

// amax of each layer's input over a tile of calibration segments: the
// encoded features (layer 0) and the ReLU outputs (layers 1..H), from the
// BF16 table the FP8 query reads and the FP32 master weights.
template <int F>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_calib_act(
    DevCfg c, const void* __restrict__ table, const float* __restrict__ W, const nbvh_probe* __restrict__ probes,
    uint32_t n, float* __restrict__ amax_act) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ld0 = (c.n_in > c.width ? c.n_in : c.width) + Pad<float>::v;
  const int ld1 = c.width + Pad<float>::v;
  float* act0 = (float*)smem;
  float* act1 = act0 + (size_t)kQM * ld0;
  float* z = act1 + (size_t)kQM * ld1;
  float4* sA = (float4*)(z + kQM * kOutPad);
  float4* sB = sA + kQM;
  int* s_valid = (int*)(sB + kQM);
  float* s_amax = (float*)(s_valid + kQM);  // [kMaxLayers], fits the 4 + 12 * kQM words after s_valid
  const uint32_t base = blockIdx.x * kQM;
  if (threadIdx.x < kQM) {
    const uint32_t i = base + threadIdx.x;
    const bool v = i < n;
    const float4* p = (const float4*)(probes + (v ? i : 0));
    sA[threadIdx.x] = p[0];
    sB[threadIdx.x] = p[1];
    s_valid[threadIdx.x] = v ? 1 : 0;
  }
  if (threadIdx.x < kMaxLayers) s_amax[threadIdx.x] = 0.0f;
  __syncthreads();
  encode_tile<float, F, true, kQWaves>(c, table, sA, sB, s_valid, act0, ld0, kQM);
  __syncthreads();
  float m0 = 0.0f;
  for (int e = threadIdx.x; e < kQM * c.n_in; e += blockDim.x) {
    const int m = e / c.n_in, k = e - m * c.n_in;
    if (s_valid[m]) m0 = fmaxf(m0, fabsf(act0[(size_t)m * ld0 + k]));
  }
  m0 = wave_max(m0);
  if ((threadIdx.x & 63) == 0) amax_lds(s_amax, m0);
  mlp_forward_tile_keep<kQM, kQWaves, float>(c, W, act0, ld0, act1, ld1, z, kOutPad,
                                             [&](int k, int m, int, f32x4 v) {
                                               if (s_valid[m]) {
                                                 const float mx = fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3]));
                                                 amax_lds(s_amax + k + 1, mx);
                                               }
                                             });
  __syncthreads();
  if (threadIdx.x <= (unsigned)c.hidden) atomicMax((unsigned int*)(amax_act + threadIdx.x), __float_as_uint(s_amax[threadIdx.x]));
}

// scales from the amax values: 448 (the largest E4M3 value) / amax, 1 where
// amax is zero
__global__ __launch_bounds__(64) void k_fp8_scales(DevCfg c, float* __restrict__ f) {
  const int k = threadIdx.x;
  if (k > c.hidden) return;
  const float aw = f[2 * kMaxLayers + k], aa = f[3 * kMaxLayers + k];
  f[k] = aw > 0.0f ? 448.0f / aw : 1.0f;
  f[kMaxLayers + k] = aa > 0.0f ? 448.0f / aa : 1.0f;
}

// E4M3 weights: W8_k = fp8(W_k * sw_k), four at a time; blockIdx.y = layer
__global__ __launch_bounds__(256) void k_quantize_weights(DevCfg c, const float* __restrict__ params,
                                                          const float* __restrict__ f, uint8_t* __restrict__ w8) {
  const int k = blockIdx.y;
  const float4* W = (const float4*)(params + c.w_off[k]);
  uint32_t* dst = (uint32_t*)(w8 + (c.w_off[k] - c.w_off[0]));
  const uint64_t cnt4 = (uint64_t)c.fan_in[k] * c.fan_out[k] / 4;
  const float s = f[k];
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt4; i += (uint64_t)gridDim.x * blockDim.x) {
    const float4 v = W[i];
    dst[i] = pack_fp8x4(v.x * s, v.y * s, v.z * s, v.w * s);
  }
}

nbvh_status launch_calibrate_fp8(const LaunchCtx& L, const nbvh_probe* probes, uint32_t n) {
  const DevCfg& c = L.cfg;
  float* f = (float*)((char*)L.aux + fp8_scales_off(c));
  uint8_t* w8 = (uint8_t*)L.aux + fp8_weights_off(c);
  k_zero_u32<<<1, 64, 0, L.stream>>>((uint32_t*)(f + 2 * kMaxLayers), 2 * kMaxLayers);
  k_weight_amax<<<dim3(64, c.hidden + 1), 256, 0, L.stream>>>(c, L.params, f + 2 * kMaxLayers);
  const size_t lds = query_lds_bytes<float>(c.n_in, c.width);
  if (lds_fits(lds, "FP8 calibration (an FP32 forward)") != NBVH_OK) return NBVH_ERR_UNSUPPORTED;
  const void* table = L.params_lp;
  if (c.n_features == 2) {
    set_lds(k_calib_act<2>, lds);
    k_calib_act<2><<<(n + kQM - 1) / kQM, 64 * kQWaves, lds, L.stream>>>(c, table, L.params, probes, n, f + 3 * kMaxLayers);
  } else {
    set_lds(k_calib_act<4>, lds);
    k_calib_act<4><<<(n + kQM - 1) / kQM, 64 * kQWaves, lds, L.stream>>>(c, table, L.params, probes, n, f + 3 * kMaxLayers);
  }
  k_fp8_scales<<<1, 64, 0, L.stream>>>(c, f);
  k_quantize_weights<<<dim3(64, c.hidden + 1), 256, 0, L.stream>>>(c, L.params, f, w8);
  return check_launch("calibrate_fp8");
}

}  // namespace nbvh
