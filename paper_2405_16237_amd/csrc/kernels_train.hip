// Training step (Sec. 4: query the model on probe segments, compare with the
// ground truth, back-propagate into the MLP weights and the hash-table
// features; Sec. 5.2: losses; Sec. 6: Adam, learning rate 0.01).
//
//  k_train_tile   per 64 probes: encode -> MLP forward (activations in LDS,
//                 ReLU masks as bits) -> loss and dL/dz (times the loss
//                 scale) -> dgrad back through the layers on the matrix
//                 cores. It stores the weight-gradient operands h_k^T and
//                 g_k^T (feature-major, batch-minor) and dL/du^T.
//  k_wgrad_rows / k_wgrad   dL/dW_k = sum_b g_k[b] h_k[b]^T as split-K MFMA
//                 GEMMs into per-split partials (BF16: every output row per
//                 workgroup, activation slices shared through LDS);
//                 k_wgrad_reduce adds them into grad in a fixed order.
//  k_scatter_* / k_bin_*   recompute every sample's cell corners and weights
//                 (no stored encodings) and add w * dL/du into the table
//                 gradient: mid levels summed per probe tile in an LDS hash
//                 (64-bit fixed point) then flushed with FP32 atomics, fine
//                 levels counting-sorted into 64 KiB table chunks and summed
//                 per chunk in LDS with no global atomics; coarse dense levels
//                 held whole in LDS and coalesced atomics are tunable routes.
//  k_check_finite / k_adam / k_adam_finalize   dense Adam with loss-scale
//                 removal and non-finite skip; writes the BF16 shadow and the
//                 transposed weight copies the dgrad reads.
#include "launch.h"
#include "mlp_tile.h"
#include "encode_tile.h"

namespace nbvh {

constexpr int kTM = 64;
constexpr int kGPad = 32;  // gradient rows of the output layer padded to 32
constexpr uint32_t kBinChunk = 8192;   // binned scatter: parameters per bin (64-bit accumulators in LDS)
constexpr int kBinWgs = 512;           // binned scatter: workgroups of the count / write passes

__host__ __device__ inline int fan_out_pad(const DevCfg& c, int k) {
  return k == c.hidden ? kGPad : c.fan_out[k];
}

// workspace carve-up (offsets in bytes)
struct TrainLayout {
  size_t hT[kMaxLayers], gT[kMaxLayers];
  size_t duT, wpart, loss_part, gmax, total;
  int nsplit;
  uint32_t n_tiles;
  // scatter: levels [0, n_lds) in LDS, [n_lds, hash_end) through the
  // per-tile LDS hash, the rest binned or by pairs
  int n_lds, hash_end;
  uint32_t lds_floats, n_bins;
  uint64_t max_records;
  bool rec8;  // binned records of two-feature tables: 8 bytes (24-bit values) instead of 12
  size_t counts, offsets, scan_sums, rec_idx, rec_val;
};
static int coarse_lds_levels(const DevCfg& c, size_t budget_bytes, uint32_t* n_floats);

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static TrainLayout train_layout(const DevCfg& c, int precision, uint64_t max_batch, const nbvh_tuning& tune) {
  TrainLayout T;
  const size_t es = precision == NBVH_FP32 ? 4 : 2;
  const uint64_t B = (max_batch + kTM - 1) / kTM * kTM;
  size_t off = 0;
  for (int k = 0; k <= c.hidden; ++k) {
    T.hT[k] = off;
    off = align256(off + (size_t)c.fan_in[k] * B * es);
  }
  for (int k = 0; k <= c.hidden; ++k) {
    T.gT[k] = off;
    off = align256(off + (size_t)fan_out_pad(c, k) * B * es);
  }
  T.duT = off;
  off = align256(off + (size_t)c.n_in * B * 4);
  T.nsplit = tune.wgrad_splits > 0 ? tune.wgrad_splits : 32;
  T.wpart = off;
  off = align256(off + (size_t)T.nsplit * (c.n_params - c.w_off[0]) * 4);
  T.n_tiles = (uint32_t)(B / kTM);
  T.loss_part = off;
  off = align256(off + (size_t)T.n_tiles * 4 * 4);
  T.gmax = off;
  off = align256(off + 4);
  const int budget_kb = tune.scatter_lds_kb < 0 ? 0 : (tune.scatter_lds_kb > 144 ? 144 : tune.scatter_lds_kb);
  T.lds_floats = 0;
  T.n_lds = budget_kb > 0 ? coarse_lds_levels(c, (size_t)budget_kb * 1024, &T.lds_floats) : 0;
  T.hash_end = T.n_lds + (tune.scatter_hash_levels > 0 ? tune.scatter_hash_levels : 0);
  if (T.hash_end > c.n_levels) T.hash_end = c.n_levels;
  T.n_bins = 0;
  T.max_records = 0;
  T.rec8 = c.n_features == 2 && precision != NBVH_FP32;
  T.counts = T.offsets = T.scan_sums = T.rec_idx = T.rec_val = off;
  if (tune.scatter_binned && T.hash_end < c.n_levels) {
    const uint64_t off0 = c.level_off[T.hash_end];
    T.n_bins = (uint32_t)((c.n_table - off0 + kBinChunk - 1) / kBinChunk);
    T.max_records = B * (uint64_t)(c.n_levels - T.hash_end) * c.n_samples * 8;
    const size_t cells = (size_t)T.n_bins * kBinWgs;
    T.counts = off;
    off = align256(off + cells * 4);
    T.offsets = off;
    off = align256(off + (cells + 1) * 4);
    T.scan_sums = off;
    off = align256(off + (cells / 1024 + 4) * 4);
    T.rec_idx = off;  // F = 2 keeps the entry inside its record
    if (c.n_features != 2) off = align256(off + T.max_records * 2);
    T.rec_val = off;
    off = align256(off + T.max_records * (c.n_features == 2 ? (T.rec8 ? 8 : 12) : c.n_features * 4));
  }
  T.total = off;
  return T;
}

size_t train_ws_bytes(const DevCfg& c, int precision, uint64_t max_batch, const nbvh_tuning& tune) {
  if (max_batch == 0) return 0;
  return train_layout(c, precision, max_batch, tune).total;
}

template <typename AT>
__host__ __device__ inline size_t train_lds_bytes(const DevCfg& c) {
  const int ld0 = (c.n_in > c.width ? c.n_in : c.width) + Pad<AT>::v;
  const int ld1 = c.width + Pad<AT>::v;
  const int ldg = kGPad + Pad<AT>::v;
  const size_t words = (size_t)c.hidden * kTM * (c.width / 32);
  return (size_t)kTM * (ld0 + ld1 + ldg) * sizeof(AT) + (size_t)kTM * kOutPad * 4 + words * 4 + (size_t)kTM * 32 +
         kTM * 4 + 64;
}

struct TrainPtrs {
  void* hT[kMaxLayers];
  void* gT[kMaxLayers];
  float* duT;
  float* loss_part;
  uint32_t* gmax;  // bits of max |dL/du| over the batch (+inf bits if a value is not finite)
  uint64_t ldb;    // batch stride of the feature-major buffers
};

template <typename AT>
__device__ inline void put(AT* p, float v) {  // a global activation or gradient entry
  global_store<AT>(p, (AT)v);
}

// Albedo (outputs 5..7 through a sigmoid; Sec. 5.2 "Auxiliary data"): relative
// L2, (a_hat - a)^2 / (a_hat^2 + 0.01) averaged over the channels. As relative
// L2 losses are defined, the denominator normalises the error and is held
// constant in the derivative: d/da_hat = 2 (a_hat - a) / (a_hat^2 + 0.01).
// Returns the term and writes d(term)/dz for the three outputs.
__device__ inline float albedo_term(const float* zr, const float* a, float dz[3]) {
  float s = 0.0f;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    const float ah = sigmoidf_(zr[5 + ch]);
    const float den = ah * ah + 0.01f;
    const float d = ah - a[ch];
    s += d * d / den;
    dz[ch] = 2.0f * d / den * ah * (1.0f - ah) * (1.0f / 3.0f);
  }
  return s * (1.0f / 3.0f);
}

__device__ inline float bce_logits(float z, float h) {
  return fmaxf(z, 0.0f) - z * h + log1pf(__expf(-fabsf(z)));
}
__device__ inline float sgnf(float v) { return (float)((v > 0.0f) - (v < 0.0f)); }

template <typename AT, int F, bool LP, bool WITH_LABELS, int kTWaves>
__global__ __launch_bounds__(64 * kTWaves) __attribute__((amdgpu_waves_per_eu(4))) void k_train_tile(DevCfg c, const void* __restrict__ table, const AT* __restrict__ W,
                                                    const AT* __restrict__ WT, const nbvh_probe* __restrict__ probes,
                                                    const nbvh_label* __restrict__ labels,
                                                    const float* __restrict__ dz_in, uint32_t n, TrainPtrs P,
                                                    DevState* __restrict__ state, float w_hit, float w_t,
                                                    float w_normal, float w_albedo) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ld0 = (c.n_in > c.width ? c.n_in : c.width) + Pad<AT>::v;
  const int ld1 = c.width + Pad<AT>::v;
  const int ldg = kGPad + Pad<AT>::v;
  const int mw = c.width / 32;  // mask words per row and layer
  AT* act0 = (AT*)smem;
  AT* act1 = act0 + (size_t)kTM * ld0;
  AT* gz = act1 + (size_t)kTM * ld1;
  float* z = (float*)(gz + (size_t)kTM * ldg);
  uint32_t* masks = (uint32_t*)(z + kTM * kOutPad);
  float4* sA = (float4*)(masks + (size_t)c.hidden * kTM * mw);
  float4* sB = sA + kTM;
  int* s_valid = (int*)(sB + kTM);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t tile = die_contiguous_tile(blockIdx.x, gridDim.x);
  const uint32_t base = tile * kTM;
  const uint64_t ldb = P.ldb;
  if (tid < kTM) {
    const uint32_t i = base + tid;
    const bool v = i < n;
    const float4* p = (const float4*)(probes + (v ? i : 0));
    sA[tid] = p[0];
    sB[tid] = p[1];
    s_valid[tid] = v ? 1 : 0;
  }
  for (int e = tid; e < c.hidden * kTM * mw; e += blockDim.x) masks[e] = 0u;
  __syncthreads();

  // 1. encode -> act0, and h_0^T (= u^T) to global
  encode_tile<AT, F, LP, kTWaves>(c, table, sA, sB, s_valid, act0, ld0, kTM);
  __syncthreads();
  {
    AT* h0 = (AT*)P.hT[0];
    for (int e = tid; e < kTM * c.n_in; e += blockDim.x) {
      const int i = e / kTM, m = e - i * kTM;
      global_store<AT>(h0 + (size_t)i * ldb + base + m, act0[(size_t)m * ld0 + i]);
    }
  }

  // 2. forward; hidden outputs -> masks + h_{k+1}^T
  mlp_forward_tile_keep<kTM, kTWaves, AT>(c, W, act0, ld0, act1, ld1, z, kOutPad,
                                          [&](int k, int m, int col, f32x4 v) {
                                            uint32_t bits = 0;
#pragma unroll
                                            for (int i = 0; i < 4; ++i) bits |= (v[i] > 0.0f ? 1u : 0u) << i;
                                            atomicOr(&masks[((size_t)k * kTM + m) * mw + (col >> 5)], bits << (col & 31));
                                            AT* hk = (AT*)P.hT[k + 1];
                                            const bool ok = s_valid[m] != 0;
#pragma unroll
                                            for (int i = 0; i < 4; ++i)
                                              put<AT>(hk + (size_t)(col + i) * ldb + base + m, ok ? v[i] : 0.0f);
                                          });

  // 3. loss and dL/dz (scaled) -> gz (LDS) and g_H^T (global)
  const float scale = state->loss_scale;
  const float invB = 1.0f / (float)n;
  float l_bce = 0.f, l_t = 0.f, l_n = 0.f, l_a = 0.f;
  if (wave == 0) {
    const int m = lane;
    const bool ok = s_valid[m] != 0;
    float g[kGPad];
#pragma unroll
    for (int o = 0; o < kGPad; ++o) g[o] = 0.0f;
    if (ok) {
      const float* zr = z + m * kOutPad;
      if (WITH_LABELS) {
        const nbvh_label lb = labels[base + m];
        const float h = lb.hit, tau = lb.tau;
        const float st = sigmoidf_(zr[1]);
        l_bce = bce_logits(zr[0], h);
        l_t = h * fabsf(st - tau);
        float ln = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) ln += fabsf(zr[2 + a] - lb.n[a]);
        l_n = h * ln * (1.0f / 3.0f);
        const float sB_ = scale * invB;
        g[0] = w_hit * (sigmoidf_(zr[0]) - h) * sB_;
        g[1] = h * w_t * sgnf(st - tau) * st * (1.0f - st) * sB_;
#pragma unroll
        for (int a = 0; a < 3; ++a) g[2 + a] = h * w_normal * sgnf(zr[2 + a] - lb.n[a]) * (1.0f / 3.0f) * sB_;
        if (c.n_out >= 8) {
          float da[3];
          l_a = h * albedo_term(zr, lb.albedo, da);
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) g[5 + ch] = h * w_albedo * da[ch] * sB_;
        }
      } else {
        for (int o = 0; o < c.n_out; ++o) g[o] = dz_in[(size_t)(base + m) * c.n_out + o] * scale;
      }
      bool fin = true;
#pragma unroll
      for (int o = 0; o < kGPad; ++o) fin = fin && isfinite(g[o]);
      if (!fin) atomicOr(&state->nonfinite_pending, 1u);
    }
    AT* gH = (AT*)P.gT[c.hidden];
#pragma unroll
    for (int o = 0; o < kGPad; ++o) {
      gz[(size_t)m * ldg + o] = (AT)g[o];
      global_store<AT>(gH + (size_t)o * ldb + base + m, (AT)g[o]);
    }
    if (WITH_LABELS) {
      // wave reduction of the per-probe loss terms
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        l_bce += __shfl_xor(l_bce, off);
        l_t += __shfl_xor(l_t, off);
        l_n += __shfl_xor(l_n, off);
        l_a += __shfl_xor(l_a, off);
      }
      if (lane == 0) {
        P.loss_part[tile * 4 + 0] = l_bce;
        P.loss_part[tile * 4 + 1] = l_t;
        P.loss_part[tile * 4 + 2] = l_n;
        P.loss_part[tile * 4 + 3] = l_a;
      }
    }
  }
  __syncthreads();

  // 4. dgrad: g_in^T = W_k^T g_k^T, masked by h_k > 0 (k >= 1); k = 0 gives du
  const AT* gcur = gz;
  int ldcur = ldg;
  AT* bufs[2] = {act0, act1};
  int lds_[2] = {ld0, ld1};
  int which = 0;
  for (int k = c.hidden; k >= 0; --k) {
    const int K = (k == c.hidden) ? Pad<AT>::kstep : c.fan_out[k];
    const int ldw = fan_out_pad(c, k);
    const AT* Wt = WT + c.wt_off[k];
    if (k > 0) {
      AT* out = bufs[which];
      const int ldo = lds_[which];
      AT* gk = (AT*)P.gT[k - 1];
      gemm_tile<kTM, kTWaves, AT>(gcur, ldcur, K, Wt, ldw, c.fan_in[k], [&](int m, int col, f32x4 v) {
        const uint32_t word = masks[((size_t)(k - 1) * kTM + m) * mw + (col >> 5)] >> (col & 31);
        const bool ok = s_valid[m] != 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = (ok && ((word >> i) & 1u)) ? v[i] : 0.0f;
        store4<AT>(out + (size_t)m * ldo + col, v);
#pragma unroll
        for (int i = 0; i < 4; ++i) put<AT>(gk + (size_t)(col + i) * ldb + base + m, v[i]);
      });
      __syncthreads();
      gcur = out;
      ldcur = ldo;
      which ^= 1;
    } else {
      float* du = P.duT;
      float gm = 0.0f;
      bool bad = false;
      gemm_tile<kTM, kTWaves, AT>(gcur, ldcur, K, Wt, ldw, c.fan_in[0], [&](int m, int col, f32x4 v) {
        const bool ok = s_valid[m] != 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float x = ok ? v[i] : 0.0f;
          global_store<float>(du + (size_t)(col + i) * ldb + base + m, x);
          gm = fmaxf(gm, fabsf(x));
          bad = bad || !isfinite(x);
        }
      });
      // the scatter's fixed-point scale comes from the largest |dL/du|
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) gm = fmaxf(gm, __shfl_xor(gm, off));
      const bool any_bad = __ballot(bad) != 0ull;
      if ((threadIdx.x & 63) == 0) atomicMax(P.gmax, any_bad ? 0x7f800000u : __float_as_uint(gm));
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: per (layer tile 64 x 64, split) one workgroup; wave w owns
// output rows o0 + 16w .. +15 and 64 columns (4 MFMA tiles).
struct WTile {
  int16_t layer, o0, i0, pad;
};
struct WTiles {
  WTile t[160];
  int n;
};

template <typename AT>
__global__ __launch_bounds__(256) void k_wgrad(DevCfg c, WTiles tiles, TrainPtrs P, uint32_t kb, int nsplit,
                                               float* __restrict__ wpart) {
  const WTile T = tiles.t[blockIdx.x];
  const int split = blockIdx.y;
  const int k = T.layer;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, q = lane >> 4;
  const int o0 = T.o0 + 16 * wave;
  const int fo_pad = fan_out_pad(c, k);
  if (o0 >= fo_pad) return;
  const int fi = c.fan_in[k];
  const uint64_t ldb = P.ldb;
  // ceil(kb / nsplit) rounded up to 32 batch entries: the splits cover the whole batch
  const uint32_t chunk = ((kb + (uint32_t)nsplit - 1u) / (uint32_t)nsplit + 31u) / 32u * 32u;
  const uint32_t b_beg = split * chunk;
  uint32_t b_end = b_beg + chunk;
  if (b_end > kb) b_end = kb;
  const AT* gT = (const AT*)P.gT[k];
  const AT* hT = (const AT*)P.hT[k];
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const AT* arow = gT + (size_t)(o0 + r16) * ldb;
  if constexpr (sizeof(AT) == 2) {
    for (uint32_t b = b_beg; b < b_end; b += 32) {
      const bf16x8 a = *(const bf16x8*)(arow + b + 8 * q);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = T.i0 + 16 * j + r16;
        const bf16x8 bv = (i < fi) ? *(const bf16x8*)(hT + (size_t)i * ldb + b + 8 * q) : zero_bf16x8();
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[j], 0, 0, 0);
      }
    }
  } else {
    for (uint32_t b = b_beg; b < b_end; b += 16) {
      const float4 a = *(const float4*)(arow + b + 4 * q);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = T.i0 + 16 * j + r16;
        const float4 bv = (i < fi) ? *(const float4*)(hT + (size_t)i * ldb + b + 4 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bv.x, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bv.y, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, bv.z, acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, bv.w, acc[j], 0, 0, 0);
      }
    }
  }
  const uint64_t span = c.n_params - c.w_off[0];
  float* dst = wpart + (size_t)split * span + (c.w_off[k] - c.w_off[0]);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = T.i0 + 16 * j + r16;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int o = o0 + 4 * q + e;
      if (o < c.fan_out[k] && i < fi) dst[(size_t)o * fi + i] = acc[j][e];
    }
  }
}

// BF16 weight gradient, one workgroup per (layer, 128-column input slice,
// split): 8 waves own all output rows (wave w: row tiles w and w + 8), the
// split's h_k^T rows of the slice are staged in LDS 32 batch entries at a time
// (double-buffered) and shared by the waves, so every h_k^T and g_k^T element
// is read from memory once per slice.
constexpr int kWgCols = 128;       // input columns per workgroup
constexpr int kWgLd = 40;          // LDS row stride (bf16): 80 B keeps 16-lane phases conflict-free
struct WSlices {
  int16_t layer[64], i0[64];
  int n;
};

__global__ __launch_bounds__(512) void k_wgrad_rows(DevCfg c, WSlices sl, TrainPtrs P, uint32_t kb, int nsplit,
                                                    float* __restrict__ wpart) {
  __shared__ __align__(16) bf16 stage[2][kWgCols * kWgLd];
  const int k = sl.layer[blockIdx.x], i0 = sl.i0[blockIdx.x];
  const int split = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, q = lane >> 4;
  const int fo_pad = fan_out_pad(c, k), fi = c.fan_in[k];
  const int ncols = min(kWgCols, fi - i0);
  const uint64_t ldb = P.ldb;
  // ceil(kb / nsplit) rounded up to 32 batch entries: the splits cover the whole batch
  const uint32_t chunk = ((kb + (uint32_t)nsplit - 1u) / (uint32_t)nsplit + 31u) / 32u * 32u;
  const uint32_t b_beg = min(kb, split * chunk);
  const uint32_t b_end = min(kb, b_beg + chunk);
  const int n_it = (int)((b_end - b_beg) / 32);
  const bf16* gT = (const bf16*)P.gT[k];
  const bf16* hT = (const bf16*)P.hT[k];
  // staging role: row sr of the slice, 8 batch entries at 8 * sp
  const int sr = tid >> 2, sp = tid & 3;
  const bool s_ok = sr < ncols;
  const bf16* s_src = hT + (size_t)(i0 + (s_ok ? sr : 0)) * ldb + 8 * sp;
  bf16* s_dst0 = &stage[0][sr * kWgLd + 8 * sp];
  bf16* s_dst1 = &stage[1][sr * kWgLd + 8 * sp];
  // compute role: row tiles wave and wave + 8
  const bool rt0 = 16 * wave < fo_pad, rt1 = 16 * (wave + 8) < fo_pad;
  const bf16* a_src0 = gT + (size_t)(16 * wave + r16) * ldb + 8 * q;
  const bf16* a_src1 = gT + (size_t)(16 * (wave + 8) + r16) * ldb + 8 * q;
  f32x4 acc0[8], acc1[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc0[j] = acc1[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (n_it > 0) {
    const bf16x8 h = s_ok ? *(const bf16x8*)(s_src + b_beg) : zero_bf16x8();
    if (sr < kWgCols) *(bf16x8*)s_dst0 = h;
  }
  bf16x8 a0 = (n_it > 0 && rt0) ? *(const bf16x8*)(a_src0 + b_beg) : zero_bf16x8();
  bf16x8 a1 = (n_it > 0 && rt1) ? *(const bf16x8*)(a_src1 + b_beg) : zero_bf16x8();
  __syncthreads();
  for (int it = 0; it < n_it; ++it) {
    const uint32_t b = b_beg + 32u * (uint32_t)it;
    const bool more = it + 1 < n_it;
    // the next slice of h^T and g^T travels while this one multiplies
    bf16x8 hn = zero_bf16x8(), an0 = zero_bf16x8(), an1 = zero_bf16x8();
    if (more && s_ok) hn = *(const bf16x8*)(s_src + b + 32);
    if (more && rt0) an0 = *(const bf16x8*)(a_src0 + b + 32);
    if (more && rt1) an1 = *(const bf16x8*)(a_src1 + b + 32);
    const bf16* cur = stage[it & 1];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (16 * j < ncols) {
        const bf16x8 bv = *(const bf16x8*)(cur + (16 * j + r16) * kWgLd + 8 * q);
        if (rt0) acc0[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv, acc0[j], 0, 0, 0);
        if (rt1) acc1[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bv, acc1[j], 0, 0, 0);
      }
    }
    if (more) *(bf16x8*)((it & 1) ? s_dst0 : s_dst1) = hn;
    a0 = an0;
    a1 = an1;
    __syncthreads();
  }
  const uint64_t span = c.n_params - c.w_off[0];
  float* dst = wpart + (size_t)split * span + (c.w_off[k] - c.w_off[0]);
  const int fo = c.fan_out[k];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = i0 + 16 * j + r16;
    if (16 * j >= ncols || i >= fi) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int o = 16 * wave + 4 * q + e;
      if (rt0 && o < fo) dst[(size_t)o * fi + i] = acc0[j][e];
      const int o1 = o + 128;
      if (rt1 && o1 < fo) dst[(size_t)o1 * fi + i] = acc1[j][e];
    }
  }
}

__global__ __launch_bounds__(256) void k_wgrad_reduce(DevCfg c, const float* __restrict__ wpart, int nsplit,
                                                      float* __restrict__ grad, DevState* __restrict__ state) {
  // four lanes per parameter, lane q summing splits q, q + 4, ...; the four
  // sums are combined in a fixed order, so the result does not depend on timing
  const uint64_t span = c.n_params - c.w_off[0];
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t j = t >> 2;
  const int part = (int)(t & 3u);
  if (j >= span) return;  // the four lanes of a parameter leave together
  // inside a layer's block (not alignment padding)?
  const uint64_t abs_i = c.w_off[0] + j;
  bool inside = false;
  for (int k = 0; k <= c.hidden; ++k)
    if (abs_i >= c.w_off[k] && abs_i < c.w_off[k] + (uint64_t)c.fan_in[k] * c.fan_out[k]) inside = true;
  if (!inside) return;
  float s = 0.f;
  for (int p = part; p < nsplit; p += 4) s += wpart[(size_t)p * span + j];
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  if (part == 0) {
    if (!isfinite(s)) atomicOr(&state->nonfinite_pending, 1u);
    grad[abs_i] += s;
  }
}

// ---------------------------------------------------------------------------
// Table-gradient scatter. Global FP32 atomics cost one request per distinct
// cache line a wave instruction touches, so the scatter is organised to put
// many updates into few lines:
//  - coarse dense levels small enough for LDS are accumulated per workgroup
//    with LDS atomics and flushed once with fully coalesced global atomics;
//  - every other level uses 2F lanes per (probe, level): lane (dx, f) owns one
//    feature of one x-neighbour, so the 2F lanes of an x-pair update one
//    contiguous run (always on dense levels; when the cell's x is even on
//    hashed ones, since the spatial hash keeps x's low bit);
//  - consecutive samples of a ray that fall into the same cell are summed in
//    registers before the atomics are issued.
// Corner indices and weights are recomputed from the probes (nothing from the
// forward pass is stored).

// levels [0, n_lds) go through LDS; returns n_lds and their float count
static int coarse_lds_levels(const DevCfg& c, size_t budget_bytes, uint32_t* n_floats) {
  uint64_t acc = 0;
  int nl = 0;
  for (int l = 0; l < c.n_levels; ++l) {
    if (!((c.dense_mask >> l) & 1u)) break;
    const uint64_t r1 = (uint64_t)c.level_res[l] + 1;
    const uint64_t fl = r1 * r1 * r1 * c.n_features;
    if ((acc + fl) * 4 > budget_bytes) break;
    acc += fl;
    ++nl;
  }
  *n_floats = (uint32_t)acc;
  return nl;
}

template <int F>
__global__ __launch_bounds__(1024) void k_scatter_lds(DevCfg c, int n_lds, uint32_t n_floats,
                                                      const nbvh_probe* __restrict__ probes, uint32_t n,
                                                      const float* __restrict__ duT, uint64_t ldb,
                                                      float* __restrict__ grad) {
  extern __shared__ __align__(16) float acc[];
  for (uint32_t i = threadIdx.x; i < n_floats; i += blockDim.x) acc[i] = 0.0f;
  __syncthreads();
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint32_t p0 = blockIdx.x * chunk;
  const uint32_t p1 = min(n, p0 + chunk);
  const uint32_t np = p1 > p0 ? p1 - p0 : 0;
  const uint32_t tasks = np * c.n_samples * n_lds;
  for (uint32_t t = threadIdx.x; t < tasks; t += blockDim.x) {
    const uint32_t p = p0 + t % np;
    const uint32_t sl = t / np;
    const int s = sl / n_lds, l = sl - s * n_lds;
    float g[F];
    bool any = false;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      g[f] = duT[(size_t)((s * c.n_levels + l) * F + f) * ldb + p];
      any = any || g[f] != 0.0f;
    }
    if (!any) continue;
    const float4* pp = (const float4*)(probes + p);
    const float4 a = pp[0], b = pp[1];
    const float o[3] = {a.x, a.y, a.z}, d[3] = {b.x, b.y, b.z};
    float x[3];
    sample_position(c, o, d, a.w, b.w, s, x);
    uint32_t idx[8];
    float w[8];
    corners_level(c, l, x, idx, w);
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int f = 0; f < F; ++f) atomicAdd(&acc[idx[k] + f], w[k] * g[f]);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n_floats; i += blockDim.x) {
    const float v = acc[i];
    if (v != 0.0f) unsafeAtomicAdd(grad + i, v);  // levels [0, n_lds) start at parameter 0
  }
}

template <int F>
__global__ __launch_bounds__(256) void k_scatter_pairs(DevCfg c, int l_begin, const nbvh_probe* __restrict__ probes,
                                                       uint32_t n, const float* __restrict__ duT, uint64_t ldb,
                                                       float* __restrict__ grad) {
  constexpr int LPT = 2 * F;  // lanes per (probe, level)
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t task = gt / LPT;
  const int q = (int)(gt % LPT);
  const int dx = q / F, f = q - dx * F;
  const uint32_t nl = (uint32_t)(c.n_levels - l_begin);
  if (task >= (uint64_t)n * nl) return;
  const uint32_t li = (uint32_t)(task / n);
  const uint32_t p = (uint32_t)(task - (uint64_t)li * n);
  const int l = l_begin + (int)li;
  const int N = c.level_res[l];
  const bool dense = (c.dense_mask >> l) & 1u;
  const uint32_t mask = (1u << c.log2_T) - 1u;
  const uint32_t base = c.level_off[l];
  const float4* pp = (const float4*)(probes + p);
  const float4 a = pp[0], b = pp[1];
  const float o[3] = {a.x, a.y, a.z}, d[3] = {b.x, b.y, b.z};
  int ccx = -1, ccy = -1, ccz = -1;
  uint32_t idx[4] = {0u, 0u, 0u, 0u};
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int s = 0; s < c.n_samples; ++s) {
    const float g = duT[(size_t)((s * c.n_levels + l) * F + f) * ldb + p];
    float x[3];
    sample_position(c, o, d, a.w, b.w, s, x);
    int cx, cy, cz;
    float wx, wy, wz;
    cell_weight(x[0], N, cx, wx);
    cell_weight(x[1], N, cy, wy);
    cell_weight(x[2], N, cz, wz);
    if (cx != ccx || cy != ccy || cz != ccz) {
      if (ccx >= 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (acc[j] != 0.0f) unsafeAtomicAdd(grad + idx[j] + f, acc[j]);
      }
      ccx = cx;
      ccy = cy;
      ccz = cz;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        idx[j] = base + corner_index(dense, N, mask, (uint32_t)(cx + dx), (uint32_t)(cy + (j & 1)),
                                     (uint32_t)(cz + (j >> 1))) * F;
        acc[j] = 0.0f;
      }
    }
    const float wxs = dx ? wx : 1.0f - wx;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float w = (wxs * ((j & 1) ? wy : 1.0f - wy)) * ((j >> 1) ? wz : 1.0f - wz);
      acc[j] = __builtin_fmaf(w, g, acc[j]);
    }
  }
  if (ccx >= 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (acc[j] != 0.0f) unsafeAtomicAdd(grad + idx[j] + f, acc[j]);
  }
}

// ---------------------------------------------------------------------------
// Mid levels: a workgroup takes 256 consecutive probes (a leaf's probes are
// consecutive in a batch, so at these resolutions their corners repeat many
// times) and, one level at a time, sums their contributions in an LDS
// open-addressing table keyed by parameter index; the table is then flushed
// with one global atomic per distinct entry and feature. A record that finds
// no slot within kHashProbe steps goes straight to global memory.
// Fixed-point accumulation. On this hardware LDS float atomics run at a
// fraction of the rate of LDS integer atomics, so the scatter routes that sum
// in LDS add 64-bit integers: a contribution v becomes round(v * 2^e). With
// g = max |dL/du| over the batch, a contribution (a run of at most S samples
// times trilinear weights <= 1) is below S g, so n_terms of them stay below
// 2^62 when e = 62 - ceil(log2 n_terms) - ceil(log2 S) - E, g < 2^E. The
// rounding error is at most 2^-(e+1) per term, 2^-38 of g or less here.
// A non-finite g flags the step (the optimiser then skips it) and the
// route adds nothing.
__device__ inline int ceil_log2(uint32_t x) { return x <= 1u ? 0 : 32 - __clz(x - 1u); }

__device__ inline bool fixed_exponent(const uint32_t* gmax, uint32_t log2_terms, int S, DevState* state, int* e) {
  const float g = __uint_as_float(*gmax);
  if (!(g <= 3.0e38f)) {
    if (threadIdx.x == 0) atomicOr(&state->nonfinite_pending, 1u);
    return false;
  }
  int E = 0;
  if (g > 0.0f) (void)frexpf(g, &E);  // g < 2^E
  *e = 62 - (int)log2_terms - ceil_log2((uint32_t)S) - E;
  return true;
}

__device__ inline long long to_fixed(float v, int e) { return __float2ll_rn(ldexpf(v, e)); }
__device__ inline float from_fixed(long long q, int e) { return ldexpf((float)q, -e); }

constexpr int kHashTile = 256;
constexpr int kHashProbe = 16;
constexpr uint32_t kHashEmpty = 0xffffffffu;
template <int F>
struct HashSlots {
  static constexpr int log2n = F == 2 ? 12 : 11;  // 80 KiB of LDS either way
  static constexpr int n = 1 << log2n;
};

template <int F>
__global__ __launch_bounds__(kHashTile) void k_scatter_hash(DevCfg c, int l_begin, int l_end,
                                                            const nbvh_probe* __restrict__ probes, uint32_t n,
                                                            const float* __restrict__ duT, uint64_t ldb,
                                                            const uint32_t* __restrict__ gmax, DevState* state,
                                                            float* __restrict__ grad) {
  constexpr int NS = HashSlots<F>::n;
  __shared__ uint32_t keys[NS];
  __shared__ long long vals[NS * F];
  int e;
  // per entry: at most kHashTile probes x S runs
  if (!fixed_exponent(gmax, ceil_log2((uint32_t)(kHashTile * c.n_samples)), c.n_samples, state, &e)) return;
  for (int i = threadIdx.x; i < NS; i += kHashTile) {
    keys[i] = kHashEmpty;
#pragma unroll
    for (int f = 0; f < F; ++f) vals[i * F + f] = 0ll;
  }
  __syncthreads();
  const uint32_t p = blockIdx.x * kHashTile + threadIdx.x;
  // workgroups (tile, y) take levels l_begin + y, + gridDim.y, ...
  for (int l = l_begin + (int)blockIdx.y; l < l_end; l += (int)gridDim.y) {
    if (p < n) {
      level_runs<F>(c, l, probes, p, duT, ldb, [&](uint32_t idx, const float* v) {
        bool any = false;
#pragma unroll
        for (int f = 0; f < F; ++f) any = any || v[f] != 0.0f;
        if (!any) return;
        uint32_t h = ((idx / F) * 2654435761u) >> (32 - HashSlots<F>::log2n);
        for (int step = 0; step < kHashProbe; ++step) {
          const uint32_t k = atomicCAS(&keys[h], kHashEmpty, idx);
          if (k == kHashEmpty || k == idx) {
#pragma unroll
            for (int f = 0; f < F; ++f)
              atomicAdd((unsigned long long*)&vals[h * F + f], (unsigned long long)to_fixed(v[f], e));
            return;
          }
          h = (h + 1) & (NS - 1);
        }
#pragma unroll
        for (int f = 0; f < F; ++f) unsafeAtomicAdd(grad + idx + f, v[f]);
      });
    }
    __syncthreads();
    // flush and clear; lanes f of one entry update one contiguous run
    for (int i = threadIdx.x; i < NS * F; i += kHashTile) {
      const int slot = i / F, f = i - slot * F;
      const uint32_t k = keys[slot];
      if (k != kHashEmpty) {
        const long long q = vals[i];
        if (q != 0ll) unsafeAtomicAdd(grad + k + f, from_fixed(q, e));
        vals[i] = 0ll;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NS; i += kHashTile) keys[i] = kHashEmpty;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Binned scatter for the levels outside LDS: a counting sort of the
// contributions by 64 KiB table chunk, then one workgroup per chunk adds its
// records with LDS atomics and updates its chunk of the gradient with plain
// coalesced read-modify-writes (it is the chunk's only writer), so these
// levels need no global atomics at all.

// Walk the samples of probe p at level l, merging consecutive samples that
// fall into the same cell, and hand every (entry, F values) contribution to
// emit(param_index, vals).
template <int F, typename Emit>
__device__ inline void level_runs(const DevCfg& c, int l, const nbvh_probe* __restrict__ probes, uint32_t p,
                                  const float* __restrict__ duT, uint64_t ldb, Emit emit) {
  const int N = c.level_res[l];
  const bool dense = (c.dense_mask >> l) & 1u;
  const uint32_t mask = (1u << c.log2_T) - 1u;
  const uint32_t base = c.level_off[l];
  const float4* pp = (const float4*)(probes + p);
  const float4 a = pp[0], b = pp[1];
  const float o[3] = {a.x, a.y, a.z}, d[3] = {b.x, b.y, b.z};
  int ccx = -1, ccy = -1, ccz = -1;
  float acc[8][F];
  float wxs = 0.f, wys = 0.f, wzs = 0.f;
  (void)wxs;
  (void)wys;
  (void)wzs;
  for (int s = 0; s < c.n_samples; ++s) {
    float g[F];
#pragma unroll
    for (int f = 0; f < F; ++f) g[f] = duT[(size_t)((s * c.n_levels + l) * F + f) * ldb + p];
    float x[3];
    sample_position(c, o, d, a.w, b.w, s, x);
    int cx, cy, cz;
    float wx, wy, wz;
    cell_weight(x[0], N, cx, wx);
    cell_weight(x[1], N, cy, wy);
    cell_weight(x[2], N, cz, wz);
    if (cx != ccx || cy != ccy || cz != ccz) {
      if (ccx >= 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
          emit(base + corner_index(dense, N, mask, ccx + (k & 1), ccy + ((k >> 1) & 1), ccz + ((k >> 2) & 1)) * F,
               acc[k]);
      }
      ccx = cx;
      ccy = cy;
      ccz = cz;
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int f = 0; f < F; ++f) acc[k][f] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float w = ((k & 1) ? wx : 1.0f - wx) * (((k >> 1) & 1) ? wy : 1.0f - wy) * (((k >> 2) & 1) ? wz : 1.0f - wz);
#pragma unroll
      for (int f = 0; f < F; ++f) acc[k][f] = __builtin_fmaf(w, g[f], acc[k][f]);
    }
  }
  if (ccx >= 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      emit(base + corner_index(dense, N, mask, ccx + (k & 1), ccy + ((k >> 1) & 1), ccz + ((k >> 2) & 1)) * F, acc[k]);
  }
}

// Binned records of two-feature tables: 12 bytes (entry, two FP32 values), or
// for the reduced-precision paths 8 bytes: each value rounded to nearest even
// on its 16 upper mantissa bits (relative error at most 2^-16, far below the
// BF16 activations' and table's own rounding) and the 13-bit entry split over
// the two freed low bytes. A finite value is never rounded up to infinity.
__device__ inline uint32_t round_f24(float v) {
  const uint32_t b = __float_as_uint(v);
  uint32_t r = b + 0x7fu + ((b >> 8) & 1u);
  if ((r & 0x7f800000u) == 0x7f800000u) r = b;
  return r & 0xffffff00u;
}

template <bool R8>
struct BinRecord;
template <>
struct BinRecord<false> {
  typedef uint3 T;
  __device__ static T pack(uint32_t e, float v0, float v1) { return uint3{e, __float_as_uint(v0), __float_as_uint(v1)}; }
  __device__ static void unpack(const T& r, uint32_t& e, float& v0, float& v1) {
    e = r.x;
    v0 = __uint_as_float(r.y);
    v1 = __uint_as_float(r.z);
  }
  __device__ static T none() { return uint3{0xffffffffu, 0u, 0u}; }
};
template <>
struct BinRecord<true> {
  typedef uint2 T;
  __device__ static T pack(uint32_t e, float v0, float v1) {
    return uint2{round_f24(v0) | (e & 0xffu), round_f24(v1) | (e >> 8)};
  }
  __device__ static void unpack(const T& r, uint32_t& e, float& v0, float& v1) {
    e = (r.x == 0xffffffffu) ? 0xffffffffu : ((r.x & 0xffu) | ((r.y & 0xffu) << 8));
    v0 = __uint_as_float(r.x & 0xffffff00u);
    v1 = __uint_as_float(r.y & 0xffffff00u);
  }
  __device__ static T none() { return uint2{0xffffffffu, 0u}; }
};
static_assert(kBinChunk <= (1u << 13), "an 8-byte record holds a 13-bit entry");

struct BinArgs {
  int l_begin;        // first binned level
  uint32_t off0;      // its first parameter
  uint32_t n_bins;
  uint32_t n_tasks;   // probes x binned levels
  uint32_t per_wg;    // tasks per workgroup
};

// pass 1: per-workgroup histogram of record bins -> counts[bin][wg]
template <int F>
__global__ __launch_bounds__(256) void k_bin_count(DevCfg c, BinArgs A, const nbvh_probe* __restrict__ probes,
                                                   uint32_t n, const float* __restrict__ duT, uint64_t ldb,
                                                   uint32_t* __restrict__ counts) {
  extern __shared__ uint32_t hist[];
  for (uint32_t i = threadIdx.x; i < A.n_bins; i += blockDim.x) hist[i] = 0u;
  __syncthreads();
  const uint32_t t0 = blockIdx.x * A.per_wg, t1 = min(A.n_tasks, t0 + A.per_wg);
  for (uint32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const uint32_t li = t / n, p = t - li * n;
    level_runs<F>(c, A.l_begin + (int)li, probes, p, duT, ldb, [&](uint32_t idx, const float*) {
      atomicAdd(&hist[(idx - A.off0) / kBinChunk], 1u);
    });
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < A.n_bins; i += blockDim.x) counts[(size_t)i * gridDim.x + blockIdx.x] = hist[i];
}

// pass 2: write every record at its place: offsets = exclusive scan of counts
template <int F, bool R8>
__global__ __launch_bounds__(256) void k_bin_write(DevCfg c, BinArgs A, const nbvh_probe* __restrict__ probes,
                                                   uint32_t n, const float* __restrict__ duT, uint64_t ldb,
                                                   const uint32_t* __restrict__ offsets, uint16_t* __restrict__ rec_idx,
                                                   float* __restrict__ rec_val) {
  extern __shared__ uint32_t cursor[];
  for (uint32_t i = threadIdx.x; i < A.n_bins; i += blockDim.x) cursor[i] = offsets[(size_t)i * gridDim.x + blockIdx.x];
  __syncthreads();
  const uint32_t t0 = blockIdx.x * A.per_wg, t1 = min(A.n_tasks, t0 + A.per_wg);
  for (uint32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const uint32_t li = t / n, p = t - li * n;
    level_runs<F>(c, A.l_begin + (int)li, probes, p, duT, ldb, [&](uint32_t idx, const float* v) {
      const uint32_t rel = idx - A.off0;
      const uint32_t slot = atomicAdd(&cursor[rel / kBinChunk], 1u);
      if constexpr (F == 2) {
        // one record (entry, value pair): one store per contribution
        typedef BinRecord<R8> Rec;
        ((typename Rec::T*)rec_val)[slot] = Rec::pack(rel % kBinChunk, v[0], v[1]);
      } else {
        rec_idx[slot] = (uint16_t)(rel % kBinChunk);
#pragma unroll
        for (int f = 0; f < F; ++f) rec_val[(size_t)slot * F + f] = v[f];
      }
    });
  }
}

// pass 2 for two-feature tables with at most kStagedBins bins: the same
// records, grouped in LDS before they are stored. Each round every thread
// advances its task by one sample (as level_runs does) and holds the 0 or 8
// records that step closes; the round's records are counted per bin, placed in
// an LDS stage in bin order and then stored in that order, so that the lanes
// of a store instruction write runs of consecutive slots of one bin instead of
// 64 scattered records.
constexpr int kStagedBins = 1024;
constexpr int kStageCap = 256 * 8;

template <bool R8>
__global__ __launch_bounds__(256) void k_bin_write_staged(DevCfg c, BinArgs A, const nbvh_probe* __restrict__ probes,
                                                          uint32_t n, const float* __restrict__ duT, uint64_t ldb,
                                                          const uint32_t* __restrict__ offsets,
                                                          typename BinRecord<R8>::T* __restrict__ rec) {
  constexpr int F = 2;
  typedef BinRecord<R8> Rec;
  __shared__ uint32_t cursor[kStagedBins];  // next slot of each bin for this workgroup
  __shared__ uint32_t cnt[kStagedBins];     // the round's records per bin
  __shared__ uint32_t off[kStagedBins];     // their exclusive offsets in the stage
  __shared__ uint32_t sbase[kStagedBins];   // slot of the round's first record of each bin
  __shared__ typename Rec::T stage[kStageCap];
  __shared__ uint32_t slot_of[kStageCap];
  __shared__ uint32_t wtot[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (uint32_t i = tid; i < kStagedBins; i += 256) {
    cursor[i] = i < A.n_bins ? offsets[(size_t)i * gridDim.x + blockIdx.x] : 0u;
    cnt[i] = 0u;
  }
  __syncthreads();
  const uint32_t t0 = blockIdx.x * A.per_wg, t1 = min(A.n_tasks, t0 + A.per_wg);
  const uint32_t rounds_per_task = (uint32_t)c.n_samples + 1u;
  const uint32_t n_tasks_thread = t1 > t0 ? (t1 - t0 + 255u) / 256u : 0u;
  for (uint32_t j = 0; j < n_tasks_thread; ++j) {
    const uint32_t t = t0 + j * 256u + (uint32_t)tid;
    const bool have = t < t1;
    const uint32_t li = have ? t / n : 0u, p = have ? t - li * n : 0u;
    const int l = A.l_begin + (int)li;
    const int N = c.level_res[l];
    const bool dense = (c.dense_mask >> l) & 1u;
    const uint32_t mask = (1u << c.log2_T) - 1u;
    const uint32_t base = c.level_off[l];
    const float4* pp = (const float4*)(probes + p);
    const float4 a = pp[0], b = pp[1];
    const float o[3] = {a.x, a.y, a.z}, d[3] = {b.x, b.y, b.z};
    int ccx = -1, ccy = -1, ccz = -1;
    float acc[8][F];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k][0] = acc[k][1] = 0.0f;
    for (uint32_t s = 0; s < rounds_per_task; ++s) {
      // one step of the run walk: the records of the run this sample closes
      bool emit = false;
      uint32_t rel[8];
      float v0[8], v1[8];
      int cx = -1, cy = -1, cz = -1;
      float wx = 0.f, wy = 0.f, wz = 0.f, g0 = 0.f, g1 = 0.f;
      const bool last = s == (uint32_t)c.n_samples;
      if (have && !last) {
        g0 = duT[(size_t)((s * c.n_levels + l) * F + 0) * ldb + p];
        g1 = duT[(size_t)((s * c.n_levels + l) * F + 1) * ldb + p];
        float x[3];
        sample_position(c, o, d, a.w, b.w, (int)s, x);
        cell_weight(x[0], N, cx, wx);
        cell_weight(x[1], N, cy, wy);
        cell_weight(x[2], N, cz, wz);
      }
      if (have && ccx >= 0 && (last || cx != ccx || cy != ccy || cz != ccz)) {
        emit = true;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          rel[k] = base + corner_index(dense, N, mask, ccx + (k & 1), ccy + ((k >> 1) & 1), ccz + ((k >> 2) & 1)) * F -
                   A.off0;
          v0[k] = acc[k][0];
          v1[k] = acc[k][1];
        }
      }
      if (have && !last) {
        if (cx != ccx || cy != ccy || cz != ccz) {
          ccx = cx;
          ccy = cy;
          ccz = cz;
#pragma unroll
          for (int k = 0; k < 8; ++k) acc[k][0] = acc[k][1] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float w = ((k & 1) ? wx : 1.0f - wx) * (((k >> 1) & 1) ? wy : 1.0f - wy) *
                          (((k >> 2) & 1) ? wz : 1.0f - wz);
          acc[k][0] = __builtin_fmaf(w, g0, acc[k][0]);
          acc[k][1] = __builtin_fmaf(w, g1, acc[k][1]);
        }
      }
      // round: rank within bin, exclusive scan over bins, stage, store
      uint32_t rank[8];
      if (emit) {
#pragma unroll
        for (int k = 0; k < 8; ++k) rank[k] = atomicAdd(&cnt[rel[k] / kBinChunk], 1u);
      }
      __syncthreads();
      uint32_t c4[4], sum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c4[q] = cnt[4 * tid + q];
        sum += c4[q];
      }
      uint32_t incl = sum;  // inclusive scan of the per-thread sums within the wave
#pragma unroll
      for (int dd = 1; dd < 64; dd <<= 1) {
        const uint32_t y = __shfl_up(incl, dd);
        if (lane >= dd) incl += y;
      }
      if (lane == 63) wtot[wave] = incl;
      __syncthreads();
      uint32_t before = incl - sum;
      for (int w2 = 0; w2 < wave; ++w2) before += wtot[w2];
      const uint32_t total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int bi = 4 * tid + q;
        off[bi] = before;
        sbase[bi] = cursor[bi];
        cursor[bi] += c4[q];
        cnt[bi] = 0u;
        before += c4[q];
      }
      __syncthreads();
      if (emit) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t bin = rel[k] / kBinChunk;
          const uint32_t i = off[bin] + rank[k];
          stage[i] = Rec::pack(rel[k] % kBinChunk, v0[k], v1[k]);
          slot_of[i] = sbase[bin] + rank[k];
        }
      }
      __syncthreads();
      for (uint32_t i = tid; i < total; i += 256) rec[slot_of[i]] = stage[i];
      __syncthreads();
    }
  }
}

// pass 3: one workgroup per bin accumulates in LDS (64-bit fixed point) and
// updates its chunk with plain read-modify-writes
template <int F, bool R8>
__global__ __launch_bounds__(1024) void k_bin_reduce(BinArgs A, const uint32_t* __restrict__ offsets, uint32_t n_wgs,
                                                     const uint16_t* __restrict__ rec_idx,
                                                     const float* __restrict__ rec_val, uint64_t n_table,
                                                     const uint32_t* __restrict__ gmax, uint32_t log2_terms, int S,
                                                     DevState* state, float* __restrict__ grad) {
  __shared__ long long acc[kBinChunk];
  int e;
  if (!fixed_exponent(gmax, log2_terms, S, state, &e)) return;
  const uint32_t bin = blockIdx.x;
  for (uint32_t i = threadIdx.x; i < kBinChunk; i += blockDim.x) acc[i] = 0ll;
  __syncthreads();
  const uint32_t r0 = offsets[(size_t)bin * n_wgs];
  const uint32_t r1 = offsets[(size_t)(bin + 1) * n_wgs];  // offsets[n_bins * n_wgs] is the total
  // kUnroll records per thread in flight before their LDS atomics
  constexpr int kUnroll = 4;
  for (uint32_t r = r0 + threadIdx.x; r < r1; r += blockDim.x * kUnroll) {
    uint32_t ix[kUnroll];
    float v[kUnroll][F];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint32_t rr = r + u * blockDim.x;
      const bool ok = rr < r1;
      if constexpr (F == 2) {
        typedef BinRecord<R8> Rec;
        const typename Rec::T rec = ok ? ((const typename Rec::T*)rec_val)[rr] : Rec::none();
        Rec::unpack(rec, ix[u], v[u][0], v[u][1]);
      } else {
        ix[u] = ok ? (uint32_t)rec_idx[rr] : 0xffffffffu;
#pragma unroll
        for (int f = 0; f < F; ++f) v[u][f] = ok ? rec_val[(size_t)rr * F + f] : 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (ix[u] != 0xffffffffu) {
#pragma unroll
        for (int f = 0; f < F; ++f)
          atomicAdd((unsigned long long*)&acc[ix[u] + f], (unsigned long long)to_fixed(v[u][f], e));
      }
    }
  }
  __syncthreads();
  const uint64_t g0 = (uint64_t)A.off0 + (uint64_t)bin * kBinChunk;
  const uint32_t len = (uint32_t)min((uint64_t)kBinChunk, n_table - g0);
  for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
    const long long q = acc[i];
    if (q != 0ll) grad[g0 + i] += from_fixed(q, e);
  }
}

// The hash-route levels [n_lds, hash_end) of the table gradient, on stream s
// (they write only their own levels' entries, so they may run beside the
// other routes).
template <int F>
static void launch_scatter_hash(const LaunchCtx& L, const TrainLayout& T, const nbvh_probe* probes, uint32_t n,
                                const float* duT, uint64_t ldb, const uint32_t* gmax, hipStream_t s) {
  if (T.hash_end <= T.n_lds) return;
  ProfScope ps(L.prof, NBVH_K_SCATTER, s);
  // small batches: one workgroup per (tile, level), so that the chip fills
  const uint32_t tiles = (n + kHashTile - 1) / kHashTile;
  const uint32_t split = tiles < 4u * (uint32_t)L.n_cu ? (uint32_t)(T.hash_end - T.n_lds) : 1u;
  k_scatter_hash<F><<<dim3(tiles, split), kHashTile, 0, s>>>(L.cfg, T.n_lds, T.hash_end, probes, n, duT, ldb, gmax,
                                                             L.state, L.grad);
}

// The other levels of the table gradient: [0, n_lds) held in LDS and
// [hash_end, L) binned or by pairs, on the context's stream.
template <int F>
static nbvh_status launch_scatter(const LaunchCtx& L, const TrainLayout& T, char* w, const nbvh_probe* probes,
                                  uint32_t n, const float* duT, uint64_t ldb, const uint32_t* gmax) {
  const DevCfg& c = L.cfg;
  {
    ProfScope ps(L.prof, NBVH_K_SCATTER, L.stream);
    if (T.n_lds > 0) {
      const size_t lds = (size_t)T.lds_floats * 4;
      (void)hipFuncSetAttribute((const void*)k_scatter_lds<F>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      k_scatter_lds<F><<<L.n_cu, 1024, lds, L.stream>>>(c, T.n_lds, T.lds_floats, probes, n, duT, ldb, L.grad);
    }
    if (T.hash_end >= c.n_levels) return check_launch("scatter");
    if (T.n_bins == 0) {
      const uint64_t threads = (uint64_t)n * (c.n_levels - T.hash_end) * 2 * F;
      k_scatter_pairs<F><<<(uint32_t)((threads + 255) / 256), 256, 0, L.stream>>>(c, T.hash_end, probes, n, duT,
                                                                                 ldb, L.grad);
      return check_launch("scatter");
    }
  }
  BinArgs A;
  A.l_begin = T.hash_end;
  A.off0 = c.level_off[T.hash_end];
  A.n_bins = T.n_bins;
  A.n_tasks = n * (uint32_t)(c.n_levels - T.hash_end);
  A.per_wg = (A.n_tasks + kBinWgs - 1) / kBinWgs;
  uint32_t* counts = (uint32_t*)(w + T.counts);
  uint32_t* offsets = (uint32_t*)(w + T.offsets);
  uint32_t* sums = (uint32_t*)(w + T.scan_sums);
  const size_t hist_lds = (size_t)T.n_bins * 4;
  if (hist_lds > 64 * 1024) return set_error("too many gradient bins (%u) for LDS", T.n_bins), NBVH_ERR_UNSUPPORTED;
  {
    ProfScope ps(L.prof, NBVH_K_SCATTER_SORT, L.stream);
    k_bin_count<F><<<kBinWgs, 256, hist_lds, L.stream>>>(c, A, probes, n, duT, ldb, counts);
    const uint32_t cells = T.n_bins * (uint32_t)kBinWgs;
    nbvh_status s = launch_exclusive_scan(L.stream, counts, cells, offsets, sums, sums + cells / 1024 + 3);
    if (s != NBVH_OK) return s;
    if (F == 2 && T.n_bins <= (uint32_t)kStagedBins) {
      if (T.rec8)
        k_bin_write_staged<true><<<kBinWgs, 256, 0, L.stream>>>(c, A, probes, n, duT, ldb, offsets,
                                                                (uint2*)(w + T.rec_val));
      else
        k_bin_write_staged<false><<<kBinWgs, 256, 0, L.stream>>>(c, A, probes, n, duT, ldb, offsets,
                                                                 (uint3*)(w + T.rec_val));
    } else if (F == 2 && T.rec8) {
      k_bin_write<F, true><<<kBinWgs, 256, hist_lds, L.stream>>>(c, A, probes, n, duT, ldb, offsets,
                                                                (uint16_t*)(w + T.rec_idx), (float*)(w + T.rec_val));
    } else {
      k_bin_write<F, false><<<kBinWgs, 256, hist_lds, L.stream>>>(c, A, probes, n, duT, ldb, offsets,
                                                                 (uint16_t*)(w + T.rec_idx), (float*)(w + T.rec_val));
    }
  }
  {
    ProfScope ps(L.prof, NBVH_K_SCATTER_REDUCE, L.stream);
    // per entry: at most n probes x S runs
    const uint32_t log2_terms = (uint32_t)(32 - __builtin_clz(n * (uint32_t)c.n_samples - 1u));
    if (F == 2 && T.rec8)
      k_bin_reduce<F, true><<<T.n_bins, 1024, 0, L.stream>>>(A, offsets, kBinWgs, (const uint16_t*)(w + T.rec_idx),
                                                             (const float*)(w + T.rec_val), c.n_table, gmax,
                                                             log2_terms, c.n_samples, L.state, L.grad);
    else
      k_bin_reduce<F, false><<<T.n_bins, 1024, 0, L.stream>>>(A, offsets, kBinWgs, (const uint16_t*)(w + T.rec_idx),
                                                              (const float*)(w + T.rec_val), c.n_table, gmax,
                                                              log2_terms, c.n_samples, L.state, L.grad);
  }
  return check_launch("scatter");
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loss_finalize(const float* __restrict__ part, uint32_t n_tiles, uint32_t n,
                                                       float w_hit, float w_t, float w_normal, float w_albedo,
                                                       float* __restrict__ out,
                                                       DevState* __restrict__ state) {
  __shared__ float sh[4][256];
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  for (uint32_t i = threadIdx.x; i < n_tiles; i += blockDim.x) {
    s0 += part[i * 4 + 0];
    s1 += part[i * 4 + 1];
    s2 += part[i * 4 + 2];
    s3 += part[i * 4 + 3];
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  sh[2][threadIdx.x] = s2;
  sh[3][threadIdx.x] = s3;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float inv = 1.0f / (float)n;
    const float b = sh[0][0] * inv, t = sh[1][0] * inv, nn = sh[2][0] * inv;
    const float tot = w_hit * b + w_t * t + w_normal * nn + w_albedo * sh[3][0] * inv;
    if (!isfinite(tot)) atomicOr(&state->nonfinite_pending, 1u);
    state->last_loss[0] = tot;
    state->last_loss[1] = b;
    state->last_loss[2] = t;
    state->last_loss[3] = nn;
    if (out) {
      out[0] = tot;
      out[1] = b;
      out[2] = t;
      out[3] = nn;
    }
  }
}

// plain loss / dz kernel (nbvh_loss): thread per probe, partial sums per block
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ z, const nbvh_label* __restrict__ labels,
                                              uint32_t n, int n_out, float w_hit, float w_t, float w_normal, float w_albedo,
                                              float* __restrict__ dz, float* __restrict__ part) {
  __shared__ float sh[4][256];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  float lb_ = 0.f, lt = 0.f, ln = 0.f, la = 0.f;
  float da[3] = {0.f, 0.f, 0.f};
  if (i < n) {
    const float* zr = z + (size_t)i * n_out;
    const nbvh_label lb = labels[i];
    const float h = lb.hit, tau = lb.tau, st = sigmoidf_(zr[1]);
    lb_ = bce_logits(zr[0], h);
    lt = h * fabsf(st - tau);
    float s = 0.f;
    for (int a = 0; a < 3; ++a) s += fabsf(zr[2 + a] - lb.n[a]);
    ln = h * s * (1.0f / 3.0f);
    if (n_out >= 8) la = h * albedo_term(zr, lb.albedo, da);
    if (dz) {
      const float invB = 1.0f / (float)n;
      float* g = dz + (size_t)i * n_out;
      for (int o = 0; o < n_out; ++o) g[o] = 0.f;
      g[0] = w_hit * (sigmoidf_(zr[0]) - h) * invB;
      g[1] = h * w_t * sgnf(st - tau) * st * (1.0f - st) * invB;
      for (int a = 0; a < 3; ++a) g[2 + a] = h * w_normal * sgnf(zr[2 + a] - lb.n[a]) * (1.0f / 3.0f) * invB;
      if (n_out >= 8)
        for (int ch = 0; ch < 3; ++ch) g[5 + ch] = h * w_albedo * da[ch] * invB;
    }
  }
  sh[0][threadIdx.x] = lb_;
  sh[1][threadIdx.x] = lt;
  sh[2][threadIdx.x] = ln;
  sh[3][threadIdx.x] = la;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 0] = sh[0][0];
    part[blockIdx.x * 4 + 1] = sh[1][0];
    part[blockIdx.x * 4 + 2] = sh[2][0];
    part[blockIdx.x * 4 + 3] = sh[3][0];
  }
}

// Per-leaf sums of the segment loss (Sec. 5.1, "Node error": a node's
// training loss q): the combined loss of each segment, unscaled and with the
// loss weights, added to leaf_loss[leaf] with one count in leaf_count[leaf].
__global__ __launch_bounds__(256) void k_leaf_loss(const float* __restrict__ z, const nbvh_label* __restrict__ labels,
                                                   const uint32_t* __restrict__ leaf_ids, uint32_t n, int n_out,
                                                   float w_hit, float w_t, float w_normal, float w_albedo,
                                                   float* __restrict__ leaf_loss, uint32_t* __restrict__ leaf_count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* zr = z + (size_t)i * n_out;
  const nbvh_label lb = labels[i];
  const float h = lb.hit, st = sigmoidf_(zr[1]);
  float s = 0.f;
  for (int a = 0; a < 3; ++a) s += fabsf(zr[2 + a] - lb.n[a]);
  float loss = w_hit * bce_logits(zr[0], h) + w_t * h * fabsf(st - lb.tau) + w_normal * h * s * (1.0f / 3.0f);
  if (n_out >= 8) {
    float da[3];
    loss += w_albedo * h * albedo_term(zr, lb.albedo, da);
  }
  const uint32_t leaf = leaf_ids[i];
  atomicAdd(&leaf_loss[leaf], loss);
  atomicAdd(&leaf_count[leaf], 1u);
}

nbvh_status launch_leaf_loss(const LaunchCtx& L, const nbvh_probe* probes, const nbvh_label* labels,
                             const uint32_t* leaf_ids, uint32_t n, float* z, float* leaf_loss, uint32_t* leaf_count) {
  if (n == 0) return NBVH_OK;
  nbvh_status s = launch_forward(L, probes, n, z);
  if (s != NBVH_OK) return s;
  k_leaf_loss<<<(n + 255) / 256, 256, 0, L.stream>>>(z, labels, leaf_ids, n, L.cfg.n_out, L.w_hit, L.w_t, L.w_normal,
                                                     L.w_albedo, leaf_loss, leaf_count);
  return check_launch("leaf_loss");
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_check_finite(const float* __restrict__ g, uint64_t n,
                                                      DevState* __restrict__ state) {
  bool bad = false;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = tid; j < n / 4; j += stride) {
    const float4 x = ((const float4*)g)[j];
    bad = bad || !isfinite(x.x) || !isfinite(x.y) || !isfinite(x.z) || !isfinite(x.w);
  }
  for (uint64_t i = (n / 4) * 4 + tid; i < n; i += stride) bad = bad || !isfinite(g[i]);
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&state->nonfinite_pending, 1u);
}

// transposed copies of the MLP weights: W_k^T [fan_in][fan_out_pad]
__device__ inline void write_transposed(const DevCfg& c, uint64_t i, float v, float* aux32, uint16_t* aux16) {
  if (i < c.w_off[0]) return;
  for (int k = 0; k <= c.hidden; ++k) {
    const uint64_t sz = (uint64_t)c.fan_in[k] * c.fan_out[k];
    if (i >= c.w_off[k] && i < c.w_off[k] + sz) {
      const uint64_t j = i - c.w_off[k];
      const uint32_t o = (uint32_t)(j / c.fan_in[k]), ii = (uint32_t)(j - (uint64_t)o * c.fan_in[k]);
      const uint64_t dst = c.wt_off[k] + (uint64_t)ii * fan_out_pad(c, k) + o;
      aux32[dst] = v;
      aux16[dst] = f32_to_bf16_bits(v);
      return;
    }
  }
}

// mode 0: Adam step; mode 1: shadow + transposed copies only
__global__ __launch_bounds__(256) void k_adam(DevCfg c, float* __restrict__ params, uint16_t* __restrict__ lp,
                                              float* __restrict__ m, float* __restrict__ v, float* __restrict__ grad,
                                              float* __restrict__ aux32, uint16_t* __restrict__ aux16,
                                              const DevState* __restrict__ state, float lr, float beta1, float beta2,
                                              float eps, int mode) {
  const bool skip = mode == 1 || state->nonfinite_pending != 0;
  const float step = (float)(state->step + 1);
  const float inv_scale = 1.0f / state->loss_scale;
  const float c1 = 1.0f - powf(beta1, step), c2 = 1.0f - powf(beta2, step);
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
  // the hash table (and its padding up to the first weight): four parameters
  // per thread with 16-byte loads and stores (w_off[0] is a multiple of 64)
  const uint64_t n4 = c.w_off[0] / 4;
  for (uint64_t j = tid; j < n4; j += stride) {
    float4 p = ((const float4*)params)[j];
    if (mode == 0) {
      const float4 g = ((const float4*)grad)[j];
      ((float4*)grad)[j] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (!skip) {
        float4 mi = ((const float4*)m)[j], vi = ((const float4*)v)[j];
        float* pp = (float*)&p;
        float* mm = (float*)&mi;
        float* vv = (float*)&vi;
        const float* gg = (const float*)&g;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float gs = gg[e] * inv_scale;
          mm[e] = beta1 * mm[e] + (1.0f - beta1) * gs;
          vv[e] = beta2 * vv[e] + (1.0f - beta2) * gs * gs;
          const float mh = mm[e] / c1, vh = vv[e] / c2;
          pp[e] -= lr * mh / (sqrtf(vh) + eps);
        }
        ((float4*)m)[j] = mi;
        ((float4*)v)[j] = vi;
        ((float4*)params)[j] = p;
      }
    }
    if (lp)
      ((uint2*)lp)[j] = uint2{(uint32_t)f32_to_bf16_bits(p.x) | ((uint32_t)f32_to_bf16_bits(p.y) << 16),
                              (uint32_t)f32_to_bf16_bits(p.z) | ((uint32_t)f32_to_bf16_bits(p.w) << 16)};
  }
  // the MLP weights: one parameter per thread, with their transposed copies
  for (uint64_t i = 4 * n4 + tid; i < c.n_params; i += stride) {
    float p = params[i];
    if (mode == 0) {
      const float g = grad[i];
      grad[i] = 0.0f;
      if (!skip) {
        const float gs = g * inv_scale;
        const float mi = beta1 * m[i] + (1.0f - beta1) * gs;
        const float vi = beta2 * v[i] + (1.0f - beta2) * gs * gs;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / c1, vh = vi / c2;
        p -= lr * mh / (sqrtf(vh) + eps);
        params[i] = p;
      }
    }
    if (lp) lp[i] = f32_to_bf16_bits(p);
    write_transposed(c, i, p, aux32, aux16);
  }
}

__global__ void k_adam_finalize(DevState* state, int mode) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (mode == 0) {
      if (state->nonfinite_pending) {
        state->skipped += 1;
        state->loss_scale *= 0.5f;
        state->flags |= NBVH_FLAG_NONFINITE;
      } else {
        state->step += 1;
      }
    }
    state->nonfinite_pending = 0u;
  }
}

__global__ void k_reset_state(DevState* state, float loss_scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    state->step = 0;
    state->skipped = 0;
    state->loss_scale = loss_scale;
    state->flags = 0u;
    for (int i = 0; i < 4; ++i) state->last_loss[i] = 0.f;
    state->last_n_segments = 0;
    state->nonfinite_pending = 0u;
    state->n_evaluated = 0ull;
  }
}

// ---------------------------------------------------------------------------
template <typename K>
static void set_lds(K kernel, size_t bytes) {
  (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static WSlices make_slices(const DevCfg& c) {
  WSlices S;
  S.n = 0;
  for (int k = 0; k <= c.hidden; ++k)
    for (int i0 = 0; i0 < c.fan_in[k]; i0 += kWgCols) {
      S.layer[S.n] = (int16_t)k;
      S.i0[S.n] = (int16_t)i0;
      ++S.n;
    }
  return S;
}

static WTiles make_tiles(const DevCfg& c) {
  WTiles T;
  T.n = 0;
  for (int k = 0; k <= c.hidden; ++k)
    for (int o0 = 0; o0 < fan_out_pad(c, k); o0 += 64)
      for (int i0 = 0; i0 < c.fan_in[k]; i0 += 64) T.t[T.n++] = WTile{(int16_t)k, (int16_t)o0, (int16_t)i0, 0};
  return T;
}

template <typename AT, int F, bool LP>
static nbvh_status train_t(const LaunchCtx& L, const nbvh_probe* probes, const nbvh_label* labels, const float* dz_in,
                           uint32_t n, float* loss_dev, void* ws, size_t ws_bytes) {
  const DevCfg& c = L.cfg;
  const TrainLayout T = train_layout(c, L.precision, n, L.tune);
  // the binned gradient pass counts, scans and places its records with 32-bit
  // indices
  if (T.max_records > 0xffffffffull) {
    set_error("batch of %u probes needs %llu gradient records, more than 2^32: split the batch", n,
              (unsigned long long)T.max_records);
    return NBVH_ERR_UNSUPPORTED;
  }
  if (ws_bytes < T.total) {
    set_error("workspace too small for a batch of %u: need %zu bytes, got %zu", n, T.total, ws_bytes);
    return NBVH_ERR_CAPACITY;
  }
  char* w = (char*)ws;
  TrainPtrs P;
  for (int k = 0; k <= c.hidden; ++k) {
    P.hT[k] = w + T.hT[k];
    P.gT[k] = w + T.gT[k];
  }
  P.duT = (float*)(w + T.duT);
  P.loss_part = (float*)(w + T.loss_part);
  P.gmax = (uint32_t*)(w + T.gmax);
  const uint32_t kb = T.n_tiles * kTM;  // padded batch
  P.ldb = kb;
  const AT* W = (sizeof(AT) == 2) ? (const AT*)L.params_lp : (const AT*)L.params;
  const AT* WT = (sizeof(AT) == 2) ? (const AT*)((char*)L.aux + c.n_wt * 4) : (const AT*)L.aux;
  const void* table = LP ? (const void*)L.params_lp : (const void*)L.params;
  const size_t lds = train_lds_bytes<AT>(c);
  if (lds > 160 * 1024) {
    set_error("training tile needs %zu bytes of LDS (> 160 KiB) for this network", lds);
    return NBVH_ERR_UNSUPPORTED;
  }
  {
    ProfScope ps(L.prof, NBVH_K_TRAIN_TILE, L.stream);
    k_zero_u32<<<1, 64, 0, L.stream>>>(P.gmax, 1);
    const int nw = L.tune.train_waves == 4 ? 4 : 8;
#define NBVH_TT(LAB, NW)                                                                                  \
  do {                                                                                                    \
    auto kern = k_train_tile<AT, F, LP, LAB, NW>;                                                         \
    set_lds(kern, lds);                                                                                   \
    kern<<<T.n_tiles, 64 * NW, lds, L.stream>>>(c, table, W, WT, probes, labels, dz_in, n, P, L.state, L.w_hit, \
                                               L.w_t, L.w_normal, L.w_albedo);                           \
  } while (0)
    if (labels) {
      if (nw == 4) NBVH_TT(true, 4);
      else NBVH_TT(true, 8);
    } else {
      if (nw == 4) NBVH_TT(false, 4);
      else NBVH_TT(false, 8);
    }
#undef NBVH_TT
  }
  // The weight gradients (loss, thin GEMMs over the batch, fixed-order split
  // reduction: HBM streaming and matrix cores) and the table gradient (LDS
  // atomics and scattered record stores) depend only on the tile's outputs and
  // write disjoint parts of the gradient, and so do the table gradient's hash
  // route and its other routes; the hash route and then the weight gradients
  // run on the context's second stream beside the other routes, and the step
  // joins both before returning. Not while the caller's stream is being
  // captured into a graph: there the step stays on that one stream.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(L.stream, &cap) != hipSuccess) cap = hipStreamCaptureStatusActive;
  const bool fork = L.side && L.ev_fork && L.ev_join && cap == hipStreamCaptureStatusNone;
  hipStream_t gs = L.stream;
  if (fork) {
    if (hipEventRecord(L.ev_fork, L.stream) != hipSuccess || hipStreamWaitEvent(L.side, L.ev_fork, 0) != hipSuccess)
      return set_error("forking the weight-gradient stream failed"), NBVH_ERR_HIP;
    gs = L.side;
  }
  launch_scatter_hash<F>(L, T, probes, n, P.duT, kb, P.gmax, gs);
  {
    ProfScope ps(L.prof, NBVH_K_WGRAD, gs);
    if (labels)
      k_loss_finalize<<<1, 256, 0, gs>>>(P.loss_part, T.n_tiles, n, L.w_hit, L.w_t, L.w_normal, L.w_albedo, loss_dev,
                                         L.state);
    float* wpart = (float*)(w + T.wpart);
    if constexpr (sizeof(AT) == 2) {
      const WSlices slices = make_slices(c);
      k_wgrad_rows<<<dim3(slices.n, T.nsplit), 512, 0, gs>>>(c, slices, P, kb, T.nsplit, wpart);
    } else {
      const WTiles tiles = make_tiles(c);
      k_wgrad<AT><<<dim3(tiles.n, T.nsplit), 256, 0, gs>>>(c, tiles, P, kb, T.nsplit, wpart);
    }
    const uint64_t span = c.n_params - c.w_off[0];
    k_wgrad_reduce<<<(uint32_t)((4 * span + 255) / 256), 256, 0, gs>>>(c, wpart, T.nsplit, L.grad, L.state);
  }
  nbvh_status s = launch_scatter<F>(L, T, w, probes, n, P.duT, kb, P.gmax);
  if (fork && (hipEventRecord(L.ev_join, L.side) != hipSuccess || hipStreamWaitEvent(L.stream, L.ev_join, 0) != hipSuccess))
    return set_error("joining the weight-gradient stream failed"), NBVH_ERR_HIP;
  if (s != NBVH_OK) return s;
  return check_launch("train");
}

nbvh_status launch_train_fwd_bwd(const LaunchCtx& L, const nbvh_probe* probes, const nbvh_label* labels,
                                 const float* dz_in, uint32_t n, float* loss_dev, void* ws, size_t ws_bytes,
                                 bool apply_grad) {
  (void)apply_grad;
  if (n == 0) return NBVH_OK;
  const int F = L.cfg.n_features;
  if (L.precision == NBVH_FP32)
    return F == 2 ? train_t<float, 2, false>(L, probes, labels, dz_in, n, loss_dev, ws, ws_bytes)
                  : train_t<float, 4, false>(L, probes, labels, dz_in, n, loss_dev, ws, ws_bytes);
  return F == 2 ? train_t<bf16, 2, true>(L, probes, labels, dz_in, n, loss_dev, ws, ws_bytes)
                : train_t<bf16, 4, true>(L, probes, labels, dz_in, n, loss_dev, ws, ws_bytes);
}

nbvh_status launch_loss(const LaunchCtx& L, const float* z, const nbvh_label* labels, uint32_t n, float* loss_dev,
                        float* dz, void* ws, size_t ws_bytes) {
  const uint32_t nb = (n + 255) / 256;
  if (ws_bytes < (size_t)nb * 16) {
    set_error("workspace too small for nbvh_loss");
    return NBVH_ERR_CAPACITY;
  }
  if (n == 0) return NBVH_OK;
  float* part = (float*)ws;
  k_loss<<<nb, 256, 0, L.stream>>>(z, labels, n, L.cfg.n_out, L.w_hit, L.w_t, L.w_normal, L.w_albedo, dz, part);
  k_loss_finalize<<<1, 256, 0, L.stream>>>(part, nb, n, L.w_hit, L.w_t, L.w_normal, L.w_albedo, loss_dev, L.state);
  return check_launch("loss");
}

// Node error rank of each leaf (Sec. 5.1): r = 2 log q + log p with q the
// mean training loss of its first-hit segments and p the fraction of the
// sampled rays crossing it; -inf without segments, crossings or loss.
__global__ __launch_bounds__(256) void k_node_rank(const float* __restrict__ loss, const uint32_t* __restrict__ count,
                                                  const uint32_t* __restrict__ hits, uint32_t n, float inv_rays,
                                                  float* __restrict__ rank) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = count[i], h = hits[i];
  float r = -INFINITY;
  if (c > 0u && h > 0u && inv_rays > 0.0f) {
    const float q = loss[i] / (float)c;
    const float p = (float)h * inv_rays;
    if (q > 0.0f) r = 2.0f * logf(q) + logf(p);
  }
  rank[i] = r;
}

// Acceptance of each leaf's first-hit training rays (Sec. 5.2, read in
// linear space): max(exp(r - r_max), floor); floor for r = -inf; 1 when no
// rank is finite. One workgroup: the maximum is a block reduction.
__global__ __launch_bounds__(1024) void k_acceptance(const float* __restrict__ rank, uint32_t n, float floor_,
                                                    float* __restrict__ accept) {
  __shared__ float red[16];
  float m = -INFINITY;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float r = rank[i];
    if (r > m && r < INFINITY) m = r;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x < 64) {
    float v = threadIdx.x < (blockDim.x >> 6) ? red[threadIdx.x] : -INFINITY;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    if (threadIdx.x == 0) red[0] = v;
  }
  __syncthreads();
  const float rmax = red[0];
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float r = rank[i];
    float a = 1.0f;
    if (rmax > -INFINITY) {
      const float e = (r > -INFINITY) ? expf(r - rmax) : 0.0f;
      a = e > floor_ ? e : floor_;
    }
    accept[i] = a;
  }
}

nbvh_status launch_node_rank(hipStream_t s, const float* loss, const uint32_t* count, const uint32_t* hits, uint32_t n,
                             uint64_t n_rays, float* rank) {
  if (n) k_node_rank<<<(n + 255) / 256, 256, 0, s>>>(loss, count, hits, n, n_rays ? 1.0f / (float)n_rays : 0.0f, rank);
  return check_launch("node_rank");
}

nbvh_status launch_acceptance(hipStream_t s, const float* rank, uint32_t n, float floor_, float* accept) {
  if (n) k_acceptance<<<1, 1024, 0, s>>>(rank, n, floor_, accept);
  return check_launch("acceptance");
}

// dL/dparams without the loss scale: out = grad / state.loss_scale (the
// scale the last backward multiplied in), grad cleared when asked.
__global__ __launch_bounds__(256) void k_unscale_grad(float* __restrict__ grad, uint64_t n, const DevState* state,
                                                     float* __restrict__ out, int clear) {
  const float inv = 1.0f / state->loss_scale;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const float g = grad[i];
    if (clear) grad[i] = 0.0f;
    out[i] = g * inv;
  }
}

nbvh_status launch_unscale_grad(const LaunchCtx& L, float* out, bool clear) {
  const uint64_t n = L.cfg.n_params;
  const uint64_t want = (n + 255) / 256;
  const uint32_t grid = (uint32_t)(want < 1 ? 1 : (want > 65536 ? 65536 : want));
  k_unscale_grad<<<grid, 256, 0, L.stream>>>(L.grad, n, L.state, out, clear ? 1 : 0);
  return check_launch("unscale_grad");
}

nbvh_status launch_optimizer(const LaunchCtx& L, bool reset, bool shadow_only) {
  const DevCfg& c = L.cfg;
  float* aux32 = (float*)L.aux;
  uint16_t* aux16 = (uint16_t*)((char*)L.aux + c.n_wt * 4);
  // a thread per four parameters (the table is updated in 16-byte vectors),
  // so every thread's loads are in flight at once
  const uint64_t want = (c.n_params / 4 + 255) / 256;
  const uint32_t grid = (uint32_t)(want < 1 ? 1 : (want > (1u << 18) ? (1u << 18) : want));
  ProfScope ps(L.prof, NBVH_K_OPTIMIZER, L.stream);
  if (reset) {
    k_reset_state<<<1, 64, 0, L.stream>>>(L.state, L.loss_scale);
  }
  if (!shadow_only) {
    k_check_finite<<<grid, 256, 0, L.stream>>>(L.grad, c.n_params, L.state);
  }
  k_adam<<<grid, 256, 0, L.stream>>>(c, L.params, (uint16_t*)L.params_lp, L.adam_m, L.adam_v, L.grad, aux32, aux16,
                                     L.state, L.lr, L.beta1, L.beta2, L.eps, shadow_only ? 1 : 0);
  k_adam_finalize<<<1, 64, 0, L.stream>>>(L.state, shadow_only ? 1 : 0);
  return check_launch("optimizer");
}

}  // namespace nbvh
