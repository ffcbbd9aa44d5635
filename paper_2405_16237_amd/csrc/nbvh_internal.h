// Internal definitions of the gfx950 N-BVH library (device config, MFMA
// fragment types, sampling + hash-grid interpolation device code).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nbvh.h"

namespace nbvh {

constexpr int kMaxLayers = 9;   // mlp_hidden <= 8, plus the output layer
constexpr int kOutPad = 16;     // output layer rows padded to one MFMA tile
constexpr int kWave = 64;
constexpr int kAlign = 64;      // parameter blocks start on 64-element boundaries

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Node of the neural BVH: the boxes of both children live in the parent, so
// one visit tests two children (64 bytes, 4 x 16-byte loads). A child index
// >= 0 is an inner node, < 0 is leaf ~index, kEmptyChild marks a missing
// second child (single-leaf trees).
struct alignas(16) Node {
  float lo0[3], hi0[3];
  float lo1[3], hi1[3];
  int32_t c0, c1;
  int32_t pad[2];
};
static_assert(sizeof(Node) == 64, "node size");
constexpr int32_t kEmptyChild = 0x7fffffff;
constexpr int kMaxDepth = 48;

// Everything a kernel needs about the network, passed by value.
struct DevCfg {
  int32_t n_levels, n_features, log2_T, n_samples;
  int32_t n_in, width, hidden, n_out;
  uint32_t dense_mask;        // bit l set: level l indexed densely
  int32_t level_res[NBVH_MAX_LEVELS];
  uint32_t level_off[NBVH_MAX_LEVELS];  // first parameter (not entry) of level l
  float scene_lo[3];
  float inv_side;             // correctly rounded 1/scene_side
  float frac[16];             // (s + 1/2) / S, correctly rounded on the host
  // parameter layout (elements): W_k starts at w_off[k] inside params
  uint64_t n_table, n_mlp, n_params;
  uint64_t n_wt;                 // elements of the transposed weight copies
  uint64_t w_off[kMaxLayers];
  uint64_t wt_off[kMaxLayers];  // same layer, transposed copy, offset inside the aux arrays
  int32_t fan_in[kMaxLayers], fan_out[kMaxLayers];
  int32_t inside_reverse;  // leaves containing the ray origin are queried along the reversed chord
};

// FP8 block of the auxiliary buffer, after the transposed FP32 and BF16
// weight copies (6 bytes per element): E4M3 weights, layer k at byte
// w_off[k] - w_off[0] in the same row-major [fan_out][fan_in] order as the
// parameters, then kFp8Floats floats: weight scales sw[k], activation scales
// sa[k] (input of layer k), and the amax values they come from.
constexpr int kFp8Floats = 4 * kMaxLayers;
__host__ __device__ inline uint64_t fp8_weights_off(const DevCfg& c) { return (c.n_wt * 6 + 255) / 256 * 256; }
__host__ __device__ inline uint64_t fp8_scales_off(const DevCfg& c) {
  return (fp8_weights_off(c) + (c.n_params - c.w_off[0]) + 255) / 256 * 256;
}
__host__ __device__ inline uint64_t aux_total_bytes(const DevCfg& c) { return fp8_scales_off(c) + kFp8Floats * 4; }

// ---------------------------------------------------------------------------
// bf16 helpers (round to nearest even, as the hardware conversion)
// ---------------------------------------------------------------------------
__device__ __host__ inline float bf16_bits_to_f32(uint32_t b16) {
  union { uint32_t u; float f; } v;
  v.u = b16 << 16;
  return v.f;
}

__device__ __host__ inline uint16_t f32_to_bf16_bits(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  uint32_t u = v.u;
  if ((u & 0x7f800000u) == 0x7f800000u) {  // inf / nan
    return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  }
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// Sampling (stratum midpoints) and the unit-cube mapping, binary32 with one
// rounding per operation (the translation units are built without FP
// contraction); identical operation order to the definition used for parity.
// ---------------------------------------------------------------------------
// Explicit address spaces for accesses through pointers whose space the
// compiler cannot infer (a pointer picked at run time from several LDS
// tiles, or read from a kernel-argument struct): LDS accesses then compile to
// ds_read/ds_write and global ones to global_load/store, not to flat ones.
#define NBVH_LDS __attribute__((address_space(3)))
#define NBVH_GLOBAL __attribute__((address_space(1)))
template <typename V, typename T>
__device__ inline V lds_load(const T* p) {
  return *(const V NBVH_LDS*)((const char NBVH_LDS*)p);
}
template <typename V, typename T>
__device__ inline void lds_store(T* p, V v) {
  *(V NBVH_LDS*)((char NBVH_LDS*)p) = v;
}
template <typename V, typename T>
__device__ inline void global_store(T* p, V v) {
  *(V NBVH_GLOBAL*)((char NBVH_GLOBAL*)p) = v;
}

// Index of the calling thread's wavefront in its workgroup, as a
// wave-uniform (scalar) value: loops and table look-ups keyed by it then use
// scalar registers, scalar loads of per-level constants and uniform branches.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ inline void sample_position(const DevCfg& c, const float o[3], const float d[3], float t0,
                                       float t1, int s, float x[3]) {
  float frac = c.frac[s];
  float span = t1 - t0;
  float step = frac * span;
  float ts = t0 + step;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float dp = ts * d[a];
    float p = o[a] + dp;
    float rel = p - c.scene_lo[a];
    float xa = rel * c.inv_side;
    xa = xa < 0.0f ? 0.0f : xa;
    xa = xa > 1.0f ? 1.0f : xa;
    x[a] = xa;
  }
}

// Cell and weight along one axis for resolution N: the exact product x*N is
// hi + lo (two-product via fma), so floor(x*N) is decided exactly; the weight
// (x*N - cell) is rounded once.
__device__ inline void cell_weight(float x, int N, int& cell, float& w) {
  float fN = (float)N;
  float hi = x * fN;
  float lo = __builtin_fmaf(x, fN, -hi);
  float fl = floorf(hi);
  if (fl == hi && lo < 0.0f) fl -= 1.0f;
  if (fl > (float)(N - 1)) fl = (float)(N - 1);
  cell = (int)fl;
  w = (hi - fl) + lo;
}

__device__ inline uint32_t corner_index(bool dense, int N, uint32_t mask, uint32_t cx, uint32_t cy,
                                        uint32_t cz) {
  if (dense) {
    uint32_t r1 = (uint32_t)N + 1u;
    return cx + r1 * (cy + r1 * cz);
  }
  return (cx ^ (cy * 2654435761u) ^ (cz * 805459861u)) & mask;
}

// Read F features of one table entry as floats.
template <int F, bool LP>
__device__ inline void load_entry(const void* table, uint32_t param_index, float v[F]) {
  if constexpr (LP) {
    const uint16_t* t = (const uint16_t*)table + param_index;
    if constexpr (F == 2) {
      uint32_t w = *(const uint32_t*)t;
      v[0] = bf16_bits_to_f32(w & 0xffffu);
      v[1] = bf16_bits_to_f32(w >> 16);
    } else {
      uint2 w = *(const uint2*)t;
      v[0] = bf16_bits_to_f32(w.x & 0xffffu);
      v[1] = bf16_bits_to_f32(w.x >> 16);
      v[2] = bf16_bits_to_f32(w.y & 0xffffu);
      v[3] = bf16_bits_to_f32(w.y >> 16);
    }
  } else {
    const float* t = (const float*)table + param_index;
    if constexpr (F == 2) {
      float2 w = *(const float2*)t;
      v[0] = w.x;
      v[1] = w.y;
    } else {
      float4 w = *(const float4*)t;
      v[0] = w.x;
      v[1] = w.y;
      v[2] = w.z;
      v[3] = w.w;
    }
  }
}

// Trilinear interpolation of level l at unit-cube point x (Sec. 3: the hash
// grid of Mueller et al. 2022).
template <int F, bool LP>
__device__ inline void interp_level(const DevCfg& c, const void* table, int l, const float x[3],
                                    float out[F]) {
  const int N = c.level_res[l];
  const bool dense = (c.dense_mask >> l) & 1u;
  const uint32_t mask = (1u << c.log2_T) - 1u;
  int cx, cy, cz;
  float wx, wy, wz;
  cell_weight(x[0], N, cx, wx);
  cell_weight(x[1], N, cy, wy);
  cell_weight(x[2], N, cz, wz);
#pragma unroll
  for (int f = 0; f < F; ++f) out[f] = 0.0f;
  const uint32_t base = c.level_off[l];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    const float w = (dx ? wx : 1.0f - wx) * (dy ? wy : 1.0f - wy) * (dz ? wz : 1.0f - wz);
    const uint32_t idx = corner_index(dense, N, mask, cx + dx, cy + dy, cz + dz);
    float v[F];
    load_entry<F, LP>(table, base + idx * F, v);
#pragma unroll
    for (int f = 0; f < F; ++f) out[f] = __builtin_fmaf(w, v[f], out[f]);
  }
}

// Corner entry indices (parameter index of feature 0) and weights of level
// l, split from the loads so that callers can issue many gathers at once.
__device__ inline void corner_params(const DevCfg& c, int l, const float x[3], uint32_t idx[8], float wts[8]) {
  const int N = c.level_res[l];
  const bool dense = (c.dense_mask >> l) & 1u;
  const uint32_t mask = (1u << c.log2_T) - 1u;
  int cx, cy, cz;
  float wx, wy, wz;
  cell_weight(x[0], N, cx, wx);
  cell_weight(x[1], N, cy, wy);
  cell_weight(x[2], N, cz, wz);
  const uint32_t base = c.level_off[l];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    wts[k] = (dx ? wx : 1.0f - wx) * (dy ? wy : 1.0f - wy) * (dz ? wz : 1.0f - wz);
    idx[k] = base + corner_index(dense, N, mask, cx + dx, cy + dy, cz + dz) * c.n_features;
  }
}

// Corner indices and weights of level l (for the backward scatter).
__device__ inline void corners_level(const DevCfg& c, int l, const float x[3], uint32_t idx[8],
                                     float wts[8]) {
  const int N = c.level_res[l];
  const bool dense = (c.dense_mask >> l) & 1u;
  const uint32_t mask = (1u << c.log2_T) - 1u;
  int cx, cy, cz;
  float wx, wy, wz;
  cell_weight(x[0], N, cx, wx);
  cell_weight(x[1], N, cy, wy);
  cell_weight(x[2], N, cz, wz);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    wts[k] = (dx ? wx : 1.0f - wx) * (dy ? wy : 1.0f - wy) * (dz ? wz : 1.0f - wz);
    idx[k] = c.level_off[l] + corner_index(dense, N, mask, cx + dx, cy + dy, cz + dz) * c.n_features;
  }
}

__device__ inline float sigmoidf_(float z) { return 1.0f / (1.0f + __expf(-z)); }

// Workgroups go to the 8 accelerator dies round-robin (workgroup b to die
// b % 8). This bijection of [0, n) gives each die a contiguous range of
// tiles, so neighbouring tiles (one leaf's probes) share that die's L2.
__device__ inline uint32_t die_contiguous_tile(uint32_t b, uint32_t n) {
  const uint32_t q = n / 8u, r = n % 8u, x = b % 8u;
  return x * q + (x < r ? x : r) + b / 8u;
}

}  // namespace nbvh
