// Encoding of a tile of segments into the LDS activation tile: lanes are
// segments (slots), so the 64 lookups of one wave instruction hit one level
// and neighbouring segments share cache lines; waves stride over the
// (sample, level) pairs.
#pragma once
#include "mlp_tile.h"
#include "nbvh_internal.h"

namespace nbvh {

template <typename AT, int F>
__device__ inline void store_features(AT* dst, const float v[F], float qscale = 1.0f) {
  if constexpr (sizeof(AT) == 1) {
    const uint32_t w = pack_fp8x4(v[0] * qscale, v[1] * qscale, F == 4 ? v[2 % F] * qscale : 0.0f,
                                  F == 4 ? v[3 % F] * qscale : 0.0f);
    if constexpr (F == 2)
      *(uint16_t*)dst = (uint16_t)w;
    else
      *(uint32_t*)dst = w;
  } else if constexpr (sizeof(AT) == 2) {
    // round to nearest even on the hardware converter (one instruction per pair)
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    if constexpr (F == 2) {
      *(bf16x2*)dst = bf16x2{(bf16)v[0], (bf16)v[1]};
    } else {
      *(bf16x4*)dst = bf16x4{(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
    }
  } else {
    if constexpr (F == 2)
      *(float2*)dst = make_float2(v[0], v[1]);
    else
      *(float4*)dst = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// Raw table entry (F features) as loaded: packed bf16 or fp32 words.
template <int F, bool LP>
struct RawEntry;
template <>
struct RawEntry<2, true> {
  typedef uint32_t T;
};
template <>
struct RawEntry<4, true> {
  typedef uint2 T;
};
template <>
struct RawEntry<2, false> {
  typedef float2 T;
};
template <>
struct RawEntry<4, false> {
  typedef float4 T;
};

template <int F, bool LP>
__device__ inline typename RawEntry<F, LP>::T load_raw(const void* table, uint32_t param_index) {
  typedef typename RawEntry<F, LP>::T T;
  // 32-bit byte offset from a uniform base: one VGPR per address (tables
  // are far below 4 GiB); the pointer is a global one, so the load is a
  // global (not a flat) load whichever other loads sit beside it
  const uint32_t byte_off = param_index * (LP ? 2u : 4u);
  typedef uint32_t W __attribute__((ext_vector_type(sizeof(T) / 4)));
  const W w = *(const W __attribute__((address_space(1)))*)((const char __attribute__((address_space(1)))*)table +
                                                             byte_off);
  T r;
  __builtin_memcpy(&r, &w, sizeof(T));
  return r;
}

template <int F, bool LP>
__device__ inline void unpack_raw(const typename RawEntry<F, LP>::T& r, float v[F]) {
  if constexpr (LP) {
    if constexpr (F == 2) {
      v[0] = bf16_bits_to_f32(r & 0xffffu);
      v[1] = bf16_bits_to_f32(r >> 16);
    } else {
      v[0] = bf16_bits_to_f32(r.x & 0xffffu);
      v[1] = bf16_bits_to_f32(r.x >> 16);
      v[2] = bf16_bits_to_f32(r.y & 0xffffu);
      v[3] = bf16_bits_to_f32(r.y >> 16);
    }
  } else {
    if constexpr (F == 2) {
      v[0] = r.x;
      v[1] = r.y;
    } else {
      v[0] = r.x;
      v[1] = r.y;
      v[2] = r.z;
      v[3] = r.w;
    }
  }
}

// The same entry from the workgroup's LDS copy of the table's leading levels
// (same parameter indices: the copy starts at parameter 0).
template <int F, bool LP>
__device__ inline typename RawEntry<F, LP>::T load_raw_lds(const unsigned char* ltab, uint32_t param_index) {
  typedef typename RawEntry<F, LP>::T T;
  typedef uint32_t W __attribute__((ext_vector_type(sizeof(T) / 4)));
  const W w = *(const W __attribute__((address_space(3)))*)((const unsigned char __attribute__((address_space(3)))*)ltab +
                                                             param_index * (LP ? 2u : 4u));
  T r;
  __builtin_memcpy(&r, &w, sizeof(T));
  return r;
}

// Two adjacent table entries (an x-neighbour pair) as loaded.
template <int F, bool LP>
struct RawPair;
template <>
struct RawPair<2, true> {
  typedef uint2 T;  // 2 entries x 2 bf16
};
template <>
struct RawPair<4, true> {
  typedef uint4 T;  // 2 entries x 4 bf16
};
template <>
struct RawPair<2, false> {
  typedef float4 T;  // 2 entries x 2 fp32
};

template <int F, bool LP>
__device__ inline typename RawPair<F, LP>::T load_pair(const void* table, uint32_t param_index) {
  typedef typename RawPair<F, LP>::T T;
  const uint32_t byte_off = param_index * (LP ? 2u : 4u);
  return *(const T*)((const char*)table + byte_off);
}

// entry 0 / 1 of a pair, as a raw entry
template <int F, bool LP>
__device__ inline typename RawEntry<F, LP>::T pair_half(const typename RawPair<F, LP>::T& p, bool second) {
  if constexpr (LP && F == 2) return second ? p.y : p.x;
  else if constexpr (LP && F == 4) return second ? uint2{p.z, p.w} : uint2{p.x, p.y};
  else return second ? float2{p.z, p.w} : float2{p.x, p.y};
}

// Encode the M segments whose (o, t0) / (d, t1) sit in sA / sB into act0.
// Wave w owns levels w, w + NWAVES, ... and walks them U at a time; for each
// group of levels it takes the samples in ray order, issuing the gathers of
// all U levels before consuming any. Consecutive samples of a segment often
// fall into the same cell at the coarser levels: such a lane keeps the
// corner values it already holds and is masked out of the gathers.
// Levels below lds_levels are gathered from ltab, the workgroup's LDS copy of
// the table's leading levels (not with PAIRS).
// With PAIRS, corners are fetched as x-neighbour pairs: on dense levels
// (x, x+1) are adjacent entries; on hashed levels they are the two halves of
// an aligned pair whenever x is even (the hash keeps x's low bit), so one
// load serves both and lanes with odd x add one masked load.
template <typename AT, int F, bool LP, int NWAVES, int UNROLL = 0, bool PAIRS = false>
__device__ inline void encode_tile(const DevCfg& c, const void* table, const float4* sA, const float4* sB,
                                   const int* s_valid, AT* act0, int ld0, int M, float qscale = 1.0f,
                                   const unsigned char* ltab = nullptr, int lds_levels = 0) {
  typedef typename RawEntry<F, LP>::T Raw;
  constexpr bool kPairs = PAIRS && !(F == 4 && !LP);  // a 32-byte fp32 pair has no single load
  constexpr int U = UNROLL > 0 ? UNROLL : 2;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int L = c.n_levels, S = c.n_samples;
  const uint32_t hmask = (1u << c.log2_T) - 1u;
  for (int m = lane; m < M; m += 64) {
    const bool valid = s_valid[m] != 0;
    const float4 a = sA[m], b = sB[m];
    const float o[3] = {a.x, a.y, a.z}, d[3] = {b.x, b.y, b.z};
    for (int lg = wave; lg < L; lg += NWAVES * U) {
      Raw raw[U][8];
      int pcx[U], pcy[U], pcz[U];
      bool act[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        act[u] = lg + u * NWAVES < L;
        pcx[u] = pcy[u] = pcz[u] = -1;
      }
      for (int s = 0; s < S; ++s) {
        float x[3];
        sample_position(c, o, d, a.w, b.w, s, x);
        float wx[U], wy[U], wz[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int l = act[u] ? lg + u * NWAVES : 0;
          const int N = c.level_res[l];
          const bool dense = (c.dense_mask >> l) & 1u;
          int cx, cy, cz;
          cell_weight(x[0], N, cx, wx[u]);
          cell_weight(x[1], N, cy, wy[u]);
          cell_weight(x[2], N, cz, wz[u]);
          const bool need = act[u] && valid && (cx != pcx[u] || cy != pcy[u] || cz != pcz[u]);
          pcx[u] = cx;
          pcy[u] = cy;
          pcz[u] = cz;
          const uint32_t base = c.level_off[l];
          if (need) {
            if constexpr (kPairs) {
              if (dense) {
                const uint32_t r1 = (uint32_t)N + 1u;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  const uint32_t i0 =
                      base + ((uint32_t)cx + r1 * ((uint32_t)(cy + (j & 1)) + r1 * (uint32_t)(cz + (j >> 1)))) * F;
                  const auto p = load_pair<F, LP>(table, i0);
                  raw[u][2 * j] = pair_half<F, LP>(p, false);
                  raw[u][2 * j + 1] = pair_half<F, LP>(p, true);
                }
              } else {
                const bool even = (cx & 1) == 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  const uint32_t hyz =
                      ((uint32_t)(cy + (j & 1)) * 2654435761u) ^ ((uint32_t)(cz + (j >> 1)) * 805459861u);
                  const uint32_t h0 = ((uint32_t)cx ^ hyz) & hmask;
                  const uint32_t h1 = ((uint32_t)(cx + 1) ^ hyz) & hmask;
                  const auto p = load_pair<F, LP>(table, base + (h0 & ~1u) * F);
                  raw[u][2 * j] = pair_half<F, LP>(p, (h0 & 1u) != 0u);
                  raw[u][2 * j + 1] = even ? pair_half<F, LP>(p, (h1 & 1u) != 0u) : load_raw<F, LP>(table, base + h1 * F);
                }
              }
            } else {
              // the 8 corner entries first (the dense/hashed choice is
              // uniform over the wave, so one branch per level), then the 8
              // loads back to back: dense levels index x + (N+1)(y + (N+1) z),
              // hashed ones XOR the per-axis products, the upper y and z
              // products being the lower ones plus the prime
              uint32_t idx[8];
              if (dense) {
                const uint32_t r1 = (uint32_t)N + 1u, r2 = r1 * r1;
                const uint32_t i0 = (uint32_t)cx + r1 * ((uint32_t)cy + r1 * (uint32_t)cz);
#pragma unroll
                for (int k = 0; k < 8; ++k)
                  idx[k] = base + (i0 + (uint32_t)(k & 1) + ((k & 2) ? r1 : 0u) + ((k & 4) ? r2 : 0u)) * F;
              } else {
                const uint32_t hy0 = (uint32_t)cy * 2654435761u, hz0 = (uint32_t)cz * 805459861u;
                const uint32_t hy1 = hy0 + 2654435761u, hz1 = hz0 + 805459861u;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                  idx[k] = base + ((((uint32_t)cx + (uint32_t)(k & 1)) ^ ((k & 2) ? hy1 : hy0) ^ ((k & 4) ? hz1 : hz0)) &
                                   hmask) * F;
              }
              if (l < lds_levels) {  // wave-uniform
#pragma unroll
                for (int k = 0; k < 8; ++k) raw[u][k] = load_raw_lds<F, LP>(ltab, idx[k]);
              } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) raw[u][k] = load_raw<F, LP>(table, idx[k]);
              }
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (!act[u]) continue;
          float out[F];
#pragma unroll
          for (int f = 0; f < F; ++f) out[f] = 0.0f;
          if (valid) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const float w = ((k & 1) ? wx[u] : 1.0f - wx[u]) * (((k >> 1) & 1) ? wy[u] : 1.0f - wy[u]) *
                              (((k >> 2) & 1) ? wz[u] : 1.0f - wz[u]);
              float v[F];
              unpack_raw<F, LP>(raw[u][k], v);
#pragma unroll
              for (int f = 0; f < F; ++f) out[f] = __builtin_fmaf(w, v[f], out[f]);
            }
          }
          const int col = s * L * F + (lg + u * NWAVES) * F;
          store_features<AT, F>(act0 + (size_t)m * ld0 + col, out, qscale);
        }
      }
    }
  }
}

}  // namespace nbvh
