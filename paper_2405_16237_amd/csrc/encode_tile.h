// Encoding of a tile of segments into the LDS activation tile: lanes are
// segments (slots), so the 64 lookups of one wave instruction hit one level
// and neighbouring segments share cache lines; waves stride over the
// (sample, level) pairs.
#pragma once
#include "nbvh_internal.h"

namespace nbvh {

template <typename AT, int F>
__device__ inline void store_features(AT* dst, const float v[F]) {
  if constexpr (sizeof(AT) == 2) {
    if constexpr (F == 2) {
      uint32_t w = (uint32_t)f32_to_bf16_bits(v[0]) | ((uint32_t)f32_to_bf16_bits(v[1]) << 16);
      *(uint32_t*)dst = w;
    } else {
      uint2 w;
      w.x = (uint32_t)f32_to_bf16_bits(v[0]) | ((uint32_t)f32_to_bf16_bits(v[1]) << 16);
      w.y = (uint32_t)f32_to_bf16_bits(v[2]) | ((uint32_t)f32_to_bf16_bits(v[3]) << 16);
      *(uint2*)dst = w;
    }
  } else {
    if constexpr (F == 2)
      *(float2*)dst = make_float2(v[0], v[1]);
    else
      *(float4*)dst = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// Encode the M segments whose (o, t0) / (d, t1) sit in sA / sB into act0.
template <typename AT, int F, bool LP, int NWAVES>
__device__ inline void encode_tile(const DevCfg& c, const void* table, const float4* sA, const float4* sB,
                                   const int* s_valid, AT* act0, int ld0, int M) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int SL = c.n_samples * c.n_levels;
  for (int m = lane; m < M; m += 64) {
    const bool valid = s_valid[m] != 0;
    const float4 a = sA[m], b = sB[m];
    const float o[3] = {a.x, a.y, a.z}, d[3] = {b.x, b.y, b.z};
    for (int sl = wave; sl < SL; sl += NWAVES) {
      const int s = sl / c.n_levels, l = sl - s * c.n_levels;
      float v[F];
      if (valid) {
        float x[3];
        sample_position(c, o, d, a.w, b.w, s, x);
        interp_level<F, LP>(c, table, l, x, v);
      } else {
#pragma unroll
        for (int f = 0; f < F; ++f) v[f] = 0.0f;
      }
      store_features<AT, F>(act0 + (size_t)m * ld0 + s * c.n_levels * F + l * F, v);
    }
  }
}

}  // namespace nbvh
