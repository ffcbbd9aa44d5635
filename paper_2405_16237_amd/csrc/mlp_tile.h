// MLP layers on one tile of M rows held in LDS, on the CDNA4 matrix cores.
//
// A layer computes out[m][n] = sum_k act[m][k] * W[n][k] (W row-major with
// row stride ldw, no bias). It is issued as the transposed product
// out^T = W x act^T so that both MFMA operands are contiguous 16-byte
// loads: the A fragment is 8 consecutive k of one W row (global/L2), the B
// fragment 8 consecutive k of one activation row (LDS). The 16x16
// accumulator tile of a lane then holds 4 consecutive output features of
// one row, handed to the epilogue (ReLU + store, mask + store, raw store).
//
// BF16 path: v_mfma_f32_16x16x32_bf16, FP32 accumulation, activations
// rounded to bf16 between layers. FP32 path: v_mfma_f32_16x16x4_f32.
#pragma once
#include "nbvh_internal.h"

namespace nbvh {

// FP8 E4M3 (OCP) activation byte
struct fp8e4 {
  uint8_t v;
};

template <typename AT>
struct Pad;
template <>
struct Pad<fp8e4> {
  static constexpr int v = 16;  // bytes: rows start 4 banks apart
  static constexpr int kstep = 32;
};
template <>
struct Pad<bf16> {
  static constexpr int v = 8;  // 16 bytes per row: rows start 4 banks apart
  static constexpr int kstep = 32;
};
template <>
struct Pad<float> {
  static constexpr int v = 4;
  static constexpr int kstep = 16;
};

__device__ inline bf16x8 zero_bf16x8() {
  bf16x8 z;
#pragma unroll
  for (int i = 0; i < 8; ++i) z[i] = (bf16)0.0f;
  return z;
}

// The first two weight fragments (k = 0..63 of its first n-tile) a wave
// needs in a BF16 layer, fetched ahead so that they are in flight while the
// previous layer (or the encoding) still computes.
struct PreBf16 {
  bf16x8 a0, a1;
};

template <int NWAVES>
__device__ inline PreBf16 prefetch_bf16(const bf16* __restrict__ W, int ldw, int K, int N) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int n = wave * 16 + (lane & 15);
  PreBf16 p{zero_bf16x8(), zero_bf16x8()};
  if (n < N) {
    const bf16* wrow = W + (size_t)n * ldw + 8 * (lane >> 4);
    p.a0 = *(const bf16x8*)wrow;
    if (32 < K) p.a1 = *(const bf16x8*)(wrow + 32);
  }
  return p;
}

// out^T tile loop. Epi(m, col, f32x4) receives rows m, columns col..col+3.
// `pre`, if given, holds the wave's first two fragments (prefetch_bf16).
template <int M, int NWAVES, typename Epi>
__device__ inline void gemm_tile_bf16(const bf16* act_in, int ld_in, int K, const bf16* __restrict__ W, int ldw,
                                      int N, Epi epi, const PreBf16* pre = nullptr) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int r16 = lane & 15, q = lane >> 4;
  const int n_tiles = (N + 15) >> 4;
  for (int nt = wave; nt < n_tiles; nt += NWAVES) {
    f32x4 acc[M / 16];
#pragma unroll
    for (int mt = 0; mt < M / 16; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int n = nt * 16 + r16;
    const bool nvalid = n < N;
    const bf16* wrow = W + (size_t)(nvalid ? n : 0) * ldw + 8 * q;
    const bf16* arow = act_in + (size_t)r16 * ld_in + 8 * q;
    for (int k0 = 0; k0 < K; k0 += 64) {
      const bool two = k0 + 32 < K;
      bf16x8 a0, a1;
      if (pre && k0 == 0 && nt == wave) {
        a0 = pre->a0;
        a1 = pre->a1;
      } else {
        a0 = nvalid ? *(const bf16x8*)(wrow + k0) : zero_bf16x8();
        a1 = (nvalid && two) ? *(const bf16x8*)(wrow + k0 + 32) : zero_bf16x8();
      }
#pragma unroll
      for (int mt = 0; mt < M / 16; ++mt) {
        bf16x8 b0 = lds_load<bf16x8>(arow + (size_t)mt * 16 * ld_in + k0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[mt], 0, 0, 0);
      }
      if (two) {
#pragma unroll
        for (int mt = 0; mt < M / 16; ++mt) {
          bf16x8 b1 = lds_load<bf16x8>(arow + (size_t)mt * 16 * ld_in + k0 + 32);
          acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[mt], 0, 0, 0);
        }
      }
    }
    const int col = nt * 16 + 4 * q;
#pragma unroll
    for (int mt = 0; mt < M / 16; ++mt) epi(mt * 16 + r16, col, acc[mt]);
  }
}

template <int M, int NWAVES, typename Epi>
__device__ inline void gemm_tile_f32(const float* act_in, int ld_in, int K, const float* __restrict__ W, int ldw,
                                     int N, Epi epi) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int r16 = lane & 15, q = lane >> 4;
  const int n_tiles = (N + 15) >> 4;
  for (int nt = wave; nt < n_tiles; nt += NWAVES) {
    f32x4 acc[M / 16];
#pragma unroll
    for (int mt = 0; mt < M / 16; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int n = nt * 16 + r16;
    const bool nvalid = n < N;
    const float* wrow = W + (size_t)(nvalid ? n : 0) * ldw + 4 * q;
    const float* arow = act_in + (size_t)r16 * ld_in + 4 * q;
    for (int k0 = 0; k0 < K; k0 += 16) {
      float4 a = nvalid ? *(const float4*)(wrow + k0) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int mt = 0; mt < M / 16; ++mt) {
        const f32x4 b = lds_load<f32x4>(arow + (size_t)mt * 16 * ld_in + k0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc[mt], 0, 0, 0);
      }
    }
    const int col = nt * 16 + 4 * q;
#pragma unroll
    for (int mt = 0; mt < M / 16; ++mt) epi(mt * 16 + r16, col, acc[mt]);
  }
}

// FP8 x FP8 -> FP32, 16x16x32 MFMA: 8 bytes of k per lane, same lane layout
// as the BF16 path.
template <int M, int NWAVES, typename Epi>
__device__ inline void gemm_tile_fp8(const uint8_t* act_in, int ld_in, int K, const uint8_t* __restrict__ W, int ldw,
                                     int N, Epi epi) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int r16 = lane & 15, q = lane >> 4;
  const int n_tiles = (N + 15) >> 4;
  for (int nt = wave; nt < n_tiles; nt += NWAVES) {
    f32x4 acc[M / 16];
#pragma unroll
    for (int mt = 0; mt < M / 16; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int n = nt * 16 + r16;
    const bool nvalid = n < N;
    const uint8_t* wrow = W + (size_t)(nvalid ? n : 0) * ldw + 8 * q;
    const uint8_t* arow = act_in + (size_t)r16 * ld_in + 8 * q;
    for (int k0 = 0; k0 < K; k0 += 32) {
      const long a = nvalid ? *(const long*)(wrow + k0) : 0l;
#pragma unroll
      for (int mt = 0; mt < M / 16; ++mt) {
        const long b = lds_load<long>(arow + (size_t)mt * 16 * ld_in + k0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc[mt], 0, 0, 0);
      }
    }
    const int col = nt * 16 + 4 * q;
#pragma unroll
    for (int mt = 0; mt < M / 16; ++mt) epi(mt * 16 + r16, col, acc[mt]);
  }
}

// Quantise to FP8 E4M3 with saturation at +-448 (the format's largest value).
__device__ inline uint32_t pack_fp8x4(float a, float b, float c, float d) {
  a = fminf(fmaxf(a, -448.0f), 448.0f);
  b = fminf(fmaxf(b, -448.0f), 448.0f);
  c = fminf(fmaxf(c, -448.0f), 448.0f);
  d = fminf(fmaxf(d, -448.0f), 448.0f);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  return (uint32_t)w;
}

// FP8 forward of a tile: act0 holds the input quantised with sa[0];
// W8 the weights quantised with sw[k]; each hidden output is dequantised,
// ReLU'd and requantised with sa[k+1]; z receives FP32 logits.
template <int M, int NWAVES>
__device__ inline void mlp_forward_tile_fp8(const DevCfg& c, const uint8_t* W8base, const float* scales,
                                            uint8_t* act0, int ld0, uint8_t* act1, int ld1, float* z, int ldz) {
  uint8_t* cur = act0;
  int ldc = ld0;
  uint8_t* nxt = act1;
  int ldn = ld1;
  for (int k = 0; k <= c.hidden; ++k) {
    const bool last = (k == c.hidden);
    const uint8_t* W = W8base + (c.w_off[k] - c.w_off[0]);
    const float dq = 1.0f / (scales[k] * scales[kMaxLayers + k]);  // 1 / (sw_k * sa_k)
    if (last) {
      gemm_tile_fp8<M, NWAVES>(cur, ldc, c.fan_in[k], W, c.fan_in[k], c.fan_out[k], [&](int m, int col, f32x4 v) {
        *(f32x4*)(z + (size_t)m * ldz + col) = v * dq;
      });
    } else {
      const float qn = scales[kMaxLayers + k + 1];
      gemm_tile_fp8<M, NWAVES>(cur, ldc, c.fan_in[k], W, c.fan_in[k], c.fan_out[k], [&](int m, int col, f32x4 v) {
        f32x4 r;
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = fmaxf(v[i] * dq, 0.0f) * qn;
        *(uint32_t*)(nxt + (size_t)m * ldn + col) = pack_fp8x4(r[0], r[1], r[2], r[3]);
      });
    }
    __syncthreads();
    uint8_t* t = cur;
    cur = nxt;
    nxt = t;
    int tl = ldc;
    ldc = ldn;
    ldn = tl;
  }
}

template <int M, int NWAVES, typename AT, typename Epi>
__device__ inline void gemm_tile(const AT* act_in, int ld_in, int K, const AT* W, int ldw, int N, Epi epi,
                                 const PreBf16* pre = nullptr) {
  if constexpr (sizeof(AT) == 2)
    gemm_tile_bf16<M, NWAVES>(act_in, ld_in, K, W, ldw, N, epi, pre);
  else
    gemm_tile_f32<M, NWAVES>(act_in, ld_in, K, W, ldw, N, epi);
}

// four consecutive activations of an LDS tile row
template <typename AT>
__device__ inline void store4(AT* dst, f32x4 v) {
  if constexpr (sizeof(AT) == 2) {
    bf16x4 b;
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = (bf16)v[i];
    lds_store<bf16x4>(dst, b);
  } else {
    lds_store<f32x4>(dst, v);
  }
}

// Full forward of the tile: act0 holds the encoded input [M][n_in]; hidden
// layers ping-pong between act0 and act1; z receives [M][kOutPad] fp32.
// keep(k, m, col, relu_vals) sees every hidden output (k = layer index).
// BF16: each layer's first weight fragments are prefetched while the
// previous layer computes (layer 0's may come from the caller, `pre0`).
template <int M, int NWAVES, typename AT, typename Keep>
__device__ inline void mlp_forward_tile_keep(const DevCfg& c, const AT* Wbase, AT* act0, int ld0, AT* act1, int ld1,
                                             float* z, int ldz, Keep keep, const PreBf16* pre0 = nullptr) {
  AT* cur = act0;
  int ldc = ld0;
  AT* nxt = act1;
  int ldn = ld1;
  PreBf16 pre{};
  if constexpr (sizeof(AT) == 2) {
    if (pre0) pre = *pre0;
    else pre = prefetch_bf16<NWAVES>((const bf16*)Wbase + c.w_off[0], c.fan_in[0], c.fan_in[0], c.fan_out[0]);
  }
  for (int k = 0; k <= c.hidden; ++k) {
    const bool last = (k == c.hidden);
    const AT* W = Wbase + c.w_off[k];
    PreBf16 pre_next{};
    if constexpr (sizeof(AT) == 2) {
      if (!last)
        pre_next = prefetch_bf16<NWAVES>((const bf16*)Wbase + c.w_off[k + 1], c.fan_in[k + 1], c.fan_in[k + 1],
                                         c.fan_out[k + 1]);
    }
    const PreBf16* pp = sizeof(AT) == 2 ? &pre : nullptr;
    if (last) {
      gemm_tile<M, NWAVES, AT>(cur, ldc, c.fan_in[k], W, c.fan_in[k], c.fan_out[k],
                               [&](int m, int col, f32x4 v) { *(f32x4*)(z + (size_t)m * ldz + col) = v; }, pp);
    } else {
      gemm_tile<M, NWAVES, AT>(
          cur, ldc, c.fan_in[k], W, c.fan_in[k], c.fan_out[k],
          [&](int m, int col, f32x4 v) {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = fmaxf(v[i], 0.0f);
            store4<AT>(nxt + (size_t)m * ldn + col, v);
            keep(k, m, col, v);
          },
          pp);
    }
    pre = pre_next;
    __syncthreads();
    AT* t = cur;
    cur = nxt;
    nxt = t;
    int tl = ldc;
    ldc = ldn;
    ldn = tl;
  }
}

template <int M, int NWAVES, typename AT>
__device__ inline void mlp_forward_tile(const DevCfg& c, const AT* Wbase, AT* act0, int ld0, AT* act1, int ld1,
                                        float* z, int ldz, const PreBf16* pre0 = nullptr) {
  mlp_forward_tile_keep<M, NWAVES, AT>(c, Wbase, act0, ld0, act1, ld1, z, ldz, [](int, int, int, f32x4) {}, pre0);
}

}  // namespace nbvh
