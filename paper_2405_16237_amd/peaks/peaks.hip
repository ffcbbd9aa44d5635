// Achievable ceilings of the MI355X units the N-BVH kernels are bound by,
// measured by small loops of the same access and instruction patterns:
//
//  - scattered table gathers: every lane of a wave loads one 4- or 8-byte
//    entry; the 64 lanes fall on `lines` distinct 64-byte lines (8 for a
//    coherent group of rays, as the query's gathers, 64 for incoherent
//    lanes), lines drawn at random over a table of the given size;
//  - streaming reads of a buffer of the given size (L2, Infinity Cache or
//    HBM resident), 16 bytes per lane, several passes;
//  - FP32 atomic adds to random words of a gradient-sized buffer, one word
//    per lane, or runs of 4 consecutive lanes on consecutive words;
//  - LDS 64-bit integer atomic adds to random slots of a 32 KiB table;
//  - matrix-core loops: BF16 16x16x32 and 32x32x16, FP8 16x16x32 (the
//    shapes the kernels use) and the gfx950 FP8 16x16x128.
//
// Each entry point launches its loop on `stream`, times it with HIP events
// and returns the elapsed milliseconds (negative on a HIP error). Addresses
// stay inside the caller's buffer: every index is masked by a power-of-two
// size no larger than the buffer.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float v4f;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float v16f;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 v8bf;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int v8i;

__device__ inline uint32_t lcg(uint32_t x) { return x * 1664525u + 1013904223u; }

// One loop iteration issues U independent gathers per lane.
template <int E, int U>
__global__ __launch_bounds__(256) void k_gather(const uint32_t* __restrict__ table, uint32_t line_mask, int lines,
                                                int iters, uint32_t* __restrict__ sink) {
  const int lane = threadIdx.x & 63;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  constexpr int kWordsPerLine = 64 / E;
  const int group = lane % lines;               // lanes of one group read one line
  const int word = (lane / lines) % kWordsPerLine;  // distinct words within it
  uint32_t x[U];
#pragma unroll
  for (int u = 0; u < U; ++u) x[u] = lcg(wave * 2654435761u + (uint32_t)(group * 97 + u * 7919));
  uint32_t acc = 0;
  for (int i = 0; i < iters; ++i) {
    uint32_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x[u] = lcg(x[u]);
      const uint32_t line = (x[u] >> 7) & line_mask;
      const uint32_t idx = line * (64u / 4u) + (uint32_t)(word * (E / 4));
      if constexpr (E == 4) {
        v[u] = table[idx];
      } else {
        const uint2 p = *(const uint2*)(table + idx);
        v[u] = p.x ^ p.y;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_stream(const uint4* __restrict__ buf, uint64_t n16, int reps,
                                                uint32_t* __restrict__ sink) {
  uint32_t acc = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (int r = 0; r < reps; ++r) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += 4 * stride) {
      uint4 a = buf[i];
      uint4 b = i + stride < n16 ? buf[i + stride] : make_uint4(0, 0, 0, 0);
      uint4 c = i + 2 * stride < n16 ? buf[i + 2 * stride] : make_uint4(0, 0, 0, 0);
      uint4 d = i + 3 * stride < n16 ? buf[i + 3 * stride] : make_uint4(0, 0, 0, 0);
      acc += a.x ^ b.y ^ c.z ^ d.w;
    }
  }
  sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <int RUN>
__global__ __launch_bounds__(256) void k_atomic_f32(float* __restrict__ buf, uint32_t mask, int iters) {
  const int lane = threadIdx.x & 63;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  uint32_t x = lcg(wave * 2654435761u + (uint32_t)(lane / RUN) * 40503u);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x = lcg(x);
      const uint32_t w = ((x >> 5) * RUN + (uint32_t)(lane % RUN)) & mask;
      atomicAdd(buf + w, 1.0f);
    }
  }
}

__global__ __launch_bounds__(256) void k_lds_atomic(int iters, unsigned long long* __restrict__ sink) {
  __shared__ unsigned long long tab[4096];
  for (int i = threadIdx.x; i < 4096; i += blockDim.x) tab[i] = 0ull;
  __syncthreads();
  uint32_t x = lcg((blockIdx.x * blockDim.x + threadIdx.x) * 2654435761u);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x = lcg(x);
      atomicAdd(&tab[(x >> 9) & 4095u], (unsigned long long)(x & 255u));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) sink[blockIdx.x] = tab[blockIdx.x & 4095u];
}

// K independent accumulator chains per wave keep the matrix pipeline full.
template <int K>
__global__ __launch_bounds__(256) void k_mfma_bf16_16(int iters, float* __restrict__ sink) {
  v8bf a, b;
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(0.001f * (float)((threadIdx.x + i) & 7));
    b[i] = (__bf16)(0.002f * (float)((threadIdx.x * 3 + i) & 7));
  }
  v4f c[K];
  for (int k = 0; k < K; ++k) c[k] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[k], 0, 0, 0);
  }
  float s = 0.f;
  for (int k = 0; k < K; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int K>
__global__ __launch_bounds__(256) void k_mfma_bf16_32(int iters, float* __restrict__ sink) {
  v8bf a, b;
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(0.001f * (float)((threadIdx.x + i) & 7));
    b[i] = (__bf16)(0.002f * (float)((threadIdx.x * 3 + i) & 7));
  }
  v16f c[K];
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < 16; ++j) c[k][j] = 0.f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[k], 0, 0, 0);
  }
  float s = 0.f;
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < 16; ++j) s += c[k][j];
  sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int K>
__global__ __launch_bounds__(256) void k_mfma_fp8_16(int iters, float* __restrict__ sink) {
  const long a = 0x3838383838383838l + (long)(threadIdx.x & 3);
  const long b = 0x3030303030303030l + (long)(threadIdx.x & 1);
  v4f c[K];
  for (int k = 0; k < K; ++k) c[k] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c[k], 0, 0, 0);
  }
  float s = 0.f;
  for (int k = 0; k < K; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int K>
__global__ __launch_bounds__(256) void k_mfma_fp8_16x128(int iters, float* __restrict__ sink) {
  v8i a, b;
  for (int i = 0; i < 8; ++i) {
    a[i] = 0x38383838 + (int)((threadIdx.x + i) & 3);
    b[i] = 0x30303030 + (int)((threadIdx.x + i) & 1);
  }
  v4f c[K];
  for (int k = 0; k < K; ++k) c[k] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      c[k] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c[k], 0, 0, 0, 0, 0, 0);
  }
  float s = 0.f;
  for (int k = 0; k < K; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

struct Timer {
  hipEvent_t a, b;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, s);
  }
  double stop() {
    (void)hipEventRecord(b, s);
    if (hipEventSynchronize(b) != hipSuccess || hipGetLastError() != hipSuccess) return -1.0;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
  }
};

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

}  // namespace

extern "C" {

// Gathers of `entry_bytes` (4 or 8) from a table of table_bytes (a power of
// two, >= 64) with `lines` (1..64, a power of two) distinct lines per wave:
// grid x 256 lanes x iters x 8 gathers. sink: grid * 256 words.
double peaks_gather(const void* table, uint64_t table_bytes, int entry_bytes, int lines, uint32_t grid, int iters,
                    void* sink, void* stream) {
  if (!pow2(table_bytes) || table_bytes < 64 || (entry_bytes != 4 && entry_bytes != 8) || !pow2((uint64_t)lines) ||
      lines > 64 || grid == 0 || iters <= 0)
    return -2.0;
  hipStream_t s = (hipStream_t)stream;
  const uint32_t line_mask = (uint32_t)(table_bytes / 64 - 1);
  if (entry_bytes == 4) k_gather<4, 8><<<grid, 256, 0, s>>>((const uint32_t*)table, line_mask, lines, 1, (uint32_t*)sink);
  else k_gather<8, 8><<<grid, 256, 0, s>>>((const uint32_t*)table, line_mask, lines, 1, (uint32_t*)sink);
  Timer t(s);
  if (entry_bytes == 4) k_gather<4, 8><<<grid, 256, 0, s>>>((const uint32_t*)table, line_mask, lines, iters, (uint32_t*)sink);
  else k_gather<8, 8><<<grid, 256, 0, s>>>((const uint32_t*)table, line_mask, lines, iters, (uint32_t*)sink);
  return t.stop();
}

// `reps` passes of 16-byte loads over buf (bytes a multiple of 16).
double peaks_stream(const void* buf, uint64_t bytes, int reps, uint32_t grid, void* sink, void* stream) {
  if (bytes < 16 || bytes % 16 || reps <= 0 || grid == 0) return -2.0;
  hipStream_t s = (hipStream_t)stream;
  k_stream<<<grid, 256, 0, s>>>((const uint4*)buf, bytes / 16, 1, (uint32_t*)sink);
  Timer t(s);
  k_stream<<<grid, 256, 0, s>>>((const uint4*)buf, bytes / 16, reps, (uint32_t*)sink);
  return t.stop();
}

// grid x 256 lanes x iters x 4 FP32 atomic adds into buf (words: a power of
// two); run 1: scattered words, run 4: 4 consecutive lanes on 4 consecutive words.
double peaks_atomic_f32(float* buf, uint64_t words, int run, uint32_t grid, int iters, void* stream) {
  if (!pow2(words) || words > (1ull << 32) || (run != 1 && run != 4) || grid == 0 || iters <= 0) return -2.0;
  hipStream_t s = (hipStream_t)stream;
  const uint32_t mask = (uint32_t)(words - 1);
  Timer t(s);
  if (run == 1) k_atomic_f32<1><<<grid, 256, 0, s>>>(buf, mask, iters);
  else k_atomic_f32<4><<<grid, 256, 0, s>>>(buf, mask, iters);
  return t.stop();
}

// grid x 256 lanes x iters x 4 LDS 64-bit atomic adds. sink: grid words.
double peaks_lds_atomic(uint32_t grid, int iters, void* sink, void* stream) {
  if (grid == 0 || iters <= 0) return -2.0;
  hipStream_t s = (hipStream_t)stream;
  Timer t(s);
  k_lds_atomic<<<grid, 256, 0, s>>>(iters, (unsigned long long*)sink);
  return t.stop();
}

// Matrix-core loop: kind 0 = BF16 16x16x32, 1 = BF16 32x32x16,
// 2 = FP8 16x16x32, 3 = FP8 16x16x128; grid x 4 waves x iters x 8 products.
// *flops_out receives the floating-point operations performed.
double peaks_mfma(int kind, uint32_t grid, int iters, void* sink, double* flops_out, void* stream) {
  if (kind < 0 || kind > 3 || grid == 0 || iters <= 0 || !flops_out) return -2.0;
  hipStream_t s = (hipStream_t)stream;
  constexpr int K = 8;
  const double per = kind == 0 ? 16.0 * 16 * 32 * 2 : kind == 1 ? 32.0 * 32 * 16 * 2 : kind == 2 ? 16.0 * 16 * 32 * 2
                                                                                                 : 16.0 * 16 * 128 * 2;
  *flops_out = per * K * (double)iters * grid * 4;
  Timer t(s);
  switch (kind) {
    case 0: k_mfma_bf16_16<K><<<grid, 256, 0, s>>>(iters, (float*)sink); break;
    case 1: k_mfma_bf16_32<K><<<grid, 256, 0, s>>>(iters, (float*)sink); break;
    case 2: k_mfma_fp8_16<K><<<grid, 256, 0, s>>>(iters, (float*)sink); break;
    default: k_mfma_fp8_16x128<K><<<grid, 256, 0, s>>>(iters, (float*)sink); break;
  }
  return t.stop();
}

}  // extern "C"
