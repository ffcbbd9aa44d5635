// N-BVH traversal (Sec. 5): per-lane stack, two child slab tests per visit,
// count -> exclusive scan -> fill into a compacted segment queue, each ray's
// run sorted front to back by (t0, leaf id).
//
// The slab test is binary32 with one rounding per operation (this file is
// built with FP contraction off) and correctly rounded reciprocals; because
// every inner box is the exact union of its children and each operation is
// monotone in the box bounds, the tree visits exactly the leaves an
// every-leaf test reports, with bit-identical intervals.
#include "launch.h"

namespace nbvh {

struct RayPre {
  float o[3], d[3], inv[3];
  float tmin, tmax;
  bool neg[3];  // the direction's sign bit: the far plane of the slab is lo
};

// inv = 1 / d, also where d is zero (inv = +-inf; see slab).
__device__ inline RayPre load_ray(const nbvh_ray* rays, uint32_t r) {
  const float4* p = (const float4*)(rays + r);
  float4 a = p[0], b = p[1];
  RayPre R;
  R.o[0] = a.x;
  R.o[1] = a.y;
  R.o[2] = a.z;
  R.tmin = a.w;
  R.d[0] = b.x;
  R.d[1] = b.y;
  R.d[2] = b.z;
  R.tmax = b.w;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R.inv[k] = 1.0f / R.d[k];
    R.neg[k] = __float_as_uint(R.d[k]) >> 31;
  }
  return R;
}

// hit iff tn <= tf; axis with zero direction: origin must lie in the slab.
// That case needs no branch: inv is +-inf, so (plane - o) * inv is -inf or
// +inf by the side of the plane the origin lies on (the interval is left
// alone or made empty) and NaN when the origin lies on the plane, which
// fmaxf / fminf ignore (the plane counts as inside).
// REV (reversed inside queries): `inside` is set when the ray's line enters
// the box before tmin (entry te = the largest near-plane distance) and the
// box is hit, i.e. the origin lies in the box; the interval is then the chord
// [te, tf] instead of [tmin, tf].
template <bool REV>
__device__ inline bool slab(const RayPre& R, const float lo[3], const float hi[3], float& t0, float& t1,
                            bool& inside) {
  float tn = R.tmin, tf = R.tmax, te = -INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float ta = (lo[a] - R.o[a]) * R.inv[a];
    const float tb = (hi[a] - R.o[a]) * R.inv[a];
    const float tnear = R.neg[a] ? tb : ta, tfar = R.neg[a] ? ta : tb;
    tn = fmaxf(tn, tnear);
    if (REV) te = fmaxf(te, tnear);
    tf = fminf(tf, tfar);
  }
  const bool hit = tn <= tf;
  inside = REV && hit && te < R.tmin;
  t0 = inside ? te : tn;
  t1 = tf;
  return hit;
}

// leaf field of a segment: the leaf id, with NBVH_SEG_INSIDE for a reversed chord
__device__ inline uint32_t seg_leaf(int32_t leaf, bool inside) {
  return (uint32_t)leaf | (inside ? NBVH_SEG_INSIDE : 0u);
}

// Walk the tree; Emit(leaf, t0, t1, inside) is called for every leaf crossed. The
// per-lane stack lives in LDS, entry i of this lane at stk[i * stride]
// (lane-contiguous, so a wave's pushes and pops touch consecutive words);
// it needs as many entries as the tree has inner levels.
template <bool REV, typename Emit>
__device__ inline void walk(const Node* __restrict__ nodes, const RayPre& R, Emit emit, int32_t* stk,
                            uint32_t stride) {
  int sp = 0;
  int32_t node = 0;
  while (true) {
    const float4* p = (const float4*)(nodes + node);
    float4 q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
    const float lo0[3] = {q0.x, q0.y, q0.z}, hi0[3] = {q0.w, q1.x, q1.y};
    const float lo1[3] = {q1.z, q1.w, q2.x}, hi1[3] = {q2.y, q2.z, q2.w};
    const int32_t c0 = __float_as_int(q3.x), c1 = __float_as_int(q3.y);
    float a0, a1, b0, b1;
    bool ia = false, ib = false;
    bool h0 = slab<REV>(R, lo0, hi0, a0, a1, ia);
    bool h1 = (c1 != kEmptyChild) && slab<REV>(R, lo1, hi1, b0, b1, ib);
    int32_t next = -1;
    if (h0) {
      if (c0 < 0) emit(~c0, a0, a1, ia);
      else next = c0;
    }
    if (h1) {
      if (c1 < 0) {
        emit(~c1, b0, b1, ib);
      } else if (next < 0) {
        next = c1;
      } else {
        // both inner children: go to the nearer one first
        if (b0 < a0) {
          stk[(sp++) * stride] = next;
          next = c1;
        } else {
          stk[(sp++) * stride] = c1;
        }
      }
    }
    if (next >= 0) {
      node = next;
    } else {
      if (sp == 0) break;
      node = stk[(--sp) * stride];
    }
  }
}

// Wave-coherent walk: the wave visits the union of its live lanes' nodes in
// one order that every lane shares. The node index is uniform, so a visit
// reads the node's 64 bytes once through the scalar cache instead of once per
// lane through the vector memory path; each lane tests both children against
// its own ray, and a child is entered when any lane hits it. The stack is one
// register holding entry i in lane i (pushes select the lane, pops read it),
// at most kMaxDepth < 64 entries. Both children entered: the one nearer along
// the guide direction g first, so that each lane's leaves come out mostly in
// front-to-back order. Must be called by every lane of the wave together.
template <bool REV, typename Emit>
__device__ inline void walk_wave(const Node* __restrict__ nodes, const RayPre& R, bool live, Emit emit, float gx,
                                 float gy, float gz) {
  const int lane = (int)(threadIdx.x & 63);
  int32_t stk = 0;
  int sp = 0;
  int32_t node = 0;
  while (true) {
    const float4* p = (const float4*)(nodes + node);
    float4 q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
    const float lo0[3] = {q0.x, q0.y, q0.z}, hi0[3] = {q0.w, q1.x, q1.y};
    const float lo1[3] = {q1.z, q1.w, q2.x}, hi1[3] = {q2.y, q2.z, q2.w};
    const int32_t c0 = __float_as_int(q3.x), c1 = __float_as_int(q3.y);
    float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
    bool ia = false, ib = false;
    const bool h0 = live && slab<REV>(R, lo0, hi0, a0, a1, ia);
    const bool h1 = live && (c1 != kEmptyChild) && slab<REV>(R, lo1, hi1, b0, b1, ib);
    if (h0 && c0 < 0) emit(~c0, a0, a1, ia);
    if (h1 && c1 < 0) emit(~c1, b0, b1, ib);
    const bool e0 = c0 >= 0 && __ballot(h0) != 0ull;
    const bool e1 = c1 >= 0 && c1 != kEmptyChild && __ballot(h1) != 0ull;
    int32_t next;
    if (e0 && e1) {
      const float k0 = (lo0[0] + hi0[0]) * gx + (lo0[1] + hi0[1]) * gy + (lo0[2] + hi0[2]) * gz;
      const float k1 = (lo1[0] + hi1[0]) * gx + (lo1[1] + hi1[1]) * gy + (lo1[2] + hi1[2]) * gz;
      const bool first1 = __builtin_amdgcn_readfirstlane((int)(k1 < k0)) != 0;
      const int32_t later = first1 ? c0 : c1;
      stk = (lane == sp) ? later : stk;
      ++sp;
      next = first1 ? c1 : c0;
    } else if (e0) {
      next = c0;
    } else if (e1) {
      next = c1;
    } else {
      if (sp == 0) break;
      --sp;
      next = __builtin_amdgcn_readlane(stk, sp);
    }
    node = __builtin_amdgcn_readfirstlane(next);
  }
}

// traverse_mode: 0 = per-lane walk, 1 = wave-coherent walk, 2 = per wave,
// the wave-coherent walk when the wave's rays are coherent: every live
// lane's unit direction within kCoherentDir (max-norm) of the first live
// lane's and its origin within 1/kCoherentOrg of the root box's largest
// extent of that lane's. Coherent rays share most of their nodes: a
// 64-pixel row of a 1920-pixel camera visits 7 % more nodes as a union than
// its slowest lane alone, and the walk per wave is 20-40 % faster on camera
// rays at 1,024 and 16,384 leaves; on scattered bounce rays and on random
// training rays it is 25-75 % slower.
constexpr float kCoherentDir = 0.25f;
constexpr float kCoherentOrg = 32.0f;

__device__ inline float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// Whether this wave walks together, and its guide direction. Called by every
// lane of the wave; lanes without a ray pass live = false.
__device__ inline bool wave_walks(int mode, const Node* __restrict__ nodes, const RayPre& R, bool live, float g[3]) {
  const uint64_t lm = __ballot(live);
  if (mode == 0 || lm == 0ull) return false;
  const int gl = __ffsll((unsigned long long)lm) - 1;
  const float n2 = R.d[0] * R.d[0] + R.d[1] * R.d[1] + R.d[2] * R.d[2];
  const float inv = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
  float dn[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dn[k] = R.d[k] * inv;
    g[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dn[k]), gl));
  }
  if (mode == 1) return true;
  const float4* p = (const float4*)nodes;
  const float4 q0 = p[0], q1 = p[1], q2 = p[2];
  const float ext = fmaxf(fmaxf(fmaxf(q0.w, q2.y) - fminf(q0.x, q1.z), fmaxf(q1.x, q2.z) - fminf(q0.y, q1.w)),
                          fmaxf(q1.y, q2.w) - fminf(q0.z, q2.x));
  float dev = 0.0f;
  if (live) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float og = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(R.o[k]), gl));
      dev = fmaxf(dev, fabsf(dn[k] - g[k]) * (1.0f / kCoherentDir));
      dev = fmaxf(dev, fabsf(R.o[k] - og) * kCoherentOrg / fmaxf(ext, 1e-30f));
    }
  }
  return wave_max(dev) <= 1.0f;
}

// The walk the mode asks for. Called by every lane of the wave (the
// wave-coherent walk needs them all); lanes with live = false emit nothing.
template <bool REV, typename Emit>
__device__ inline void walk_mode(int mode, const Node* __restrict__ nodes, const RayPre& R, bool live, Emit emit,
                                 int32_t* stk, uint32_t stride) {
  float g[3] = {0.f, 0.f, 0.f};
  if (wave_walks(mode, nodes, R, live, g))
    walk_wave<REV>(nodes, R, live, emit, g[0], g[1], g[2]);
  else if (live)
    walk<REV>(nodes, R, emit, stk, stride);
}

// The last record of a sorted run, kept in registers: a segment that sorts
// after it is appended without reading the run back.
struct RunTail {
  float t0 = 0.0f;
  uint32_t tag = 0u;
  __device__ bool before(float t, uint32_t g) const { return t0 < t || (t0 == t && tag < g); }
};

// Staged runs are plane-major: record i of ray r is (leaf, t0, t1) at
// planes 3i, 3i+1, 3i+2 of n_rays floats each, so that neighbouring rays
// (lanes) touch neighbouring words. Insert (tag, t0, t1) into ray r's sorted
// run of k records (order (t0, tag)).
__device__ inline void insert_staged(float* st, size_t plane, uint32_t k, uint32_t tag, float t0, float t1,
                                     RunTail& tail) {
  uint32_t j = k;
  if (k == 0 || tail.before(t0, tag)) {
    tail.t0 = t0;
    tail.tag = tag;
  } else {
    while (j > 0) {
      const float p0 = st[(3 * (j - 1) + 1) * plane];
      const uint32_t pl = __float_as_uint(st[(3 * (j - 1)) * plane]);
      if (p0 > t0 || (p0 == t0 && pl > tag)) {
        st[(3 * j) * plane] = __uint_as_float(pl);
        st[(3 * j + 1) * plane] = p0;
        st[(3 * j + 2) * plane] = st[(3 * (j - 1) + 2) * plane];
        --j;
      } else {
        break;
      }
    }
  }
  st[(3 * j) * plane] = __uint_as_float(tag);
  st[(3 * j + 1) * plane] = t0;
  st[(3 * j + 2) * plane] = t1;
}

// Insert (tag, t0, t1) into ray r's sorted run segs[beg, k) of the queue.
__device__ inline void insert_queue(nbvh_segment* __restrict__ segs, uint32_t beg, uint32_t k, uint32_t r, uint32_t tag,
                                    float t0, float t1, RunTail& tail) {
  uint32_t j = k;
  if (k == beg || tail.before(t0, tag)) {
    tail.t0 = t0;
    tail.tag = tag;
  } else {
    while (j > beg) {
      const nbvh_segment prev = segs[j - 1];
      if (prev.t0 > t0 || (prev.t0 == t0 && prev.leaf > tag)) {
        segs[j] = prev;
        --j;
      } else {
        break;
      }
    }
  }
  segs[j] = nbvh_segment{r, tag, t0, t1};
}

// A ray's precomputed form, or an inert one for lanes without a ray.
__device__ inline RayPre load_ray_or_none(const nbvh_ray* rays, uint32_t r, bool live) {
  if (live) return load_ray(rays, r);
  RayPre R;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R.o[k] = R.d[k] = R.inv[k] = 0.0f;
    R.neg[k] = false;
  }
  R.tmin = 1.0f;
  R.tmax = 0.0f;
  return R;
}

// counts[r] = leaves crossed. If `hits` is given (full query), rays with no
// segment get their miss record here (rays with segments are listed by the
// compaction, at positions from a scan of the counts). If `staging` is
// given, the first kStage segments of ray r are also kept there, sorted, so
// that the compaction after the scan need not walk the tree again.
constexpr uint32_t kStage = 16;
template <bool REV>
__global__ __launch_bounds__(256) void k_traverse_count(const Node* __restrict__ nodes, const nbvh_ray* __restrict__ rays,
                                                        uint32_t n_rays, uint32_t* __restrict__ counts,
                                                        nbvh_hit* __restrict__ hits, float* __restrict__ staging,
                                                        int mode, const uint32_t* __restrict__ perm) {
  extern __shared__ int32_t s_stack[];
  // thread i takes ray perm[i] (ray i without a ray order); its staged run
  // is column i, so a wave's staging stores stay coalesced
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < n_rays;
  const uint32_t r = (perm && live) ? perm[i] : i;
  uint32_t cnt = 0;
  RunTail tail;
  const RayPre R = load_ray_or_none(rays, r, live);
  float* run = (staging && live) ? staging + i : nullptr;
  walk_mode<REV>(
      mode, nodes, R, live,
      [&](int32_t leaf, float t0, float t1, bool inside) {
        if (run && cnt < kStage) insert_staged(run, n_rays, cnt, seg_leaf(leaf, inside), t0, t1, tail);
        ++cnt;
      },
      s_stack + threadIdx.x, blockDim.x);
  if (live) {
    counts[r] = cnt;
    if (hits && cnt == 0) {
      float4* h = (float4*)(hits + r);
      h[0] = make_float4(0.f, 0.f, 0.f, 0.f);
      h[1] = make_float4(0.f, 0.f, 0.f, __uint_as_float(NBVH_MISS));
    }
  }
}

// Compaction from the staging runs: rays with more than kStage segments walk
// the tree again and insert their segments into the queue directly. A wave
// whose rays all have short runs copies them together: its runs are one
// contiguous range of the queue, each lane records in LDS which (lane, run
// record) fills each slot of the range, then the lanes take consecutive
// slots, so the stores are coalesced and the wave waits on two or three
// rounds of loads instead of its longest run's.
constexpr uint32_t kWaveSlots = 64 * kStage;
template <bool REV>
__global__ __launch_bounds__(256) void k_traverse_compact(const Node* __restrict__ nodes,
                                                          const nbvh_ray* __restrict__ rays, uint32_t n_rays,
                                                          const uint32_t* __restrict__ offsets,
                                                          const float* __restrict__ staging,
                                                          nbvh_segment* __restrict__ segs, uint64_t capacity, int mode,
                                                          const uint32_t* __restrict__ inv,
                                                          const uint32_t* __restrict__ apos,
                                                          uint32_t* __restrict__ active) {
  extern __shared__ int32_t s_stack[];
  __shared__ uint16_t s_slot[4][kWaveSlots];
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if ((uint64_t)offsets[n_rays] > capacity) return;  // overflow flagged by the scan (uniform)
  const uint32_t beg = r < n_rays ? offsets[r] : 0u, end = r < n_rays ? offsets[r + 1] : 0u;
  // the rays with segments at their positions among them (in ray order, or
  // in the order the counting pass followed)
  if (active && end > beg) active[apos[inv ? inv[r] : r]] = r;
  const bool live = end - beg > kStage;
  const size_t plane = n_rays;
  if (__ballot(live) == 0ull) {
    const uint32_t lane = threadIdx.x & 63u, r0 = r - lane;
    if (r0 >= n_rays) return;  // the whole wave
    const uint32_t wbeg = offsets[r0], wend = offsets[min(r0 + 64u, n_rays)];  // wend - wbeg <= kWaveSlots
    uint16_t* slot = s_slot[threadIdx.x >> 6];
    for (uint32_t i = 0; i < end - beg; ++i) slot[beg - wbeg + i] = (uint16_t)(lane | (i << 6));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t k = lane; k < wend - wbeg; k += 64u) {
      const uint32_t e = slot[k], o = r0 + (e & 63u), i = e >> 6;
      const float* run = staging + (inv ? inv[o] : o);
      segs[wbeg + k] = nbvh_segment{o, __float_as_uint(run[(3 * i) * plane]), run[(3 * i + 1) * plane],
                                    run[(3 * i + 2) * plane]};
    }
    return;
  }
  if (end > beg && !live) {
    const float* run = staging + (inv ? inv[r] : r);
    for (uint32_t i = 0; i < end - beg; ++i)
      segs[beg + i] = nbvh_segment{r, __float_as_uint(run[(3 * i) * plane]), run[(3 * i + 1) * plane],
                                   run[(3 * i + 2) * plane]};
  }
  const RayPre R = load_ray_or_none(rays, r, live);
  uint32_t k = beg;
  RunTail tail;
  walk_mode<REV>(
      mode, nodes, R, live,
      [&](int32_t leaf, float t0, float t1, bool inside) {
        // the counting pass found end - beg leaves along this ray; a walk
        // reports the same ones (every inner box is the union of its
        // children's), the bound keeps the writes inside the run regardless
        if (k < end) insert_queue(segs, beg, k, r, seg_leaf(leaf, inside), t0, t1, tail);
        ++k;
      },
      s_stack + threadIdx.x, blockDim.x);
}

// Training-ray selection (Sec. 5.2, "Ray distribution"): each ray trains only
// the first leaf it crosses (smallest t0, ties to the lower leaf id), and that
// leaf is kept with probability accept[leaf] (kept iff u[r] < accept[leaf]).
// Every leaf a ray crosses also counts one hit towards its hit-probability
// estimate (Sec. 5.1, "Node error"). Kept segments are appended in wave order.
template <bool REV>
__global__ __launch_bounds__(256) void k_first_hits(const Node* __restrict__ nodes, const nbvh_ray* __restrict__ rays,
                                                    uint32_t n, const float* __restrict__ u,
                                                    const float* __restrict__ accept, nbvh_probe* __restrict__ probes,
                                                    uint32_t* __restrict__ leaf_out, uint32_t* __restrict__ n_out,
                                                    uint32_t* __restrict__ leaf_hits, int mode) {
  extern __shared__ int32_t s_stack[];
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = r < n;
  bool take = false, b_in = false;
  int32_t best = -1;
  float b0 = 0.f, b1 = 0.f;
  const RayPre R = load_ray_or_none(rays, r, live);
  walk_mode<REV>(
      mode, nodes, R, live,
      [&](int32_t leaf, float t0, float t1, bool inside) {
        if (leaf_hits) atomicAdd(&leaf_hits[leaf], 1u);
        if (best < 0 || t0 < b0 || (t0 == b0 && leaf < best)) {
          best = leaf;
          b0 = t0;
          b1 = t1;
          b_in = inside;
        }
      },
      s_stack + threadIdx.x, blockDim.x);
  take = live && best >= 0 && u[r] < accept[best];
  const uint64_t mask = __ballot(take);
  if (mask) {
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(n_out, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (take) {
      const uint32_t k = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
      float4* p = (float4*)(probes + k);
      if (b_in) {  // the chord crossed backwards from its exit point
        p[0] = make_float4(R.o[0], R.o[1], R.o[2], -b1);
        p[1] = make_float4(-R.d[0], -R.d[1], -R.d[2], -b0);
      } else {
        p[0] = make_float4(R.o[0], R.o[1], R.o[2], b0);
        p[1] = make_float4(R.d[0], R.d[1], R.d[2], b1);
      }
      leaf_out[k] = (uint32_t)best;
    }
  }
}

// LDS for the walk stacks of a 256-thread workgroup
static size_t stack_lds(const LaunchCtx& L) { return (size_t)256 * (L.stack_depth > 0 ? L.stack_depth : 1) * 4; }

nbvh_status launch_first_hits(const LaunchCtx& L, const nbvh_ray* rays, uint32_t n, const float* u,
                              const float* accept, nbvh_probe* probes, uint32_t* leaf_out, uint32_t* n_out,
                              uint32_t* leaf_hits) {
  k_zero_u32<<<1, 64, 0, L.stream>>>(n_out, 1);
  if (n > 0)
    (L.cfg.inside_reverse ? k_first_hits<true> : k_first_hits<false>)<<<(n + 255) / 256, 256, stack_lds(L), L.stream>>>(
        L.nodes, rays, n, u, accept, probes, leaf_out, n_out, leaf_hits, L.tune.traverse_mode);
  return check_launch("first_hits");
}

// ---------------------------------------------------------------------------
// exclusive scan of uint32 counts (3 kernels: tile scan, scan of tile sums,
// add). Tile = 256 threads x 4 items.
// ---------------------------------------------------------------------------
constexpr int kScanItems = 4;
constexpr int kScanTile = 256 * kScanItems;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // inclusive scan within the wave
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  uint32_t wsum = 0, tot = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wave) wsum += sh[w];
    tot += sh[w];
  }
  __syncthreads();
  total = tot;
  return wsum + x - v;
}

__global__ __launch_bounds__(256) void k_scan_tiles(const uint32_t* __restrict__ in, uint32_t n, uint32_t* __restrict__ out,
                                                    uint32_t* __restrict__ tile_sums) {
  __shared__ uint32_t sh[8];
  const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems], s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_scan(s, sh, total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// one block: exclusive scan of the tile sums in place; total -> *total_out
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t* __restrict__ sums, uint32_t n_tiles,
                                                    uint32_t* __restrict__ total_out) {
  __shared__ uint32_t sh[16];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < n_tiles; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t v = (i < n_tiles) ? sums[i] : 0u;
    uint32_t total;
    uint32_t ex = block_exclusive_scan(v, sh, total);
    const uint32_t c0 = carry;
    if (i < n_tiles) sums[i] = ex + c0;
    __syncthreads();
    if (threadIdx.x == 0) carry = c0 + total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t* __restrict__ out, uint32_t n, const uint32_t* __restrict__ sums,
                                                  const uint32_t* __restrict__ total, uint64_t capacity,
                                                  DevState* __restrict__ state) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / kScanTile];
  if (i == 0) {
    const uint32_t t = *total;
    out[n] = t;
    if (state) {
      state->last_n_segments = t;
      if ((uint64_t)t > capacity) atomicOr(&state->flags, NBVH_FLAG_CAPACITY);
    }
  }
}

// The traversal's two scans at once: segment offsets of the counts and, for
// the active-ray list, positions among the rays with a segment (tile scans,
// one block per scan of the tile sums, add; the totals go to total_seg and
// total_ray).
// (positions follow the ray order `perm` when one is given: pos[i] is the
// place of ray perm[i])
__global__ __launch_bounds__(256) void k_scan2_tiles(const uint32_t* __restrict__ in, uint32_t n,
                                                     const uint32_t* __restrict__ perm, uint32_t* __restrict__ out,
                                                     uint32_t* __restrict__ pos, uint32_t* __restrict__ sums_seg,
                                                     uint32_t* __restrict__ sums_ray) {
  __shared__ uint32_t sh[8];
  const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems], g[kScanItems], s = 0, f = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const bool ok = base + i < n;
    v[i] = ok ? in[base + i] : 0u;
    g[i] = ok ? ((perm ? in[perm[base + i]] : v[i]) > 0u ? 1u : 0u) : 0u;
    s += v[i];
    f += g[i];
  }
  uint32_t total_s, total_f;
  uint32_t ex = block_exclusive_scan(s, sh, total_s);
  uint32_t ef = block_exclusive_scan(f, sh, total_f);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) {
      out[base + i] = ex;
      pos[base + i] = ef;
    }
    ex += v[i];
    ef += g[i];
  }
  if (threadIdx.x == 0) {
    sums_seg[blockIdx.x] = total_s;
    sums_ray[blockIdx.x] = total_f;
  }
}

__global__ __launch_bounds__(1024) void k_scan2_sums(uint32_t* __restrict__ sums_seg, uint32_t* __restrict__ sums_ray,
                                                     uint32_t n_tiles, uint32_t* __restrict__ total_seg,
                                                     uint32_t* __restrict__ total_ray) {
  __shared__ uint32_t sh[16];
  __shared__ uint32_t carry;
  uint32_t* sums = blockIdx.x == 0 ? sums_seg : sums_ray;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < n_tiles; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t v = (i < n_tiles) ? sums[i] : 0u;
    uint32_t total;
    uint32_t ex = block_exclusive_scan(v, sh, total);
    const uint32_t c0 = carry;
    if (i < n_tiles) sums[i] = ex + c0;
    __syncthreads();
    if (threadIdx.x == 0) carry = c0 + total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *(blockIdx.x == 0 ? total_seg : total_ray) = carry;
}

__global__ __launch_bounds__(256) void k_scan2_add(uint32_t* __restrict__ out, uint32_t* __restrict__ pos, uint32_t n,
                                                   const uint32_t* __restrict__ sums_seg,
                                                   const uint32_t* __restrict__ sums_ray,
                                                   const uint32_t* __restrict__ total_seg,
                                                   const uint32_t* __restrict__ total_ray, uint64_t capacity,
                                                   DevState* __restrict__ state) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    out[i] += sums_seg[i / kScanTile];
    pos[i] += sums_ray[i / kScanTile];
  }
  if (i == 0) {
    const uint32_t t = *total_seg;
    out[n] = t;
    pos[n] = *total_ray;
    if (state) {
      state->last_n_segments = t;
      if ((uint64_t)t > capacity) atomicOr(&state->flags, NBVH_FLAG_CAPACITY);
    }
  }
}

// ---------------------------------------------------------------------------
// Grouping of training probes by leaf: a stable least-significant-digit radix
// sort of the leaf ids, 4 bits per pass over the bits that ids below the leaf
// count use, then one gather of the probes. Each pass counts every block's
// 256 keys per digit (digit-major, so one exclusive scan gives every
// (digit, block) its first output slot) and scatters them, a key's rank
// among its block's equal digits taken from wave ballots in element order.
constexpr int kGroupDigits = 16;
static inline size_t group_a256(size_t x) { return (x + 255) & ~(size_t)255; }

__global__ __launch_bounds__(256) void k_group_count(const uint32_t* __restrict__ keys, uint32_t n, int shift,
                                                     uint32_t* __restrict__ counts) {
  __shared__ uint32_t wc[4][kGroupDigits];
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t d = i < n ? (keys[i] >> shift) & (kGroupDigits - 1) : (uint32_t)kGroupDigits;
#pragma unroll
  for (uint32_t q = 0; q < (uint32_t)kGroupDigits; ++q) {
    const uint64_t m = __ballot(d == q);
    if (lane == 0) wc[wave][q] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < kGroupDigits) {
    const int q = threadIdx.x;
    counts[(size_t)q * gridDim.x + blockIdx.x] = wc[0][q] + wc[1][q] + wc[2][q] + wc[3][q];
  }
}

// vals == nullptr: the values are the element indices (first pass)
__global__ __launch_bounds__(256) void k_group_scatter(const uint32_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ vals, uint32_t n, int shift,
                                                       const uint32_t* __restrict__ offs,
                                                       uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t wc[4][kGroupDigits];
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool ok = i < n;
  const uint32_t key = ok ? keys[i] : 0u;
  const uint32_t d = ok ? (key >> shift) & (kGroupDigits - 1) : (uint32_t)kGroupDigits;
  uint64_t mine = 0ull;
#pragma unroll
  for (uint32_t q = 0; q < (uint32_t)kGroupDigits; ++q) {
    const uint64_t m = __ballot(d == q);
    if (lane == 0) wc[wave][q] = (uint32_t)__popcll(m);
    if (d == q) mine = m;
  }
  __syncthreads();
  if (ok) {
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wc[w][d];
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint32_t dst = offs[(size_t)d * gridDim.x + blockIdx.x] + before + (uint32_t)__popcll(mine & below);
    keys_out[dst] = key;
    vals_out[dst] = vals ? vals[i] : i;
  }
}

__global__ __launch_bounds__(256) void k_group_gather(const nbvh_probe* __restrict__ in,
                                                      const uint32_t* __restrict__ perm,
                                                      const uint32_t* __restrict__ keys, uint32_t n,
                                                      nbvh_probe* __restrict__ out, uint32_t* __restrict__ ids_out) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const float4* src = (const float4*)(in + perm[i]);
  float4* dst = (float4*)(out + i);
  dst[0] = src[0];
  dst[1] = src[1];
  if (ids_out) ids_out[i] = keys[i];
}

size_t group_ws_bytes(uint64_t n) {
  const uint64_t nb = (n + 255) / 256, cells = nb * kGroupDigits;
  return 4 * group_a256(n * 4) + group_a256((cells + 1) * 4) * 2 + group_a256((cells / kScanTile + 2) * 4) + 256;
}

nbvh_status launch_exclusive_scan(hipStream_t s, const uint32_t* in, uint32_t n, uint32_t* out, uint32_t* sums,
                                  uint32_t* total_out);

nbvh_status launch_group_by_leaf(const LaunchCtx& L, uint32_t n_leaves, const nbvh_probe* in, const uint32_t* ids,
                                 uint32_t n, nbvh_probe* out, uint32_t* ids_out, void* ws) {
  if (n == 0) return NBVH_OK;
  const uint32_t nb = (n + 255) / 256, cells = nb * kGroupDigits;
  char* w = (char*)ws;
  uint32_t* kbuf[2];
  uint32_t* vbuf[2];
  size_t off = 0;
  for (int j = 0; j < 2; ++j) {
    kbuf[j] = (uint32_t*)(w + off);
    off += group_a256((size_t)n * 4);
    vbuf[j] = (uint32_t*)(w + off);
    off += group_a256((size_t)n * 4);
  }
  uint32_t* counts = (uint32_t*)(w + off);
  off += group_a256(((size_t)cells + 1) * 4);
  uint32_t* offs = (uint32_t*)(w + off);
  off += group_a256(((size_t)cells + 1) * 4);
  uint32_t* sums = (uint32_t*)(w + off);
  off += group_a256(((size_t)cells / kScanTile + 2) * 4);
  uint32_t* total = (uint32_t*)(w + off);
  const int bits = n_leaves > 1 ? 32 - __builtin_clz(n_leaves - 1) : 1;
  const int passes = (bits + 3) / 4;
  const uint32_t* kin = ids;
  const uint32_t* vin = nullptr;
  for (int p = 0; p < passes; ++p) {
    k_group_count<<<nb, 256, 0, L.stream>>>(kin, n, 4 * p, counts);
    nbvh_status s = launch_exclusive_scan(L.stream, counts, cells, offs, sums, total);
    if (s != NBVH_OK) return s;
    k_group_scatter<<<nb, 256, 0, L.stream>>>(kin, vin, n, 4 * p, offs, kbuf[p & 1], vbuf[p & 1]);
    kin = kbuf[p & 1];
    vin = vbuf[p & 1];
  }
  k_group_gather<<<nb, 256, 0, L.stream>>>(in, vin, kin, n, out, ids_out);
  return check_launch("group_by_leaf");
}

// ---------------------------------------------------------------------------
nbvh_status launch_exclusive_scan(hipStream_t s, const uint32_t* in, uint32_t n, uint32_t* out, uint32_t* sums,
                                  uint32_t* total_out) {
  const uint32_t n_tiles = (n + kScanTile - 1) / kScanTile;
  if (n > 0) k_scan_tiles<<<n_tiles, 256, 0, s>>>(in, n, out, sums);
  k_scan_sums<<<1, 1024, 0, s>>>(sums, n_tiles, total_out);
  k_scan_add<<<n > 0 ? (n + 255) / 256 : 1, 256, 0, s>>>(out, n, sums, total_out, 0, nullptr);
  return check_launch("scan");
}

size_t traverse_staging_bytes(uint64_t n_rays) { return (size_t)n_rays * kStage * 3 * sizeof(float); }

// Ray order (tuning query_order): a permutation of the rays by a Morton key,
// built before the traversal so that the counting pass takes the rays in that
// order (its waves, and the active list it fills, hold neighbouring rays)
// while every ray keeps its index. Keys are relative to the box of the ray
// origins (a min/max reduction first). Order 1: the origin's cell on a 256^3
// grid (24 bits). Order 2: five coordinates at 6 bits each (30 bits), the
// origin's cell on a 64^3 grid and the direction's cell on a 64^2 grid of its
// octahedral map.
__device__ inline uint32_t spread8(uint32_t v) {
  v = (v | (v << 8)) & 0x00F00Fu;
  v = (v | (v << 4)) & 0x0C30C3u;
  v = (v | (v << 2)) & 0x249249u;
  return v;
}

__device__ inline uint32_t cell_of(float x, float cells) {
  const float y = x * cells;
  return y > 0.0f ? (uint32_t)fminf(y, cells - 1.0f) : 0u;  // NaN -> 0
}

// order-preserving map of floats to unsigned integers
__device__ inline uint32_t float_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// min / max of the ray origins per axis (as float_key), one partial per
// block, then one block folds the partials
__device__ inline void wave_minmax(uint32_t lo[3], uint32_t hi[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo[a] = min(lo[a], (uint32_t)__shfl_xor((int)lo[a], off));
      hi[a] = max(hi[a], (uint32_t)__shfl_xor((int)hi[a], off));
    }
  }
}

__global__ __launch_bounds__(256) void k_origin_box(const nbvh_ray* __restrict__ rays, uint32_t n,
                                                    uint32_t* __restrict__ part) {
  __shared__ uint32_t red[4][6];
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
  if (i < n) {
    const float4 o = *(const float4*)(rays + i);
    const float p[3] = {o.x, o.y, o.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = float_key(p[a]);
  }
  wave_minmax(lo, hi);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      red[wave][a] = lo[a];
      red[wave][3 + a] = hi[a];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    uint32_t v = red[0][threadIdx.x];
    for (int w = 1; w < 4; ++w)
      v = threadIdx.x < 3 ? min(v, red[w][threadIdx.x]) : max(v, red[w][threadIdx.x]);
    part[(size_t)blockIdx.x * 6 + threadIdx.x] = v;
  }
}

__global__ __launch_bounds__(256) void k_origin_box_fold(const uint32_t* __restrict__ part, uint32_t n_parts,
                                                         uint32_t* __restrict__ box) {
  __shared__ uint32_t red[4][6];
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
  for (uint32_t b = threadIdx.x; b < n_parts; b += 256u)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = min(lo[a], part[(size_t)b * 6 + a]);
      hi[a] = max(hi[a], part[(size_t)b * 6 + 3 + a]);
    }
  wave_minmax(lo, hi);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      red[wave][a] = lo[a];
      red[wave][3 + a] = hi[a];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    uint32_t v = red[0][threadIdx.x];
    for (int w = 1; w < 4; ++w)
      v = threadIdx.x < 3 ? min(v, red[w][threadIdx.x]) : max(v, red[w][threadIdx.x]);
    box[threadIdx.x] = v;
  }
}

// key of ray idx[i] (ray i without a list); entries at or past *n_valid (when
// given) get the largest key, so a stable sort keeps them behind the others
__global__ __launch_bounds__(256) void k_order_keys(const nbvh_ray* __restrict__ rays, const uint32_t* __restrict__ idx,
                                                    const uint32_t* __restrict__ n_valid, uint32_t n,
                                                    const uint32_t* __restrict__ box, int order,
                                                    uint32_t* __restrict__ keys) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  if (n_valid && i >= *n_valid) {
    keys[i] = 0xFFFFFFFFu;
    return;
  }
  const float4* p = (const float4*)(rays + (idx ? idx[i] : i));
  const float4 o = p[0];
  const float ov[3] = {o.x, o.y, o.z};
  float org[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = key_float(box[a]), hi = key_float(box[3 + a]);
    org[a] = hi > lo ? (ov[a] - lo) / (hi - lo) : 0.0f;
  }
  uint32_t key = 0u;
  if (order == 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) key |= spread8(cell_of(org[a], 256.0f)) << a;
  } else {
    const float4 d = p[1];
    // octahedral map of the direction onto [-1, 1]^2
    const float l1 = fabsf(d.x) + fabsf(d.y) + fabsf(d.z);
    float u = l1 > 0.0f ? d.x / l1 : 0.0f, v = l1 > 0.0f ? d.y / l1 : 0.0f;
    if (d.z < 0.0f) {
      const float uu = (1.0f - fabsf(v)) * (u >= 0.0f ? 1.0f : -1.0f);
      v = (1.0f - fabsf(u)) * (v >= 0.0f ? 1.0f : -1.0f);
      u = uu;
    }
    const uint32_t q[5] = {cell_of(org[0], 64.0f), cell_of(org[1], 64.0f), cell_of(org[2], 64.0f),
                           cell_of(0.5f * (u + 1.0f), 64.0f), cell_of(0.5f * (v + 1.0f), 64.0f)};
#pragma unroll
    for (int b = 0; b < 6; ++b)
#pragma unroll
      for (int k = 0; k < 5; ++k) key |= ((q[k] >> b) & 1u) << (5 * b + k);
  }
  keys[i] = key;
}

__global__ __launch_bounds__(256) void k_invert(const uint32_t* __restrict__ perm, uint32_t n,
                                                uint32_t* __restrict__ inv) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) inv[perm[i]] = i;
}

size_t ray_order_bytes(uint64_t n) { return group_ws_bytes(n); }

// Sorts n (key, value) pairs by key with the stable 4-bit radix passes that
// group training probes by leaf (values = the indices when vin is null); the
// keys come from k_order_keys in the workspace's second key buffer. Returns
// the sorted values: `vout` when given (written by the last pass), else a
// workspace buffer. `box` receives the ray origins' box first.
struct OrderWs {
  uint32_t *kbuf[2], *vbuf[2], *counts, *offs, *sums, *total, *box;
};

static OrderWs order_ws(void* ws, uint32_t n) {
  const uint32_t nb = (n + 255) / 256, cells = nb * kGroupDigits;
  char* w = (char*)ws;
  OrderWs O;
  size_t off = 0;
  for (int j = 0; j < 2; ++j) {
    O.kbuf[j] = (uint32_t*)(w + off);
    off += group_a256((size_t)n * 4);
    O.vbuf[j] = (uint32_t*)(w + off);
    off += group_a256((size_t)n * 4);
  }
  O.counts = (uint32_t*)(w + off);
  off += group_a256(((size_t)cells + 1) * 4);
  O.offs = (uint32_t*)(w + off);
  off += group_a256(((size_t)cells + 1) * 4);
  O.sums = (uint32_t*)(w + off);
  off += group_a256(((size_t)cells / kScanTile + 2) * 4);
  O.total = (uint32_t*)(w + off);  // then the origin box (6 words) in the same 256 bytes
  O.box = O.total + 16;
  return O;
}

static nbvh_status sort_rays(const LaunchCtx& L, const nbvh_ray* rays, const uint32_t* idx, const uint32_t* n_valid,
                             uint32_t n, int order, const OrderWs& O, uint32_t* vout, const uint32_t** sorted) {
  const uint32_t nb = (n + 255) / 256, cells = nb * kGroupDigits;
  // the origins' box over all rays; its per-block partials use the digit counts' space
  k_origin_box<<<nb, 256, 0, L.stream>>>(rays, n, O.counts);
  k_origin_box_fold<<<1, 256, 0, L.stream>>>(O.counts, nb, O.box);
  k_order_keys<<<nb, 256, 0, L.stream>>>(rays, idx, n_valid, n, O.box, order, O.kbuf[1]);
  const int passes = order == 1 ? 6 : 8;  // 24- or 30-bit keys
  const uint32_t* kin = O.kbuf[1];
  const uint32_t* vin = idx;
  for (int p = 0; p < passes; ++p) {
    uint32_t* vo = (p == passes - 1 && vout) ? vout : O.vbuf[p & 1];
    k_group_count<<<nb, 256, 0, L.stream>>>(kin, n, 4 * p, O.counts);
    nbvh_status s = launch_exclusive_scan(L.stream, O.counts, cells, O.offs, O.sums, O.total);
    if (s != NBVH_OK) return s;
    k_group_scatter<<<nb, 256, 0, L.stream>>>(kin, vin, n, 4 * p, O.offs, O.kbuf[p & 1], vo);
    kin = O.kbuf[p & 1];
    vin = vo;
  }
  *sorted = vin;
  return NBVH_OK;
}

// The permutation (grouped queries: one order for every object).
nbvh_status launch_ray_order(const LaunchCtx& L, const nbvh_ray* rays, uint32_t n, int order, void* ws,
                             RayOrder* out) {
  out->perm = out->inv = nullptr;
  if (n == 0 || order == 0) return NBVH_OK;
  const OrderWs O = order_ws(ws, n);
  const uint32_t* perm = nullptr;
  nbvh_status s = sort_rays(L, rays, nullptr, nullptr, n, order, O, nullptr, &perm);
  if (s != NBVH_OK) return s;
  uint32_t* inv = O.kbuf[0];  // free after the last pass, which read it and wrote kbuf[1]
  k_invert<<<(n + 255) / 256, 256, 0, L.stream>>>(perm, n, inv);
  out->perm = perm;
  out->inv = inv;
  return check_launch("ray order");
}

// The active list of one object's query, reordered in place after the
// counting pass (the pass keeps the rays' own order, so its loads and
// stores stay coalesced; only the evaluation follows the key order).
static nbvh_status order_active_list(const LaunchCtx& L, const nbvh_ray* rays, uint32_t n, uint32_t* active,
                                     const uint32_t* n_active, int order, void* ws) {
  const uint32_t* sorted = nullptr;
  return sort_rays(L, rays, active, n_active, n, order, order_ws(ws, n), active, &sorted);
}

nbvh_status launch_traverse(const LaunchCtx& L, const nbvh_ray* rays, uint32_t n_rays, uint32_t* offsets,
                            nbvh_segment* segs, uint64_t capacity, nbvh_hit* hits, uint32_t* active,
                            uint32_t* n_active, uint32_t* scratch_counts, uint32_t* scratch_sums,
                            uint32_t* scratch_total, float* staging, const RayOrder* order,
                            void* active_order_ws, uint32_t* scratch_pos, uint32_t* scratch_sums2) {
  if (segs && !staging) return set_error("traversal staging buffer missing"), NBVH_ERR_INVALID_ARG;
  if (active && (!n_active || !segs || !scratch_pos || !scratch_sums2))
    return set_error("active-ray list without its buffers"), NBVH_ERR_INVALID_ARG;
  ProfScope ps(L.prof, NBVH_K_TRAVERSE, L.stream);
  const int grid = (int)((n_rays + 255) / 256);
  if (n_active) {
    k_zero_u32<<<1, 64, 0, L.stream>>>(n_active, 9);  // n_active and the query's 8 ray-queue counters
  }
  if (n_rays > 0)
    (L.cfg.inside_reverse ? k_traverse_count<true> : k_traverse_count<false>)<<<grid, 256, stack_lds(L), L.stream>>>(
        L.nodes, rays, n_rays, scratch_counts, hits, segs ? staging : nullptr, L.tune.traverse_mode,
        order ? order->perm : nullptr);
  const uint32_t n_tiles = (n_rays + kScanTile - 1) / kScanTile;
  if (active) {
    // offsets and the active-list positions in one set of scan launches
    if (n_rays > 0)
      k_scan2_tiles<<<n_tiles, 256, 0, L.stream>>>(scratch_counts, n_rays, order ? order->perm : nullptr, offsets,
                                                   scratch_pos, scratch_sums, scratch_sums2);
    k_scan2_sums<<<2, 1024, 0, L.stream>>>(scratch_sums, scratch_sums2, n_tiles, scratch_total, n_active);
    k_scan2_add<<<grid > 0 ? grid : 1, 256, 0, L.stream>>>(offsets, scratch_pos, n_rays, scratch_sums, scratch_sums2,
                                                           scratch_total, n_active, capacity, L.state);
  } else {
    if (n_rays > 0) k_scan_tiles<<<n_tiles, 256, 0, L.stream>>>(scratch_counts, n_rays, offsets, scratch_sums);
    k_scan_sums<<<1, 1024, 0, L.stream>>>(scratch_sums, n_tiles, scratch_total);
    k_scan_add<<<grid > 0 ? grid : 1, 256, 0, L.stream>>>(offsets, n_rays, scratch_sums, scratch_total, capacity,
                                                          L.state);
  }
  if (segs && n_rays > 0)
    (L.cfg.inside_reverse ? k_traverse_compact<true> : k_traverse_compact<false>)<<<grid, 256, stack_lds(L),
                                                                                     L.stream>>>(
        L.nodes, rays, n_rays, offsets, staging, segs, capacity, L.tune.traverse_mode, order ? order->inv : nullptr,
        active ? scratch_pos : nullptr, active);
  if (active_order_ws && active && n_rays > 0 && L.tune.query_order != 0) {
    nbvh_status s = order_active_list(L, rays, n_rays, active, n_active, L.tune.query_order, active_order_ws);
    if (s != NBVH_OK) return s;
  }
  return check_launch("traverse");
}

}  // namespace nbvh
