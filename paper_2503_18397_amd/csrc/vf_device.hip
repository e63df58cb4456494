// gfx950 kernels of the epsilon-cost sharded VFunc / VFilter (S. Vigna,
// arXiv 2503.18397): signature hashing and shard bucketing (section 4), the
// per-shard fuse-graph construction (section 4.2) with round-synchronous
// peeling and Gaussian elimination of the 2-core over GF(2) (sections 3.3,
// 4.2, 4.3), reverse-order assignment (section 4.3) and the three-probe
// query (eq. (MWHC)).
//
// Definitions every kernel follows (the library's reading of the paper):
//  * signature = (fin(key ^ k_hi), fin(key ^ k_lo)) with fin the SplitMix64
//    finalizer and (k_hi, k_lo, k_fp) the first three SplitMix64 outputs
//    from the user seed;
//  * shard = top h bits of the first word; segment g = (F * l) >> 32
//    (fixed-point inversion) with F the 32 bits right below the shard bits
//    for local seed t = 0 and the top 32 bits of the offset word for t > 0
//    (a retry draws a new graph, segments included);
//  * offsets = three sigma-bit fields of the offset word: the second word
//    (local seed t = 0) or fin(second word + t * golden gamma) (t > 0);
//  * fingerprint = top b bits of fin(hi ^ lo ^ k_fp);
//  * MWHC (section 4.1): three parts of `part` vertices, vertex i the
//    fixed-point image of the i-th 21-bit field of the offset word; an
//    attempt that does not peel completely fails (peel-only);
//  * peeling is round-synchronous (degrees frozen at the start of a round,
//    hinge = first degree-one vertex of the edge);
//  * the 2-core system gets its lexicographically smallest solution
//    (vertex 0 most significant): the pivot of every row is its highest
//    vertex and free vertices are zero.  The elimination below visits
//    columns from the top of the shard down, so every pivot row it emits
//    already has its highest vertex as pivot; any pivot choice among the
//    candidate rows leads to the same solution.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>

#include "vf_launch.h"

// Workspace of the allocation-free grouped filter query: one copy per
// device (each GPU the library runs on holds it until the process ends).
// Host code never passes this name to a kernel: it stands for the array
// only on the device; the host uses the address hipGetSymbolAddress gives
// for the current device (noalloc_scratch below).
static __device__ __align__(256) uint8_t scratch[vfk::kNoAllocScratchBytes];

// Stage clocks (a build with -DVF_STAGE_CLOCKS only): per build workgroup,
// 100 MHz wall-clock ticks spent in each stage of k_build, read back by
// vf_stage_clocks.  Slots: see kClk* in vf_launch.h.
#ifdef VF_STAGE_CLOCKS
static __device__ unsigned long long stage_clk[vfk::kClkWGs * vfk::kClkSlots];
#define VF_CLK(v) const uint64_t v = wall_clock64()
#define VF_CLKV(v) uint64_t v = wall_clock64()
#define VF_CLK_SET(v) v = wall_clock64()
#define VF_CLK_ADD(slot, ticks)                                                        \
  do {                                                                                 \
    if (lane_id() == 0 && blockIdx.x < vfk::kClkWGs)                                   \
      atomicAdd(&stage_clk[blockIdx.x * vfk::kClkSlots + (slot)],                      \
                (unsigned long long)(ticks));                                          \
  } while (0)
#define VF_CLK_MAX(slot, ticks)                                                        \
  do {                                                                                 \
    if (lane_id() == 0 && blockIdx.x < vfk::kClkWGs)                                   \
      atomicMax(&stage_clk[blockIdx.x * vfk::kClkSlots + (slot)],                      \
                (unsigned long long)(ticks));                                          \
  } while (0)
#else
#define VF_CLK(v)
#define VF_CLKV(v)
#define VF_CLK_SET(v)
#define VF_CLK_ADD(slot, ticks)
#define VF_CLK_MAX(slot, ticks)
#endif

namespace vfk {

hipError_t stage_clocks(uint64_t *out, int reset) {
#ifdef VF_STAGE_CLOCKS
  static const unsigned long long zero[kClkWGs * kClkSlots] = {};
  if (reset) return hipMemcpyToSymbol(HIP_SYMBOL(stage_clk), zero, sizeof(zero));
  return hipMemcpyFromSymbol(out, HIP_SYMBOL(stage_clk), sizeof(zero));
#else
  (void)out;
  (void)reset;
  return hipErrorNotSupported;
#endif
}

hipError_t noalloc_scratch(void **ptr, uint64_t *bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kNoAllocScratchBytes;
  return hipSuccess;
}

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

__device__ __forceinline__ uint64_t fin64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t shard_of(uint64_t hi, uint32_t h) {
  return h ? (uint32_t)(hi >> (64 - h)) : 0u;
}

// Fuse 3-graph edge of a signature: one vertex in each of the segments
// g, g + 1, g + 2 of the shard.
// MWHC (section 4.1): one vertex in each of three parts, the fixed-point
// image of a 21-bit field of the offset word.
__device__ __forceinline__ void edge3(const Geo &G, uint64_t hi, uint64_t lo,
                                      uint32_t t, uint32_t &v0, uint32_t &v1,
                                      uint32_t &v2) {
  if (G.mwhc) {
    const uint64_t L = t ? fin64(lo + (uint64_t)t * kGamma) : lo, p = G.part;
    v0 = (uint32_t)(((L & 0x1FFFFFull) * p) >> 21);
    v1 = (uint32_t)(p + ((((L >> 21) & 0x1FFFFFull) * p) >> 21));
    v2 = (uint32_t)(2 * p + ((((L >> 42) & 0x1FFFFFull) * p) >> 21));
    return;
  }
  const uint64_t L = t ? fin64(lo + (uint64_t)t * kGamma) : lo;
  const uint32_t F = t ? (uint32_t)(L >> 32) : (uint32_t)((hi << G.h) >> 32);
  uint32_t g = __umulhi(F, G.l);
  uint32_t s = 1u << G.sigma, m = s - 1;
  v0 = g * s + ((uint32_t)L & m);
  v1 = (g + 1) * s + ((uint32_t)(L >> G.sigma) & m);
  v2 = (g + 2) * s + ((uint32_t)(L >> (2 * G.sigma)) & m);
}

__device__ __forceinline__ uint64_t fingerprint(const Geo &G, uint64_t hi, uint64_t lo) {
  uint64_t f = fin64(hi ^ lo ^ G.kfp);
  return G.b >= 64 ? f : f >> (64 - G.b);
}

// Packed edge: three 21-bit vertices (cells per shard < 2^21).
__device__ __forceinline__ uint64_t pack3(uint32_t a, uint32_t b, uint32_t c) {
  return (uint64_t)a | ((uint64_t)b << 21) | ((uint64_t)c << 42);
}
__device__ __forceinline__ void unpack3(uint64_t e, uint32_t v[3]) {
  v[0] = (uint32_t)(e & 0x1FFFFF);
  v[1] = (uint32_t)((e >> 21) & 0x1FFFFF);
  v[2] = (uint32_t)(e >> 42);
}

// ---------------------------------------------------------------- helpers

// Orders LDS traffic between the lanes of one wavefront (the LDS serves a
// wavefront's instructions in order; this only stops compiler reordering).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Also waits for the wavefront's global-memory stores, for data exchanged
// between lanes through global memory.
__device__ __forceinline__ void wave_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Two 16-bit lanes of one register (packed saturating arithmetic).
typedef int16_t ss2 __attribute__((ext_vector_type(2)));

// Cross-lane reductions with DPP (VALU only, no LDS round trip): within each
// row of 16 lanes quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror
// and row_mirror leave the row's total in every lane.  For the idempotent
// reductions (or, min) row_bcast:15 (into rows 1 and 3) and row_bcast:31
// (into rows 2 and 3) then carry the lower rows' totals up, so lane 63 holds
// the wavefront's; the sum combines the rows from lanes 0, 16, 32 and 48.
#define VF_DPP(x, ctrl, id) __builtin_amdgcn_update_dpp((id), (x), (ctrl), 0xF, 0xF, false)
#define VF_BCAST(x, ctrl, rows) __builtin_amdgcn_update_dpp((x), (x), (ctrl), (rows), 0xF, false)
constexpr int kQuadSwap1 = 0xB1, kQuadSwap2 = 0x4E, kRowHalfMirror = 0x141, kRowMirror = 0x140;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

__device__ __forceinline__ uint32_t readlane(uint32_t x, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}
// Lane `lane` of old set to a value the wavefront holds alike (the LLVM
// intrinsic behind v_writelane_b32, which has no clang builtin).
extern "C" __device__ int vf_writelane_i32(int, int, int) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ uint32_t writelane(uint32_t old, uint32_t val, uint32_t lane) {
  return (uint32_t)vf_writelane_i32((int)val, (int)lane, (int)old);
}
// A value the whole wavefront holds alike, kept in a scalar register.
__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t readlane64(uint64_t x, int lane) {
  return (uint64_t)readlane((uint32_t)x, lane) | ((uint64_t)readlane((uint32_t)(x >> 32), lane) << 32);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
  x += VF_DPP(x, kQuadSwap1, 0u);
  x += VF_DPP(x, kQuadSwap2, 0u);
  x += VF_DPP(x, kRowHalfMirror, 0u);
  x += VF_DPP(x, kRowMirror, 0u);
  return readlane(x, 0) + readlane(x, 16) + readlane(x, 32) + readlane(x, 48);
}

__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
  x |= VF_DPP(x, kQuadSwap1, 0u);
  x |= VF_DPP(x, kQuadSwap2, 0u);
  x |= VF_DPP(x, kRowHalfMirror, 0u);
  x |= VF_DPP(x, kRowMirror, 0u);
  x |= (uint32_t)VF_BCAST(x, kRowBcast15, 0xA);
  x |= (uint32_t)VF_BCAST(x, kRowBcast31, 0xC);
  return readlane(x, 63);
}

__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
  x = min(x, (uint32_t)VF_DPP(x, kQuadSwap1, 0xFFFFFFFFu));
  x = min(x, (uint32_t)VF_DPP(x, kQuadSwap2, 0xFFFFFFFFu));
  x = min(x, (uint32_t)VF_DPP(x, kRowHalfMirror, 0xFFFFFFFFu));
  x = min(x, (uint32_t)VF_DPP(x, kRowMirror, 0xFFFFFFFFu));
  x = min(x, (uint32_t)VF_BCAST(x, kRowBcast15, 0xA));
  x = min(x, (uint32_t)VF_BCAST(x, kRowBcast31, 0xC));
  return readlane(x, 63);
}

// Number of set bits of mask in lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Reserve one slot per lane with pred in a list whose length lives in LDS;
// every lane of the wave must call it.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t *counter) {
  uint64_t mask = __ballot(pred);
  if (mask == 0) return 0;
  uint32_t lane = lane_id();
  int leader = __ffsll((long long)mask) - 1;
  uint32_t base = 0;
  if ((int)lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = readlane(base, leader);
  return base + lanes_below(mask);
}

// ------------------------------------------------------------ small kernels

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Problem 1 stores b-bit values: flag (bit 0 of *flag) any value with a bit
// at or above b.  Values of one structure share b.
__global__ void k_check_values(const uint64_t *__restrict__ vals, uint64_t n, uint32_t b,
                               uint32_t *flag) {
  uint64_t bad = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    bad |= vals[i] >> b;
  if (__ballot(bad != 0) && lane_id() == 0) atomicOr(flag, 1u);
}

// The same for a batch: workgroup i checks the values of instances i,
// i + gridDim.x, ... against their own b.
__global__ void k_check_batch_values(const BatchItem *__restrict__ items, uint64_t count,
                                     const uint64_t *__restrict__ vals, uint32_t *flag) {
  uint64_t bad = 0;
  for (uint64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const BatchItem I = items[it];
    if (I.b >= 64) continue;
    for (uint32_t i = threadIdx.x; i < I.n; i += blockDim.x) bad |= vals[I.key_off + i] >> I.b;
  }
  if (__ballot(bad != 0) && lane_id() == 0) atomicOr(flag, 1u);
}

constexpr uint32_t kLdsHistMax = 16384;

// Keys per shard (section 4: shard = high signature bits).
__global__ void k_count(const uint64_t *__restrict__ keys, uint64_t n, uint64_t khi,
                        uint32_t h, uint32_t S, uint32_t *__restrict__ counts) {
  extern __shared__ uint32_t hist[];
  const bool lds = S <= kLdsHistMax;
  if (lds) {
    for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) hist[i] = 0;
    __syncthreads();
  }
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t j = shard_of(fin64(keys[i] ^ khi), h);
    if (lds) atomicAdd(&hist[j], 1u);
    else atomicAdd(&counts[j], 1u);
  }
  if (lds) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < S; i += blockDim.x)
      if (hist[i]) atomicAdd(&counts[i], hist[i]);
  }
}

// Exclusive scan of the shard counts (one workgroup) and the largest shard;
// clear (the counts themselves, or null) is zeroed after the scan read it.
__global__ void k_scan(const uint32_t *counts, uint32_t S, uint64_t *__restrict__ offsets,
                       uint64_t *__restrict__ cursor, uint32_t *__restrict__ max_out,
                       uint32_t *clear) {
  __shared__ uint64_t part[1024];
  __shared__ uint32_t mx[1024];
  const uint32_t T = blockDim.x, tid = threadIdx.x;
  const uint32_t per = (S + T - 1) / T;
  const uint32_t lo = tid * per, hi = min(S, lo + per);
  uint64_t sum = 0;
  uint32_t m = 0;
  for (uint32_t i = lo; i < hi; i++) {
    sum += counts[i];
    m = max(m, counts[i]);
  }
  part[tid] = sum;
  mx[tid] = m;
  __syncthreads();
  for (uint32_t d = 1; d < T; d <<= 1) {
    uint64_t add = tid >= d ? part[tid - d] : 0;
    uint32_t mm = tid >= d ? mx[tid - d] : 0;
    __syncthreads();
    part[tid] += add;
    mx[tid] = max(mx[tid], mm);
    __syncthreads();
  }
  uint64_t run = part[tid] - sum;
  for (uint32_t i = lo; i < hi; i++) {
    offsets[i] = run;
    cursor[i] = run;
    run += counts[i];
    if (clear) clear[i] = 0;
  }
  if (tid == T - 1) {
    offsets[S] = part[tid];
    *max_out = mx[tid];
  }
}

constexpr int kScatterThreads = 256;
constexpr int kScatterPer = 16;
constexpr uint32_t kScatterLdsMax = 8192;

// Group keys (and values, or each key's index) by shard: a counting sort
// whose per-workgroup counts reserve each shard's range with one atomic per
// shard.
__global__ void k_scatter(const uint64_t *__restrict__ keys, const uint64_t *__restrict__ vals,
                          uint64_t n, uint64_t khi, uint32_t h, uint32_t S,
                          unsigned long long *__restrict__ cursor,
                          uint64_t *__restrict__ bkeys, uint64_t *__restrict__ bvals,
                          uint32_t *__restrict__ bidx) {
  extern __shared__ uint64_t sbase[];
  uint32_t *cnt = (uint32_t *)(sbase + (S <= kScatterLdsMax ? S : 0));
  const bool lds = S <= kScatterLdsMax;
  const uint64_t chunk = (uint64_t)kScatterThreads * kScatterPer;
  const uint64_t nchunks = (n + chunk - 1) / chunk;
  for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    if (lds) {
      for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) cnt[i] = 0;
      __syncthreads();
    }
    uint32_t js[kScatterPer], rk[kScatterPer];
#pragma unroll
    for (int q = 0; q < kScatterPer; q++) {
      uint64_t i = c * chunk + (uint64_t)q * kScatterThreads + threadIdx.x;
      js[q] = 0xFFFFFFFFu;
      if (i < n) {
        js[q] = shard_of(fin64(keys[i] ^ khi), h);
        if (lds) rk[q] = atomicAdd(&cnt[js[q]], 1u);
      }
    }
    if (lds) {
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < S; j += blockDim.x)
        if (cnt[j]) sbase[j] = atomicAdd(&cursor[j], (unsigned long long)cnt[j]);
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kScatterPer; q++) {
      uint64_t i = c * chunk + (uint64_t)q * kScatterThreads + threadIdx.x;
      if (js[q] != 0xFFFFFFFFu) {
        uint64_t pos = lds ? sbase[js[q]] + rk[q] : atomicAdd(&cursor[js[q]], 1ull);
        bkeys[pos] = keys[i];
        if (vals) bvals[pos] = vals[i];
        if (bidx) bidx[pos] = (uint32_t)i;
      }
    }
    if (lds) __syncthreads();
  }
}

// Grouping of keys by shard (a filter's keys before the build, a chunk of
// queries before answering them) with one global atomic per shard and
// segment.  The keys are cut into contiguous segments, one per workgroup.
// k_count_rows writes each segment's shard histogram as a row and adds it
// to the shard totals; k_scan turns the totals into shard starts;
// k_scatter_rows reserves its segment's run in every shard (one atomic per
// shard), sorts sub-chunks of the segment by shard in LDS, then writes
// every shard's part of the sub-chunk with consecutive lanes (coalesced),
// continuing where the previous sub-chunk's part ended.  The order of keys
// within a shard depends on the order of the reservations; a query key
// carries its index.
constexpr uint32_t kRowThreads = 1024;
constexpr uint32_t kRowBlocksMax = 1024;
constexpr uint32_t kRowSub = 8192;   // keys per sub-chunk staged in LDS
constexpr uint32_t kRowSub2 = 12288; // the same for hashed words with their positions
constexpr uint32_t kRowMaxS = 4096;
constexpr uint32_t kPackMaxS = 2048;  // packed edges stage their shard ids too

// Exclusive prefix sum over the workgroup (threads in order); *total gets
// the sum.  wsum: one LDS word per wavefront.  Every thread must call it.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *wsum, uint32_t *total) {
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t inc = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d);
    if (lane >= (uint32_t)d) inc += y;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (uint32_t i = 0; i < nw; i++) {
    const uint32_t x = wsum[i];
    base += i < w ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

__global__ void __launch_bounds__(kRowThreads) k_count_rows(const uint64_t *__restrict__ keys,
                                                            uint64_t n, uint64_t seg,
                                                            uint64_t khi, uint32_t h, uint32_t S,
                                                            uint32_t *__restrict__ rows,
                                                            uint32_t *__restrict__ totals) {
  extern __shared__ uint32_t hist[];
  for (uint32_t j = threadIdx.x; j < S; j += kRowThreads) hist[j] = 0;
  __syncthreads();
  const uint64_t lo = blockIdx.x * seg, hi = lo < n ? min(n, lo + seg) : lo;
  constexpr int U = 8;  // independent loads in flight per thread
  for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (uint64_t)U * kRowThreads) {
    uint64_t k[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint64_t i = i0 + (uint64_t)u * kRowThreads;
      k[u] = i < hi ? keys[i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (i0 + (uint64_t)u * kRowThreads < hi) atomicAdd(&hist[shard_of(fin64(k[u] ^ khi), h)], 1u);
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < S; j += kRowThreads) {
    const uint32_t c = hist[j];
    rows[(uint64_t)blockIdx.x * S + j] = c;
    if (c) atomicAdd(&totals[j], c);
  }
}

// Queries of a structure with geometry G and local seeds tseed may be
// written hashed, which leaves the answering kernel no hashing to do:
//   MODE 1: the edge and fingerprint, vb bits per vertex:
//           v0 | v1 << vb | v2 << 2 vb | fingerprint << 3 vb (3 vb + b <= 64);
//   MODE 2 (fuse graphs): first segment g (vb bits), the three offsets in
//           segments g, g + 1, g + 2 (sigma bits each), the fingerprint, and
//           in bits 48..63 the key's position in its segment, which then
//           needs no index array (vb + 3 sigma + b <= 48).
__device__ __forceinline__ uint64_t pack_compact(const Geo &G, uint64_t hi, uint64_t lo,
                                                 uint32_t t, uint32_t gb) {
  const uint64_t L = t ? fin64(lo + (uint64_t)t * kGamma) : lo;
  const uint32_t F = t ? (uint32_t)(L >> 32) : (uint32_t)((hi << G.h) >> 32);
  const uint64_t g = __umulhi(F, G.l);
  const uint32_t sg = G.sigma;
  const uint64_t m = (1ull << sg) - 1;
  uint64_t w = g | ((L & m) << gb) | (((L >> sg) & m) << (gb + sg)) |
               (((L >> (2 * sg)) & m) << (gb + 2 * sg));
  if (G.is_filter) w |= fingerprint(G, hi, lo) << (gb + 3 * sg);
  return w;
}

template <int MODE>
__global__ void __launch_bounds__(kRowThreads) k_scatter_rows(
    const uint64_t *__restrict__ keys, uint64_t n, uint64_t seg, uint64_t khi, uint32_t h,
    uint32_t S, const uint32_t *__restrict__ rows, unsigned long long *__restrict__ cursor,
    uint64_t *__restrict__ bkeys, uint32_t *__restrict__ bidx, uint32_t *__restrict__ starts,
    Geo G, const uint8_t *__restrict__ tseed, uint32_t vb) {
  // keys per sub-chunk: mode 2 stages no indices, which leaves LDS for more
  constexpr uint32_t SUB = MODE == 2 ? kRowSub2 : kRowSub;
  extern __shared__ uint64_t skey[];                      // SUB keys (or hashed words)
  uint32_t *const sidx = (uint32_t *)(skey + SUB);        // their indices (not in mode 2)
  uint16_t *const ssh = (uint16_t *)(MODE == 2 ? (uint32_t *)(skey + SUB) : sidx + SUB);  // MODE 1, 2: shards
  uint32_t *const cnt = MODE ? (uint32_t *)(ssh + SUB) : sidx + SUB;  // S: per shard
  uint32_t *const lofs = cnt + S;                         // S: first staged slot
  uint32_t *const wptr = lofs + S;                        // S: next output position
  __shared__ uint32_t wsum[kRowThreads / 64];
  constexpr int KPT = SUB / kRowThreads;
  const uint32_t tid = threadIdx.x;
  const uint64_t lo = blockIdx.x * seg, hi = lo < n ? min(n, lo + seg) : lo;
  for (uint32_t j = tid; j < S; j += kRowThreads) {
    const uint32_t c = rows[(uint64_t)blockIdx.x * S + j];
    wptr[j] = c ? (uint32_t)atomicAdd(&cursor[j], (unsigned long long)c) : 0u;
    if (starts) starts[(uint64_t)blockIdx.x * S + j] = wptr[j];
  }
  const uint32_t per = (S + kRowThreads - 1) / kRowThreads;
  const uint32_t j0 = min(S, tid * per), j1 = min(S, j0 + per);
  // the keys of the next sub-chunk are loaded while this one is sorted
  uint64_t nkey[KPT];
#pragma unroll
  for (int k = 0; k < KPT; k++) {
    const uint64_t i = lo + (uint64_t)k * kRowThreads + tid;
    nkey[k] = i < hi ? keys[i] : 0ull;
  }
  for (uint64_t c = lo; c < hi; c += SUB) {
    for (uint32_t j = tid; j < S; j += kRowThreads) cnt[j] = 0;
    uint64_t key[KPT];
#pragma unroll
    for (int k = 0; k < KPT; k++) {
      key[k] = nkey[k];
      const uint64_t i = c + SUB + (uint64_t)k * kRowThreads + tid;
      nkey[k] = i < hi ? keys[i] : 0ull;
    }
    __syncthreads();
    uint32_t js[KPT], rk[KPT];
#pragma unroll
    for (int k = 0; k < KPT; k++) {
      const uint64_t i = c + (uint64_t)k * kRowThreads + tid;
      js[k] = 0xFFFFFFFFu;
      rk[k] = 0;
      if (i < hi) {
        const uint64_t hk = fin64(key[k] ^ khi);
        js[k] = shard_of(hk, h);
        rk[k] = atomicAdd(&cnt[js[k]], 1u);
        if (MODE == 1) {
          const uint64_t lk = fin64(key[k] ^ G.klo);
          uint32_t v0, v1, v2;
          edge3(G, hk, lk, tseed[js[k]], v0, v1, v2);
          const uint64_t fp = G.is_filter ? fingerprint(G, hk, lk) : 0ull;
          key[k] = (uint64_t)v0 | ((uint64_t)v1 << vb) | ((uint64_t)v2 << (2 * vb)) |
                   (fp << (3 * vb));
        } else if (MODE == 2) {
          key[k] = pack_compact(G, hk, fin64(key[k] ^ G.klo), tseed[js[k]], vb) |
                   ((i - lo) << 48);
        }
      }
    }
    __syncthreads();
    uint32_t s = 0;
    for (uint32_t j = j0; j < j1; j++) s += cnt[j];
    uint32_t tot;
    uint32_t run = block_scan(s, wsum, &tot);
    for (uint32_t j = j0; j < j1; j++) {
      lofs[j] = run;
      run += cnt[j];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KPT; k++)
      if (js[k] != 0xFFFFFFFFu) {
        const uint32_t p = lofs[js[k]] + rk[k];
        skey[p] = key[k];
        if (MODE != 2) sidx[p] = (uint32_t)(c + (uint64_t)k * kRowThreads + tid);
        if (MODE) ssh[p] = (uint16_t)js[k];
      }
    __syncthreads();
    for (uint32_t e = tid; e < tot; e += kRowThreads) {
      const uint64_t x = skey[e];
      const uint32_t j = MODE ? (uint32_t)ssh[e] : shard_of(fin64(x ^ khi), h);
      const uint32_t d = wptr[j] + (e - lofs[j]);
      bkeys[d] = x;
      if (MODE != 2 && bidx) bidx[d] = sidx[e];
    }
    __syncthreads();
    for (uint32_t j = tid; j < S; j += kRowThreads) wptr[j] += cnt[j];
    __syncthreads();
  }
}

// Answers of a chunk grouped by shard (ans, in the order of bkeys) moved to
// their positions.  Workgroup b owns segment b of the chunk, whose keys
// occupy one run in every shard (starts[b][j], rows[b][j] long): its
// wavefronts read the runs of their share of the shards, place each answer
// in an LDS window over the segment's part of out, and the window is
// written out contiguously.
constexpr uint32_t kPlaceLdsMax = 150 * 1024;

__host__ __device__ inline uint32_t place_lds_bytes(uint32_t S, uint64_t seg, uint32_t ob) {
  const uint64_t win = (seg * ob + 15) & ~15ull;
  const uint32_t per_w = (S + kRowThreads / 64 - 1) / (kRowThreads / 64);
  const uint64_t b = win + (uint64_t)(kRowThreads / 64) * 2 * per_w * 4;
  return b <= kPlaceLdsMax ? (uint32_t)b : 0u;
}

// WORD: positions come from bits 48..63 of the grouped words (bwords,
// k_scatter_rows<2>) instead of bidx.
template <typename T, bool WORD>
__global__ void __launch_bounds__(kRowThreads) k_place_rows(
    const uint32_t *__restrict__ rows, const uint32_t *__restrict__ starts, uint32_t S,
    uint64_t n, uint64_t seg, const T *__restrict__ ans, const uint32_t *__restrict__ bidx,
    const uint64_t *__restrict__ bwords, T *__restrict__ out) {
  extern __shared__ uint4 place_lds[];
  constexpr uint32_t nw = kRowThreads / 64;
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t per_w = (S + nw - 1) / nw;
  T *const win = (T *)place_lds;
  uint32_t *const pre = (uint32_t *)((uint8_t *)place_lds + ((seg * sizeof(T) + 15) & ~15ull)) +
                        w * 2 * per_w;
  uint32_t *const beg = pre + per_w;
  const uint64_t lo = blockIdx.x * seg, hi = lo < n ? min(n, lo + seg) : lo;
  const uint32_t j0 = min(S, w * per_w), nj = min(S, j0 + per_w) - j0;
  const uint64_t rb = (uint64_t)blockIdx.x * S + j0;
  // run lengths of this wavefront's shards -> exclusive prefix in LDS
  const uint32_t per_l = (nj + 63) / 64, k0 = min(nj, lane * per_l), k1 = min(nj, k0 + per_l);
  uint32_t sum = 0;
  for (uint32_t k = k0; k < k1; k++) sum += rows[rb + k];
  uint32_t inc = sum;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d);
    if (lane >= (uint32_t)d) inc += y;
  }
  const uint32_t total = __shfl(inc, 63);
  uint32_t run = inc - sum;
  for (uint32_t k = k0; k < k1; k++) {
    pre[k] = run;
    beg[k] = starts[rb + k];
    run += rows[rb + k];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  constexpr int U = 4;  // elements in flight per lane
  for (uint32_t e0 = lane; e0 < total; e0 += 64 * U) {
    uint32_t p[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t e = e0 + 64 * u;
      p[u] = 0xFFFFFFFFu;
      if (e < total) {
        // last shard k with pre[k] <= e (runs of length 0 share a prefix)
        uint32_t a = 0, b = nj - 1;
        while (a < b) {
          const uint32_t m = (a + b + 1) >> 1;
          if (pre[m] <= e) a = m;
          else b = m - 1;
        }
        p[u] = beg[a] + (e - pre[a]);
      }
    }
    T v[U];
    uint32_t i[U];
#pragma unroll
    for (int u = 0; u < U; u++)
      if (p[u] != 0xFFFFFFFFu) {
        v[u] = ans[p[u]];
        i[u] = WORD ? (uint32_t)(bwords[p[u]] >> 48) : (uint32_t)(bidx[p[u]] - lo);
      }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (p[u] != 0xFFFFFFFFu) win[i[u]] = v[u];
  }
  __syncthreads();
  for (uint64_t i = threadIdx.x; i < hi - lo; i += kRowThreads) out[lo + i] = win[i];
}

// ------------------------------------------------------------- shard build
//
// A workgroup of five wavefronts builds shards as a pipeline: one hashes
// and peels the next shard, three eliminate the 2-core of the current one,
// one assigns the cells of a solved one.
// Several workgroups share a CU (as many as the LDS of their elimination
// windows allows).  Vertex state for peeling lives in global memory (cached
// in L2), the elimination window in LDS.

// A shard in flight has a record of its own in global memory (sized for the
// largest shard): its edges, right sides and peeling order (kept for the
// assignment), its 2-core grouped for the elimination and the pivot rows.
struct ShardBufs {
  uint64_t *E;      // packed edges
  uint64_t *R;      // right sides (values or fingerprints)
  uint32_t *stack;  // peeled edges in round order: index | side << 30
  uint32_t *rst;    // round starts in stack
  uint64_t *cE;     // packed edges of the 2-core, grouped by entry group
  uint64_t *cR;     // their right sides
  uint32_t *cb;     // group starts
  uint32_t *poff;   // pivot record offsets
  uint32_t *plog;   // pivot records
};

// Vertex state of the peeling wavefront (one copy per workgroup).  A
// vertex's degree and the sum of the indices of its incident edges share
// one 64-bit word (degree in the high half), updated by one atomic add:
// when one incident edge is left, the sum is its index (section 4.3 keeps
// the xor of the edges for the same purpose; a sum serves as well and
// takes one atomic instead of two).
struct FrontBufs {
  uint64_t *st;      // (degree << 32) + sum of incident edge indices
  uint8_t *pe;       // 1 = edge peeled
  uint32_t *F0, *F1; // frontiers of degree-one vertices
  uint32_t *cc;      // group cursors
};
constexpr uint64_t kDegOne = 1ull << 32;
// Elements per lane in flight in the peel's passes over edges and vertices.
constexpr uint32_t kPU = 4;

// Shard records per workgroup: one being peeled, one being eliminated and
// one being assigned.
constexpr uint32_t kSlots = 3;

__host__ __device__ inline uint64_t align8(uint64_t x) { return (x + 7) & ~7ull; }

// Entries the back-substitution loads with each pivot record's header, all
// of them whatever the record's length: the pivot log has as many words of
// slack after its capacity.
constexpr uint32_t kBackPre = 8;

// Core rows enter the elimination window in groups: the 32 columns of one
// ring word (segments of at least 32 vertices) or one segment (smaller
// segments), keyed by the row's top vertex.
__host__ __device__ inline uint32_t entry_shift(uint32_t sigma) { return sigma < 5 ? sigma : 5; }
__host__ __device__ inline uint64_t max_groups(uint64_t V, uint32_t l) { return (V >> 5) + l + 8; }

// Buffers of one shard record at base (nullptr: sizes only); returns its bytes.
__host__ __device__ inline uint64_t slot_layout(uint8_t *base, uint32_t M, uint64_t V, uint32_t l,
                                               uint32_t logcap, ShardBufs *sb) {
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    uint8_t *p = base ? base + o : nullptr;
    o += align8(bytes);
    return p;
  };
  const uint64_t m = (uint64_t)M + 1;
  ShardBufs t;
  t.E = (uint64_t *)take(8 * m);
  t.R = (uint64_t *)take(8 * m);
  t.stack = (uint32_t *)take(4 * m);
  t.rst = (uint32_t *)take(4 * (m + 2));
  t.cE = (uint64_t *)take(8 * m);
  t.cR = (uint64_t *)take(8 * m);
  t.cb = (uint32_t *)take(4 * max_groups(V, l));
  t.poff = (uint32_t *)take(4 * m);
  t.plog = (uint32_t *)take(4 * ((uint64_t)logcap + kBackPre));
  if (sb) *sb = t;
  return o;
}

// Vertex state of the peeling wavefront at base; returns its bytes.
__host__ __device__ inline uint64_t front_layout(uint8_t *base, uint32_t M, uint64_t V, uint32_t l,
                                                FrontBufs *fb) {
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    uint8_t *p = base ? base + o : nullptr;
    o += align8(bytes);
    return p;
  };
  const uint64_t m = (uint64_t)M + 1;
  FrontBufs f;
  f.st = (uint64_t *)take(8 * V);
  f.pe = (uint8_t *)take(m);
  f.F0 = (uint32_t *)take(4 * V);
  f.F1 = (uint32_t *)take(4 * V);
  f.cc = (uint32_t *)take(4 * max_groups(V, l));
  if (fb) *fb = f;
  return o;
}

// Scratch of one workgroup: kSlots shard records, then the vertex state.
uint64_t build_scratch_bytes(uint32_t M, uint64_t V, uint32_t l, uint32_t logcap) {
  return kSlots * slot_layout(nullptr, M, V, l, logcap, nullptr) +
         front_layout(nullptr, M, V, l, nullptr);
}

// The elimination window stores each row over a ring of vertex positions.
// While segment G is swept a window row only has vertices in segments
// G-2..G, so segments of at least 32 vertices use a ring of 3 segments
// (segment g at position (g mod 3) s); smaller segments use a ring of 4
// segments (vertex v at v mod 4s), at most two words.
struct Ring {
  uint32_t sigma, s, three, words;
  __host__ __device__ explicit Ring(uint32_t sg) : sigma(sg), s(1u << sg), three(sg >= 5) {
    const uint32_t bits = three ? 3u * s : 4u * s;
    words = bits < 32 ? 1u : bits / 32;
  }
  __device__ uint32_t pos(uint32_t v) const {
    return three ? ((v >> sigma) % 3u) * s + (v & (s - 1)) : v & (4u * s - 1);
  }
  // vertex at ring position p of a row in the window of segment Gs
  __device__ uint32_t vertex(uint32_t p, uint32_t Gs) const {
    if (three) {
      const uint32_t d = (Gs % 3u + 3u - (p >> sigma)) % 3u;
      return (Gs - d) * s + (p & (s - 1));
    }
    const uint32_t gbase = Gs >= 2 ? (Gs - 2) * s : 0u, mask = 4u * s - 1;
    return gbase + ((p - (gbase & mask)) & mask);
  }
};

// Rows are stored with a stride of ring words + 1: lanes that read the same
// word of consecutive slots then hit distinct LDS banks.
__host__ __device__ inline uint32_t row_stride(uint32_t sigma) { return Ring(sigma).words + 1; }

// Bytes of one window slot: ring row + rhs (8) + popcount (2) + free-list entry (2).
__host__ __device__ inline uint32_t slot_bytes(uint32_t sigma) { return 4 * row_stride(sigma) + 12; }

constexpr uint32_t kMaxSlots = 512;
constexpr uint32_t kBcolBytes = 256;  // batch columns of the back-substitution

__host__ __device__ inline uint32_t window_slots_for(uint32_t sigma, uint32_t lds_bytes) {
  uint32_t n = (lds_bytes - kLdsTail) / slot_bytes(sigma);
  n = n > kMaxSlots ? kMaxSlots : n;
  return n & ~7u;  // keeps the 8-byte right sides after the rows aligned
}

uint32_t window_slots(uint32_t sigma, uint32_t lds_bytes) {
  return window_slots_for(sigma, lds_bytes);
}

enum { kSolveOk = 0, kSolveInconsistent = 1, kSolveCapacity = 2 };

// A group count known at compile time (the elimination is instantiated per
// count so that its per-group work unrolls without run-time guards).
template <int N> struct Groups { static constexpr int value = N; };

// Control block in LDS shared by the two wavefronts of a build workgroup.
// The pivots found in one 32-column word travel from the eliminating
// wavefront to the emitting one as a batch; the emitter hands the slots of
// the emitted rows back in a return list.  Batches, return lists and the
// abort flags are double-buffered by word parity: an entry written during
// word i is read after the barrier that ends word i and rewritten only
// during word i + 2, after every reader has passed the barrier of word i + 1.
struct BandCtl {
  uint32_t np;                   // pivots emitted
  uint32_t flag[2];              // kSolveInconsistent | kSolveCapacity
  uint32_t adv[2];               // 0: the word is taken again (window full)
  uint32_t k[2], gs[2];          // pivots of each batch and its segment
  uint32_t nq[2];                // slot groups in use during the batch's word
  uint32_t nret[2][2];           // returned slots per batch parity and emitter
  uint32_t bseq;                 // words whose batch wavefront 0 has published
  uint32_t slot[2][32], col[2][32], cm[2][32];
  uint16_t ret[2][2][64];        // slots handed back to the searching wavefront
                                 // (kRetClear: its ring words still need clearing)
};

// Shard records in flight and their states.  Each state has one owner, the
// only wavefront that moves a record on from it: the peeling wavefront
// (free, retry, give-up), the eliminating pair (ready, eliminating) or the
// assigning wavefront (solved).
enum : uint32_t {
  kRecFree = 0,    // unused
  kRecFront = 1,   // being peeled
  kRecReady = 2,   // peeled, its 2-core waits for the elimination
  kRecBand = 3,    // being eliminated
  kRecSolved = 4,  // solved (or no 2-core), waits for the assignment
  kRecRetry = 5,   // the elimination failed: peel again with the next local seed
  kRecGiveUp = 6   // outgrew the window: cells cleared, shard left for a relaunch
};
struct ShardRec {
  uint32_t state;
  uint32_t shard, t;      // work item, local seed of the attempt
  uint32_t m;             // keys
  uint64_t base;          // first key of the item
  uint64_t V, vmask;      // geometry of the item
  uint64_t cells;         // address of the item's cells
  uint32_t l, sigma, b;
  uint32_t core, rounds;  // 2-core rows and peeling rounds of the attempt
  uint32_t np;            // pivots of the solved 2-core
  uint32_t order;         // position in the order records became ready
  uint32_t pad;
};
struct PipeCtl {
  ShardRec rec[kSlots];
  uint32_t fcnt[7];  // list counts of a peel (see the peeling stage)
  uint32_t first[2]; // the workgroup's first work item and its first seed
  uint32_t quit;     // no work is left and every record is free
  uint32_t abort;    // a wait ran out: every wavefront of the workgroup ends
  uint32_t bar[3];   // barriers reached by each eliminating wavefront
  uint32_t pick;     // record the pair eliminates next (kSlots: none left)
};
constexpr uint32_t kPipeOff = (sizeof(BandCtl) + 15) & ~15u;
static_assert(kPipeOff + sizeof(PipeCtl) + kBcolBytes <= kLdsTail, "LDS tail too small");

__device__ __forceinline__ BandCtl *band_ctl(uint8_t *lds, uint32_t lds_bytes) {
  return (BandCtl *)(lds + lds_bytes - kLdsTail);
}
__device__ __forceinline__ PipeCtl *pipe_ctl(uint8_t *lds, uint32_t lds_bytes) {
  return (PipeCtl *)(lds + lds_bytes - kLdsTail + kPipeOff);
}

__device__ __forceinline__ uint32_t lds_load(const uint32_t *p) {
  return uniform(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
}
// Publishes v at p after every earlier memory write of the wavefront.
__device__ __forceinline__ void lds_publish(uint32_t *p, uint32_t v) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if (lane_id() == 0) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void acquire_wg() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup"); }

// Longest wait of a build wavefront, in ticks of the 100 MHz wall clock.
constexpr uint64_t kWaitLimit = 60ull * 100000000ull;

// Waits until ready() (a value uniform across the wavefront) holds.  Every
// wait ends: when another wavefront of the workgroup gave up, this one ends
// too; after kWaitLimit it gives up itself (status kStatusStalled).
template <class F>
__device__ __forceinline__ void wait_for(PipeCtl *pc, uint32_t *work, F &&ready) {
  if (ready()) return;
  const uint64_t t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    if (ready()) return;
    if (lds_load(&pc->abort)) __builtin_amdgcn_endpgm();
    if (wall_clock64() - t0 > kWaitLimit) {
      if (lane_id() == 0) atomicOr(&work[kWorkStatus], kStatusStalled);
      lds_publish(&pc->abort, 1u);
      __builtin_amdgcn_endpgm();
    }
  }
}

// Barrier of the three eliminating wavefronts (the other wavefronts of the
// workgroup run loops of their own, so the workgroup barrier is not
// available): each publishes how many barriers it has reached and waits
// until the other two have reached as many.
__device__ __forceinline__ void band_sync(PipeCtl *pc, uint32_t *work, uint32_t me,
                                          uint32_t &gen) {
  gen++;
  lds_publish(&pc->bar[me], gen);
  const uint32_t g = gen, o1 = me == 0 ? 1u : 0u, o2 = me == 2 ? 1u : 2u;
  wait_for(pc, work, [&] { return min(lds_load(&pc->bar[o1]), lds_load(&pc->bar[o2])) >= g; });
  acquire_wg();
}

// A returned slot whose ring words the searching wavefront clears before
// reusing it (a pivot row another pivot of its batch reads).
constexpr uint16_t kRetClear = 0x8000;

// Gaussian elimination of the 2-core over GF(2) by the two wavefronts of
// the workgroup.  Core rows enter the window when the sweep reaches their
// entry group; columns are visited from the highest vertex down.  For
// column c every window row that contains c is a candidate; one of them
// (fewest nonzeros first: least fill) becomes the pivot row of c and is
// xored into the other candidates.
//
// Wavefront 0 eliminates, one 32-column word at a time.  Slot s of the
// window belongs to its lane s % 64, which keeps the slot's word of the
// current 32 columns, its popcount and its right side in registers;
// candidates, pivot choice and the column mask need no LDS traffic, only
// the row updates do.
//
// Wavefront 1 runs one word behind and appends the pivot rows of the
// previous word to a log: [column, count, rhs lo, rhs hi, vertices below
// the column]; poff[i] is the offset of the i-th (descending column).  A
// pivot row is frozen once chosen, so emitting it overlaps the elimination
// of the next word; its slot returns to wavefront 0 after the emission.
//
// Both wavefronts walk the same sequence of words and meet at one barrier
// per word; the result (kSolve*) and the pivot count are the same in both.
// Xor of word au of the rows of the pivots in the (wavefront-uniform) mask
// cm: rows[pivot slot * mu + au], pivot k's slot in lane k of pivtab.  Four
// loads are in flight at a time.
__device__ __forceinline__ uint32_t xor_rows(const uint32_t *rows, uint32_t pivtab, uint32_t cm,
                                             uint32_t mu, uint32_t au) {
  uint32_t acc = 0;
  while (__popc(cm) >= 4) {
    const uint32_t j0 = __ffs(cm) - 1;
    cm &= cm - 1;
    const uint32_t j1 = __ffs(cm) - 1;
    cm &= cm - 1;
    const uint32_t j2 = __ffs(cm) - 1;
    cm &= cm - 1;
    const uint32_t j3 = __ffs(cm) - 1;
    cm &= cm - 1;
    const uint32_t a0 = rows[__umul24(readlane(pivtab, (int)j0), mu) + au];
    const uint32_t a1 = rows[__umul24(readlane(pivtab, (int)j1), mu) + au];
    const uint32_t a2 = rows[__umul24(readlane(pivtab, (int)j2), mu) + au];
    const uint32_t a3 = rows[__umul24(readlane(pivtab, (int)j3), mu) + au];
    acc ^= (a0 ^ a1) ^ (a2 ^ a3);
  }
  for (; cm; cm &= cm - 1) acc ^= rows[__umul24(readlane(pivtab, (int)(__ffs(cm) - 1)), mu) + au];
  return acc;
}

// wid: 0 searches the pivots, 1 and 2 emit (emitter wid - 1).
template <int QM>
__device__ __forceinline__ int band_solve(const BuildArgs &A, const Geo &G, uint32_t W,
                                          const ShardBufs &sc, uint8_t *lds, BandCtl *ctl,
                                          uint32_t wid, uint32_t *np_out, PipeCtl *pc,
                                          uint32_t &gen) {
  auto psync = [&] { band_sync(pc, A.work, wid, gen); };
  const uint32_t em = wid - 1;  // emitter index (wid != 0)
  uint32_t *const plog = sc.plog;
  uint32_t *const poff = sc.poff;
  const uint32_t *const cb = sc.cb;
  const uint64_t *const cE = sc.cE;
  const uint64_t *const cR = sc.cR;
  const uint32_t logcap = A.logcap;
  const uint32_t lane = lane_id();
  const Ring ring(G.sigma);
  const uint32_t s = ring.s;
  const uint32_t RW = ring.words;
  const uint32_t RS = RW + 1;
  uint32_t *rows = (uint32_t *)lds;
  uint64_t *rrhs = (uint64_t *)(lds + (uint64_t)4 * RS * W);
  uint16_t *rpop = (uint16_t *)(rrhs + W);
  uint16_t *freel = rpop + W;
  const uint32_t NW = (RW + 2 + 63) / 64;  // row words and the right side, per lane
  // Word u of the row in slot x is rows[x * umul(u) + uadd(u)]: words below
  // RW are ring words, words RW and RW + 1 the low and high half of the
  // right side, so one pass over u combines rows and right sides together.
  auto umul = [&](uint32_t u) { return u < RW ? RS : 2u; };
  auto uadd = [&](uint32_t u) { return u < RW ? u : RS * W + (u - RW); };

  // ring words of free slots are kept zero (dead rows are zero, emitted
  // pivot rows are cleared by their emitter or, when another pivot of the
  // batch reads them, by the searching wavefront before reuse), so a row
  // enters by setting its three bits
  for (uint32_t i = wid * 64 + lane; i < W * RS; i += 192) rows[i] = 0;
  // free slots form a stack that hands out low slots first; only slot groups
  // below the high-water mark are ever scanned
  if (wid == 0) {
    for (uint32_t i = lane; i < W; i += 64) {
      rpop[i] = 0;
      freel[i] = (uint16_t)(W - 1 - i);
    }
    if (lane == 0) {
      ctl->flag[0] = ctl->flag[1] = 0;
      ctl->nret[0][0] = ctl->nret[0][1] = ctl->nret[1][0] = ctl->nret[1][1] = 0;
      ctl->k[0] = ctl->k[1] = 0;
      ctl->bseq = 0;
    }
  }
  psync();
  uint32_t nfree = W, NQ = 0;  // searching wavefront
  // each emitter writes its own half of the pivot log
  const uint32_t loglo = wid ? em * (logcap / 2) : 0u, loghi = loglo + logcap / 2;
  uint32_t lp = loglo, np = 0;  // emitters
  const uint32_t gsh = entry_shift(G.sigma);

  // core rows [rb, re) join the window (wavefront 0; re - rb <= nfree)
  // The rows of the next word are loaded while the current word is
  // searched (pre_rb: the first row they hold, ~0: none).
  uint64_t pre_e = 0, pre_r = 0;
  uint32_t pre_rb = 0xFFFFFFFFu;
  auto enter = [&](uint32_t rb, uint32_t re) {
    for (uint32_t r0 = rb; r0 < re; r0 += 64) {
      const uint32_t cnt = min(64u, re - r0);
      const bool pre = r0 == pre_rb;
      if (lane < cnt) {
        const uint64_t e = pre ? pre_e : cE[r0 + lane];
        const uint64_t rhs = pre ? pre_r : cR[r0 + lane];
        const uint32_t slot = freel[nfree - 1 - lane];
        uint32_t v[3];
        unpack3(e, v);
        uint32_t *row = rows + (uint64_t)slot * RS;
        for (int k = 0; k < 3; k++) {
          const uint32_t p = ring.pos(v[k]);
          atomicOr(&row[p >> 5], 1u << (p & 31));
        }
        rrhs[slot] = rhs;
        rpop[slot] = 3;
      }
      nfree -= cnt;
      NQ = max(NQ, (W - nfree + 63) / 64);
      wave_sync();
    }
  };

  // pivot rows of batch bsel with this emitter's parity, last first (a row
  // reads only rows of earlier pivots, none of which is rewritten), their
  // slots into return list rsel; false if the emitter's half of the log is
  // full
  auto emit = [&](uint32_t bsel, uint32_t rsel) -> bool {
    const uint32_t kp = uniform(ctl->k[bsel]), Gs = uniform(ctl->gs[bsel]);
    const uint32_t pivtab = lane < kp ? ctl->slot[bsel][lane] : 0u;
    const uint32_t pivcol = lane < kp ? ctl->col[bsel][lane] : 0u;
    const uint32_t pivcm = lane < kp ? ctl->cm[bsel][lane] : 0u;
    // pivots whose row another pivot of the batch reads (possibly the other
    // emitter's): their slots go back uncleared
    const uint32_t refd = wave_or(pivcm);
    // with segments of 32 or more vertices a ring word lies in one segment:
    // its bit bb is vertex vbase(u) + bb
    auto vbase = [&](uint32_t u) { return ring.three && u < RW ? ring.vertex(u * 32, Gs) : 0u; };
    const uint32_t vb0 = vbase(lane), mu0 = umul(lane), au0 = uadd(lane);
    uint32_t nr = 0;
    // pivot kk; when the row and its right side fit one word per lane
    // (NW == 1), w0 is the lane's word of the pivot's row
    auto one = [&](int kk, uint32_t w0) -> bool {
      const uint32_t x = readlane(pivtab, kk);
      const uint32_t col = readlane(pivcol, kk);
      const uint32_t cmx = readlane(pivcm, kk);
      const uint32_t cb_ = ring.pos(col);
      // a record takes at most 4 + 32 RW words (every ring bit set)
      if (lp + 4 + 32 * RW > loghi) return false;
      uint32_t pos = lp + 4;
      for (uint32_t w = 0; w < NW; w++) {
        const uint32_t u = w * 64 + lane;
        const uint32_t vb = w == 0 ? vb0 : vbase(u);
        uint32_t bits = 0;
        if (u < RW + 2) {
          // the pivot row as it was chosen: its row at the start of the word
          // plus the earlier pivots of the word it absorbed
          const uint32_t mu = w == 0 ? mu0 : umul(u), au = w == 0 ? au0 : uadd(u);
          bits = NW == 1 ? w0 : rows[__umul24(x, mu) + au];
          if (cmx) bits ^= xor_rows(rows, pivtab, cmx, mu, au);
          if (u == (cb_ >> 5)) bits &= ~(1u << (cb_ & 31));
          if (u >= RW) {
            plog[lp + 2 + (u - RW)] = bits;  // right side, low word first
            bits = 0;
          }
        }
        for (;;) {
          const uint64_t m = __ballot(bits != 0);
          if (!m) break;
          if (bits) {
            const uint32_t bb = __ffs(bits) - 1;
            bits &= bits - 1;
            plog[pos + lanes_below(m)] = ring.three ? vb + bb : ring.vertex(u * 32 + bb, Gs);
          }
          pos += (uint32_t)__popcll(m);
        }
      }
      const bool keep = (refd >> kk) & 1u;
      if (!keep)
        for (uint32_t w = 0; w < NW; w++)
          if (w * 64 + lane < RW) rows[x * RS + w * 64 + lane] = 0u;
      if (lane == 0) {
        plog[lp] = col;
        plog[lp + 1] = pos - (lp + 4);
        poff[np + (uint32_t)kk] = lp;
        ctl->ret[rsel][em][nr] = (uint16_t)(x | (keep ? kRetClear : 0u));
      }
      nr++;
      lp = pos;
      return true;
    };
    // this emitter's pivots: kk = em, em + 2, ..., last first
    const int top = (int)kp - 1 - (int)(((kp - 1) ^ em) & 1u);
    if (NW == 1) {
      // the rows of up to eight pivots are loaded together
      const bool in = lane < RW + 2;
      for (int k0 = top; k0 >= 0; k0 -= 16) {
        uint32_t wv[8];
#pragma unroll
        for (int i = 0; i < 8; i++)
          wv[i] = k0 - 2 * i >= 0 && in ? rows[__umul24(readlane(pivtab, k0 - 2 * i), mu0) + au0]
                                       : 0u;
#pragma unroll
        for (int i = 0; i < 8; i++)
          if (k0 - 2 * i >= 0 && !one(k0 - 2 * i, wv[i])) return false;
      }
    } else {
      for (int kk = top; kk >= 0; kk -= 2)
        if (!one(kk, 0u)) return false;
    }
    np += kp;
    if (lane == 0) ctl->nret[rsel][em] = nr;
    return true;
  };

  // Rows absorb this word's pivots through a combination mask (bit k: the
  // row of pivot k as it was when the word started).  A row that becomes
  // zero is dead (inconsistent if its right side is not zero) and frees its
  // slot.  apply() xors the masked pivot rows (slots in lanes of ptab) into
  // row x, right side included; true if the row became zero, rset: its
  // right side is not zero.
  const uint32_t mu_l = umul(lane), au_l = uadd(lane);  // the lane's word (NW == 1)
  auto apply = [&](uint32_t x, uint32_t cmx, uint32_t ptab, bool &rset) -> bool {
    if (NW == 1) {
      const bool in = lane < RW + 2;
      uint32_t acc = 0;
      if (in) {
        const uint32_t xa = __umul24(x, mu_l) + au_l;
        acc = rows[xa] ^ xor_rows(rows, ptab, cmx, mu_l, au_l);
        rows[xa] = acc;
      }
      rset = __ballot(in && lane >= RW && acc != 0) != 0;
      return __ballot(lane < RW && acc != 0) == 0;
    }
    uint32_t any = 0, rany = 0;
    for (uint32_t w = 0; w < NW; w++) {
      const uint32_t u = w * 64 + lane;
      if (u < RW + 2) {
        const uint32_t mu = umul(u), au = uadd(u), xa = __umul24(x, mu) + au;
        const uint32_t acc = rows[xa] ^ xor_rows(rows, ptab, cmx, mu, au);
        rows[xa] = acc;
        if (u < RW) any |= acc;
        else rany |= acc;
      }
    }
    rset = __ballot(rany != 0) != 0;
    return __ballot(any != 0) == 0;
  };

  // Active rows of a word (a bit within the word's columns) are gathered
  // into up to QM register groups in slot order ("compact" index c =
  // group * 64 + lane); csl holds their slots (kNoSlot past the last).
  // The searching wavefront takes the rows whose compact index is below
  // kW0Share mod 8 from its registers; the emitters take the others through
  // the rows' padding words, split by slot parity.
  constexpr uint32_t kNoSlot = 0xFFFFu, kW0Share = 3;
  auto w1share = [](uint32_t c) { return (c & 7u) >= kW0Share; };
  uint32_t csl[QM], ccw[QM], cpop[QM], ccm[QM];
  uint32_t it = 0;
  bool stop = false;
  for (int Gs = (int)G.l + 1; Gs >= 0 && !stop; Gs--) {
    // group starts of this segment, one per lane (readlane per word)
    const uint32_t g0 = gsh == 5 ? ((uint32_t)Gs * s) >> 5 : (uint32_t)Gs;
    const uint32_t ng = gsh == 5 ? s >> 5 : 1u;  // groups (words) in the segment
    const bool cached = ng < 64;
    const uint32_t cbl = wid == 0 && cached && lane <= ng ? cb[g0 + lane] : 0u;
    auto cbv = [&](uint32_t i) { return cached ? readlane(cbl, (int)i) : cb[g0 + i]; };
    const uint32_t segtop = (uint32_t)(Gs + 1) * s - 1, segbot = (uint32_t)Gs * s;
    uint32_t c = segtop;
    for (bool first = true;;) {
      const uint32_t cpos = ring.pos(c), word = cpos >> 5;
      const uint32_t wbase = c - (cpos & 31);  // column of bit 0 of this word
      const uint32_t wlo_col = max(segbot, wbase);
      const uint32_t cur = it & 1u, prev = cur ^ 1u;
      VF_CLK(tw0);
      VF_CLKV(tw1);
      VF_CLKV(tw2);
      VF_CLKV(tw3);
      VF_CLKV(tw4);
      bool incons = false;
      if (wid == 0) {
        // slots emitted during the previous word come back (those marked
        // kRetClear with their ring words cleared here)
        for (uint32_t e2 = 0; e2 < 2; e2++) {
          const uint32_t nr = uniform(ctl->nret[prev][e2]);
          const uint32_t ent = lane < nr ? (uint32_t)ctl->ret[prev][e2][lane] : 0u;
          for (uint64_t fm = __ballot(lane < nr && (ent & kRetClear)); fm; fm &= fm - 1) {
            const uint32_t x = readlane(ent, (int)(__ffsll((long long)fm) - 1)) & ~(uint32_t)kRetClear;
            for (uint32_t w = 0; w < NW; w++)
              if (w * 64 + lane < RW) rows[x * RS + w * 64 + lane] = 0u;
          }
          if (lane < nr) freel[nfree + lane] = (uint16_t)(ent & ~(uint32_t)kRetClear);
          nfree += nr;
        }
        wave_sync();
        // rows whose top vertex is in this word (segment, below 32 vertices)
        uint32_t rb = 0, re = 0;
        if (gsh == 5) {
          const uint32_t wi = (c >> 5) - g0;
          rb = cbv(wi);
          re = cbv(wi + 1);
        } else if (first) {
          rb = cbv(0);
          re = cbv(1);
        }
        uint32_t k = 0, adv = 1;
        bool published = false;
        // the word's batch (pivots, masks, counts) goes to wavefront 1
        auto publish = [&] {
          if (lane == 0) {
            ctl->k[cur] = k;
            ctl->gs[cur] = (uint32_t)Gs;
            ctl->adv[cur] = adv;
            ctl->nq[cur] = NQ;
          }
          lds_publish(&ctl->bseq, it + 1);
          published = true;
        };
        if (re - rb > nfree) {
          // window full: if the previous word's pivot rows are being
          // emitted, wait one word for their slots; otherwise give up
          if (it > 0 && uniform(ctl->k[prev]) > 0) adv = 0;
          else if (lane == 0) atomicOr(&ctl->flag[cur], (uint32_t)kSolveCapacity);
        } else {
          enter(rb, re);
          VF_CLK_SET(tw1);
          // rows of the next word of the segment, loaded ahead
          if (gsh == 5 && wlo_col != segbot) {
            const uint32_t wi2 = ((wlo_col - 1) >> 5) - g0;
            const uint32_t rb2 = cbv(wi2), re2 = cbv(wi2 + 1);
            if (rb2 < re2) {
              pre_rb = rb2;
              if (lane < min(64u, re2 - rb2)) {
                pre_e = cE[rb2 + lane];
                pre_r = cR[rb2 + lane];
              }
            }
          }
          const uint32_t lowbit = wlo_col - wbase, hibit = cpos & 31;
          const uint32_t range = (hibit >= 31 ? 0xFFFFFFFFu : ((2u << hibit) - 1u)) &
                                 ~((1u << lowbit) - 1u);
          // 1. pivots of the word's columns, top down, on the active rows'
          //    words in registers: lane k of pivtab/pivcol/pivcm describes
          //    pivot k (slot, column, mask); bit g of cpiv marks the lane's
          //    row of compact group g as a pivot row.  The pivot row takes
          //    part in its own update (its word becomes zero, so it is never
          //    a candidate again).  Right sides follow in the passes over
          //    whole rows.
          auto search = [&](auto cgroups) {
            constexpr int NC = decltype(cgroups)::value;
            uint32_t pivtab = 0, pivcol = 0, pivcm = 0, cpiv = 0;
            uint32_t orv = 0;
#pragma unroll
            for (int g = 0; g < NC; g++) {
              const bool v = csl[g] != kNoSlot;
              const uint32_t sl = v ? csl[g] : 0u;
              cpop[g] = rpop[sl];
              ccw[g] = rows[(uint64_t)sl * RS + word];
              if (!v) cpop[g] = 0;
              ccw[g] = v ? ccw[g] & range : 0u;
              ccm[g] = 0;
              orv |= ccw[g];
            }
            // key of a row: popcount estimate (high half, below 2^15) and
            // compact index (low half)
            uint32_t key[NC];
#pragma unroll
            for (int g = 0; g < NC; g++) key[g] = (cpop[g] << 16) | ((uint32_t)g * 64 + lane);
            uint32_t colmask = wave_or(orv);
            // One path through the loop body (a column whose rows all lost it
            // finds no pivot and changes nothing), so that the loop carries
            // its registers without copies.
            while (colmask) {
              const uint32_t b = 31 - __clz(colmask), bit = 1u << b;
              // all ones where the row has column b
              uint32_t hm[NC];
#pragma unroll
              for (int g = 0; g < NC; g++) hm[g] = (uint32_t)__builtin_amdgcn_sbfe((int)ccw[g], (int)b, 1);
              uint32_t best = 0xFFFFFFFFu;
#pragma unroll
              for (int g = 0; g < NC; g++) best = min(best, key[g] | ~hm[g]);
              best = wave_min(best);
              const bool found = best != 0xFFFFFFFFu;
              const uint32_t p = best & 0xFFFFu, pg = p >> 6, pl = p & 63u;
              // a row that takes the pivot row: its estimate grows by the
              // pivot's less the two copies of column b (the high half of
              // the key, saturating at 2^15 - 1; the low half is unchanged)
              const ss2 grow = {0, (int16_t)((int32_t)(best >> 16) - 2)};
              uint32_t pw = 0, pcm = 0, ps = 0;
#pragma unroll
              for (int g = 0; g < NC; g++) {
                if ((uint32_t)g == pg) {
                  pw = readlane(ccw[g], (int)pl);
                  pcm = readlane(ccm[g], (int)pl);
                  ps = readlane(csl[g], (int)pl);
                }
              }
              // lane k describes pivot k (written whether or not a pivot was
              // found: lanes from k on are read only once they hold one)
              pivtab = writelane(pivtab, ps, k);
              pivcol = writelane(pivcol, wbase + b, k);
              pivcm = writelane(pivcm, pcm, k);
              cpiv |= found && lane == pl ? 1u << (pg & 31u) : 0u;
              const uint32_t kbit = pcm | (1u << (k & 31u));
#pragma unroll
              for (int g = 0; g < NC; g++) {
                ccw[g] ^= pw & hm[g];
                ccm[g] ^= kbit & hm[g];
                const ss2 nk = __builtin_elementwise_add_sat(__builtin_bit_cast(ss2, key[g]), grow);
                key[g] ^= (key[g] ^ __builtin_bit_cast(uint32_t, nk)) & hm[g];
              }
              k += found ? 1u : 0u;
              // columns below b that may still have rows: the earlier ones
              // and those of the pivot word (a column whose rows all lost
              // it is skipped when visited)
              colmask = (colmask | pw) & (bit - 1u);
            }
#pragma unroll
            for (int g = 0; g < NC; g++) cpop[g] = key[g] >> 16;
            if (k) {
              // popcount estimates back to LDS (zero marks a pivot row, no
              // longer live in the window); padding words: zero for every
              // slot in use, then the masks of wavefront 1's rows
              for (uint32_t q = 0; q < NQ; q++) {
                const uint32_t slot = q * 64 + lane;
                if (slot < W) rows[(uint64_t)slot * RS + RW] = 0u;
              }
#pragma unroll
              for (int g = 0; g < NC; g++) {
                const bool piv = (cpiv >> g) & 1u;
                if (csl[g] != kNoSlot) {
                  rpop[csl[g]] = piv ? (uint16_t)0 : (uint16_t)cpop[g];
                  if (!piv && ccm[g] && w1share((uint32_t)g * 64 + lane))
                    rows[(uint64_t)csl[g] * RS + RW] = ccm[g];
                }
              }
              // the batch for wavefront 1
              if (lane < k) {
                ctl->slot[cur][lane] = pivtab;
                ctl->col[cur][lane] = pivcol;
                ctl->cm[cur][lane] = pivcm;
              }
            }
            publish();
            VF_CLK_SET(tw3);
            // 2. whole rows, wavefront 0's share (see apply)
            if (k) {
#pragma unroll
              for (int g = 0; g < NC; g++) {
                const bool mine = csl[g] != kNoSlot && !((cpiv >> g) & 1u) && ccm[g] != 0 &&
                                  !w1share((uint32_t)g * 64 + lane);
                uint64_t m = __ballot(mine);
                while (m) {
                  const uint32_t xl = (uint32_t)(__ffsll((long long)m) - 1);
                  m &= m - 1;
                  const uint32_t x = readlane(csl[g], (int)xl);
                  bool rset;
                  if (apply(x, readlane(ccm[g], (int)xl), pivtab, rset)) {
                    incons |= rset;
                    if (lane == 0) {
                      rpop[x] = 0;
                      freel[nfree] = (uint16_t)x;
                    }
                    nfree++;
                  }
                }
              }
            }
          };
          // the slot of the c-th active row: each active slot writes itself
          // to position c (its group's offset plus the active lanes below
          // it) in the rows' padding words, which hold nothing between the
          // end of the previous word and this word's masks (the search
          // zeroes them for every slot in use before writing masks, and the
          // emitters read them only for a word with pivots)
          auto compact = [&](auto groups) -> uint32_t {
            constexpr int NG = decltype(groups)::value;
            // every group's state loads before the first position is written
            // (the writes go to the same rows array)
            bool a[NG];
#pragma unroll
            for (int q = 0; q < NG; q++) {
              const uint32_t slot = (uint32_t)q * 64 + lane;
              const uint32_t sl = slot < W ? slot : 0u;
              const uint32_t pop = rpop[sl], wd = rows[(uint64_t)sl * RS + word];
              a[q] = slot < W && pop != 0 && (wd & range) != 0;
            }
            uint32_t off = 0;
#pragma unroll
            for (int q = 0; q < NG; q++) {
              const uint64_t act = __ballot(a[q]);
              if (a[q]) rows[(uint64_t)(off + lanes_below(act)) * RS + RW] = (uint32_t)q * 64 + lane;
              off += (uint32_t)__popcll(act);
            }
            const uint32_t na = off, nc = (na + 63) >> 6;
            wave_sync();
#pragma unroll
            for (int g = 0; g < QM; g++) {
              const uint32_t ci = (uint32_t)g * 64 + lane;
              csl[g] = (uint32_t)g < nc && ci < na ? rows[(uint64_t)ci * RS + RW] : kNoSlot;
            }
            return nc;
          };
          uint32_t nc = 0;
          switch (uniform(NQ)) {
            case 1: nc = compact(Groups<1>{}); break;
            case 2: nc = compact(Groups<2>{}); break;
            case 3: nc = compact(Groups<3>{}); break;
            case 4: nc = compact(Groups<4>{}); break;
            case 5: nc = compact(Groups<5>{}); break;
            case 6: nc = compact(Groups<6>{}); break;
            case 7: if constexpr (QM >= 7) nc = compact(Groups<7>{}); break;
            case 8: if constexpr (QM >= 8) nc = compact(Groups<8>{}); break;
            default: break;
          }
          VF_CLK_SET(tw2);
          switch (uniform(nc)) {
            case 1: search(Groups<1>{}); break;
            case 2: search(Groups<2>{}); break;
            case 3: search(Groups<3>{}); break;
            case 4: search(Groups<4>{}); break;
            case 5: search(Groups<5>{}); break;
            case 6: search(Groups<6>{}); break;
            case 7: if constexpr (QM >= 7) search(Groups<7>{}); break;
            case 8: if constexpr (QM >= 8) search(Groups<8>{}); break;
            default: break;
          }
        }
        if (!published) publish();
        VF_CLK_SET(tw4);
      } else {
        VF_CLK_SET(tw1);
        if (it == 0) {
          if (lane == 0) ctl->nret[cur][em] = 0;
        } else if (!emit(prev, cur)) {
          if (lane == 0) {
            ctl->nret[cur][em] = 0;
            atomicOr(&ctl->flag[cur], (uint32_t)kSolveCapacity);
          }
        }
        // this word's batch from wavefront 0
        VF_CLK_SET(tw2);
        const uint32_t want = it + 1;
        wait_for(pc, A.work, [&] { return lds_load(&ctl->bseq) >= want; });
        acquire_wg();
        // 2. whole rows, the emitters' share: rows whose padding word holds
        //    a mask, this emitter's slot parity
        if (const uint32_t kc = uniform(ctl->k[cur])) {
          const uint32_t ptab = lane < kc ? ctl->slot[cur][lane] : 0u;
          const uint32_t nq = uniform(ctl->nq[cur]);
          uint32_t nr = uniform(ctl->nret[cur][em]);
          for (uint32_t q = 0; q < nq; q++) {
            const uint32_t slot = q * 64 + lane;
            const uint32_t cmv = slot < W ? rows[(uint64_t)slot * RS + RW] : 0u;
            uint64_t m = __ballot(cmv != 0 && (slot & 1u) == em);
            while (m) {
              const uint32_t xl = (uint32_t)(__ffsll((long long)m) - 1);
              m &= m - 1;
              const uint32_t x = q * 64 + xl;
              bool rset;
              if (apply(x, readlane(cmv, (int)xl), ptab, rset)) {
                incons |= rset;
                if (lane == 0) {
                  rpop[x] = 0;
                  if (nr < 64) ctl->ret[cur][em][nr] = (uint16_t)x;
                }
                nr = nr < 64 ? nr + 1 : nr;  // beyond 64 a dead slot stays taken
              }
            }
          }
          if (lane == 0) ctl->nret[cur][em] = nr;
        }
        VF_CLK_SET(tw3);
        VF_CLK_SET(tw4);
      }
      if (incons && lane == 0) atomicOr(&ctl->flag[cur], (uint32_t)kSolveInconsistent);
      VF_CLK(tw5);
      psync();
#ifdef VF_STAGE_CLOCKS
      if (wid != 2) {
        const uint32_t o = wid == 0 ? kClkSearch : kClkEmit;
        VF_CLK_ADD(o + 0, tw1 - tw0);
        VF_CLK_ADD(o + 1, tw2 - tw1);
        VF_CLK_ADD(o + 2, tw3 - tw2);
        VF_CLK_ADD(o + 3, tw4 - tw3);
        VF_CLK_ADD(o + 4, tw5 - tw4);
        VF_CLK_ADD(o + 5, wall_clock64() - tw5);
        VF_CLK_ADD(o + 6, 1);
      }
#endif
      it++;
      if (uniform(ctl->flag[cur])) {
        stop = true;
        break;
      }
      if (!uniform(ctl->adv[cur])) continue;
      first = false;
      if (wlo_col == segbot) break;
      c = wlo_col - 1;
    }
  }
  uint32_t fl;
  if (stop) {
    fl = uniform(ctl->flag[(it - 1) & 1u]);
  } else {
    // the pivots of the last word
    const uint32_t cur = it & 1u, prev = cur ^ 1u;
    if (wid != 0) {
      if (it > 0 && !emit(prev, cur) && lane == 0)
        atomicOr(&ctl->flag[cur], (uint32_t)kSolveCapacity);
      if (wid == 1 && lane == 0) ctl->np = np;
    }
    psync();
    fl = uniform(ctl->flag[cur]);
  }
  *np_out = uniform(ctl->np);
  if (fl & kSolveInconsistent) return kSolveInconsistent;
  return fl ? kSolveCapacity : kSolveOk;
}

// Xor of a 64-bit value over the wavefront, in every lane.
__device__ __forceinline__ uint64_t wave_xor64(uint64_t x) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, d);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), d);
    x ^= (uint64_t)lo | ((uint64_t)hi << 32);
  }
  return x;
}

// Xor and or of a 64-bit value over the wavefront, in every lane (the DPP
// row steps, then the four rows' totals); every lane must take part.
__device__ __forceinline__ uint64_t wave_xor64_total(uint64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  lo ^= VF_DPP(lo, kQuadSwap1, 0u);
  hi ^= VF_DPP(hi, kQuadSwap1, 0u);
  lo ^= VF_DPP(lo, kQuadSwap2, 0u);
  hi ^= VF_DPP(hi, kQuadSwap2, 0u);
  lo ^= VF_DPP(lo, kRowHalfMirror, 0u);
  hi ^= VF_DPP(hi, kRowHalfMirror, 0u);
  lo ^= VF_DPP(lo, kRowMirror, 0u);
  hi ^= VF_DPP(hi, kRowMirror, 0u);
  lo = readlane(lo, 0) ^ readlane(lo, 16) ^ readlane(lo, 32) ^ readlane(lo, 48);
  hi = readlane(hi, 0) ^ readlane(hi, 16) ^ readlane(hi, 32) ^ readlane(hi, 48);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ uint64_t wave_or64_total(uint64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  lo |= VF_DPP(lo, kQuadSwap1, 0u);
  hi |= VF_DPP(hi, kQuadSwap1, 0u);
  lo |= VF_DPP(lo, kQuadSwap2, 0u);
  hi |= VF_DPP(hi, kQuadSwap2, 0u);
  lo |= VF_DPP(lo, kRowHalfMirror, 0u);
  hi |= VF_DPP(hi, kRowHalfMirror, 0u);
  lo |= VF_DPP(lo, kRowMirror, 0u);
  hi |= VF_DPP(hi, kRowMirror, 0u);
  lo = readlane(lo, 0) | readlane(lo, 16) | readlane(lo, 32) | readlane(lo, 48);
  hi = readlane(hi, 0) | readlane(hi, 16) | readlane(hi, 32) | readlane(hi, 48);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Back-substitution of the pivot log (records [column, count, rhs lo, rhs
// hi, vertices below the column], poff[i] the i-th in decreasing column
// order): from the lowest pivot up, 64 pivots at a time, the value of a
// pivot column is its right side xor the values of its record's vertices.
// Vertices below the batch have their final values; a vertex inside the
// batch's range is a pivot column of the batch (a dependency, resolved in
// lane order) or free (value 0).
//
// Loads run ahead of their use: the next batch's record headers with their
// first kBackPre entries (read whole: the pivot log has kBackPre words of
// slack) and the offsets of the batch after it load while the current
// batch gathers.  The longer records are gathered by the whole wavefront,
// 64 entries per step, each step's entries loading while the step before
// is combined (the first step's from before the end of the previous batch).
//
// With ring (LDS, rl cells: a power of two up to kRing, kRing but for test
// builds), the values of the columns up to rl below the batch are kept
// there too: most of a record's vertices lie within three segments below
// its column, so with 3 s + 64 <= rl nearly every
// gather is an LDS read and a batch waits for no global store of the batch
// before it.  A vertex farther down (records grown by elimination) is read
// from the cells after the wavefront's stores have completed.  The columns
// between consecutive pivots (free or outside the 2-core) are cleared in
// the ring as the sweep passes them.  While a batch that spans fewer than
// rl / 2 columns gathers, the slots of its own columns hold the lane of
// each of its pivots, so a dependency takes two LDS reads (the lane, then
// its column to confirm) instead of a binary search over the batch.
constexpr uint32_t kRing = kRingCols;
// LDS of the ring for cells of T (none for 8-byte cells, whose ring would
// cost the window too many slots).
template <typename T>
__host__ __device__ constexpr uint32_t ring_bytes() {
  return sizeof(T) <= 4 ? kRing * (uint32_t)sizeof(T) : 0u;
}
template <typename T, bool kTestRing>
__device__ __forceinline__ void back_substitute(const ShardBufs &sc, uint32_t np, T *wl,
                                                uint32_t *bcol, T *ring, uint32_t ring_cols) {
  // a compile-time ring length but for test builds
  const uint32_t rl = kTestRing ? ring_cols : kRing;
  constexpr uint32_t kPre = kBackPre;
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const uint32_t lane = lane_id();
  const uint32_t *const plog = sc.plog;
  const uint32_t *const poff = sc.poff;
  auto load_off = [&](uint32_t bs) -> uint32_t {
    const uint32_t i = bs + lane;
    return i < np ? poff[np - 1 - i] : kNone;
  };
  struct Head {
    uint32_t col, cnt, off;
    uint64_t rhs;
    uint32_t ent[kPre];  // entries k < cnt are the record's
  };
  auto load_head = [&](uint32_t off) {
    Head hd;
    hd.off = off;
    hd.col = kNone;
    hd.cnt = 0;
    hd.rhs = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPre; k++) hd.ent[k] = kNone;
    if (off != kNone) {
      const uint32_t *const rec = plog + off;
      hd.col = rec[0];
      hd.cnt = rec[1];
      hd.rhs = (uint64_t)rec[2] | ((uint64_t)rec[3] << 32);
      // independent of cnt, so that all of them load at once
#pragma unroll
      for (uint32_t k = 0; k < kPre; k++) hd.ent[k] = rec[4 + k];
    }
    return hd;
  };
  // one step over a record longer than kPre: lanes lm of such records still
  // to gather (the lowest, L, in this step), L's offset and count, the
  // step's first entry e and this lane's entry v (kNone: none)
  struct Step {
    uint64_t lm;
    uint32_t L, off, cnt, e, v;
  };
  auto first_step = [&](const Head &h) {
    Step st;
    st.lm = __ballot(h.cnt > kPre);
    st.L = 64;
    st.off = st.cnt = 0;
    st.e = kPre;
    st.v = kNone;
    if (st.lm) {
      st.L = (uint32_t)__ffsll((long long)st.lm) - 1;
      st.off = readlane(h.off, (int)st.L);
      st.cnt = readlane(h.cnt, (int)st.L);
      if (kPre + lane < st.cnt) st.v = plog[st.off + 4 + kPre + lane];
    }
    return st;
  };
  Head cur = load_head(load_off(0));
  uint32_t off_next = load_off(64);
  if (ring) {
    for (uint32_t i = lane; i < rl; i += 64) ring[i] = (T)0;
    wave_sync();
  }
  Step st = first_step(cur);
  uint32_t prev_last = kNone;  // the previous batch's highest pivot column
  for (uint32_t bs = 0; bs < np; bs += 64) {
    const bool valid = bs + lane < np;
    const uint32_t bmin = readlane(cur.col, 0);
    const uint32_t last = readlane(cur.col, (int)min(63u, np - 1 - bs));
    bcol[lane] = cur.col;
    const bool tags = ring && last - bmin < rl / 2;
    if (ring) {
      // the columns between the previous batch and this one, which this
      // batch's records may reference, are cleared before they are read
      if (bs) {
        const uint32_t gap = min(bmin - prev_last - 1u, rl);
        for (uint32_t g = lane; g < gap; g += 64) ring[(bmin - 1u - g) & (rl - 1)] = (T)0;
      }
      wave_sync();
      if (tags && valid) ring[cur.col & (rl - 1)] = (T)lane;
    }
    wave_sync();
    // the ring holds the values of columns [rtop - rl, bmin)
    const uint32_t rtop = tags ? last + 1u : bmin;
    auto in_ring = [&](uint32_t v) { return ring && rtop - v <= rl; };
    auto cell = [&](uint32_t v) -> uint64_t {
      return in_ring(v) ? (uint64_t)ring[v & (rl - 1)] : (uint64_t)wl[v];
    };
    // dependency bit of vertex v of this batch's range (bcol increases
    // with the lane; a pivot only depends on lower lanes)
    auto depbit = [&](uint32_t v, uint32_t below) -> uint64_t {
      uint32_t i;
      if (tags) {
        i = (uint32_t)ring[v & (rl - 1)] & 63u;
      } else {
        uint32_t lo = 0, hi = below;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (bcol[mid] < v) lo = mid + 1;
          else hi = mid;
        }
        i = lo;
      }
      return i < below && bcol[i] == v ? 1ull << i : 0ull;
    };
    // the next batch's headers and the offsets of the one after it
    const Head nxt = load_head(off_next);
    const uint32_t off_after = load_off(bs + 128);
    uint64_t acc = cur.rhs, dep = 0;
    {
      if (ring) {
        bool far = false;
#pragma unroll
        for (uint32_t k = 0; k < kPre; k++)
          far |= k < cur.cnt && cur.ent[k] < bmin && !in_ring(cur.ent[k]);
        if (__ballot(far)) wave_sync_global();
      }
      uint64_t w[kPre];
#pragma unroll
      for (uint32_t k = 0; k < kPre; k++)
        w[k] = k < cur.cnt && cur.ent[k] < bmin ? cell(cur.ent[k]) : 0ull;
#pragma unroll
      for (uint32_t k = 0; k < kPre; k++) {
        if (k < cur.cnt) {
          if (cur.ent[k] < bmin) acc ^= w[k];
          else dep |= depbit(cur.ent[k], lane);
        }
      }
    }
    // records longer than kPre, one step of 64 entries at a time
    if (st.lm) {
      uint64_t pacc = 0, pdep = 0;
      for (;;) {
        // the step after this one: record L's next entries, or the next
        // long record's first
        Step nx = st;
        nx.e = st.e + 64;
        const bool rec_done = nx.e >= st.cnt;
        if (rec_done) {
          nx.lm &= nx.lm - 1;
          nx.e = kPre;
          if (nx.lm) {
            nx.L = (uint32_t)__ffsll((long long)nx.lm) - 1;
            nx.off = readlane(cur.off, (int)nx.L);
            nx.cnt = readlane(cur.cnt, (int)nx.L);
          }
        }
        nx.v = kNone;
        if (nx.lm && nx.e + lane < nx.cnt) nx.v = plog[nx.off + 4 + nx.e + lane];
        const uint32_t v = st.v;
        if (ring && __ballot(v < bmin && !in_ring(v))) wave_sync_global();
        if (v < bmin) pacc ^= cell(v);
        else if (v != kNone) pdep |= depbit(v, st.L);
        if (rec_done) {
          const uint64_t ta = wave_xor64_total(pacc), td = wave_or64_total(pdep);
          if (lane == st.L) {
            acc ^= ta;
            dep |= td;
          }
          pacc = pdep = 0;
        }
        st = nx;
        if (!st.lm) break;
      }
    }
    // the next batch's first long step loads while this one finishes
    st = first_step(nxt);
    // dependencies in lane order (only lanes some pivot depends on)
    uint64_t x = acc;
    for (uint64_t dm = wave_or64_total(dep); dm; dm &= dm - 1) {
      const uint32_t k = (uint32_t)__ffsll((long long)dm) - 1;
      const uint64_t xk = readlane64(x, (int)k);
      if ((dep >> k) & 1ull) x ^= xk;
    }
    if (valid) wl[cur.col] = (T)x;
    if (ring) {
      // this batch's pivots into the ring, the columns between them
      // cleared (below the first, at the start of the next batch).  Only
      // the ring's rl columns up to the batch's highest pivot are written, so
      // no two lanes write one slot (the batch may span more columns).
      const uint32_t below = __shfl_up(cur.col, 1);
      const uint32_t pc = lane == 0 ? cur.col - 1u : below;
      if (valid && last - cur.col < rl) {
        const uint32_t gap = min(cur.col - pc - 1u, rl - 1u - (last - cur.col));
        for (uint32_t g = 0; g < gap; g++) ring[(cur.col - 1u - g) & (rl - 1)] = (T)0;
        ring[cur.col & (rl - 1)] = (T)x;
      }
      prev_last = last;
      wave_sync();
    } else {
      wave_sync_global();
    }
    cur = nxt;
    off_next = off_after;
  }
  if (ring) wave_sync_global();
}

// Exclusive prefix sum of a[0..n) in place (one wavefront), returns the total.
__device__ __forceinline__ uint32_t wave_scan_array(uint32_t *a, uint32_t *b, uint32_t n) {
  const uint32_t lane = lane_id();
  const uint32_t per = (n + 63) / 64, lo = lane * per, hi = min(n, lo + per);
  uint32_t sum = 0;
  for (uint32_t i = lo; i < hi; i++) sum += a[i];
  uint32_t inc = sum;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d);
    if (lane >= (uint32_t)d) inc += y;
  }
  const uint32_t total = readlane(inc, 63);
  uint32_t run = inc - sum;
  for (uint32_t i = lo; i < hi; i++) {
    const uint32_t c = a[i];
    a[i] = run;
    b[i] = run;
    run += c;
  }
  return total;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  return (uint64_t)uniform((uint32_t)x) | ((uint64_t)uniform((uint32_t)(x >> 32)) << 32);
}

// A grid of workgroups of five wavefronts takes work items (shards, or
// instances of a batch) from a shared counter until none is left.  Within a
// workgroup the items flow through three stages, each on its own records:
//  - wavefront 3 takes an item, computes its right sides, then per attempt
//    its edges, peeling order and 2-core; it retries failed attempts with
//    the next local seed and clears the cells of items that fail them all;
//  - wavefronts 0, 1 and 2 eliminate the 2-core of the oldest ready record
//    (0 searches the pivots, 1 and 2 emit the pivot rows);
//  - wavefront 4 assigns the cells of solved records.
// Peeling, elimination and assignment of consecutive items thus overlap.
// The roles follow where the wavefronts run: a CU deals the wavefronts of
// its two workgroups to its four SIMDs in turn, one workgroup after the
// other, so a workgroup's wavefronts 0 and 4 share a SIMD with the other
// workgroup's wavefront 3, and its wavefront 1 with the other's 0 and 4.
// With these roles the searching wavefront (a chain of dependent vector
// instructions) shares its SIMD with the two that mostly wait on memory,
// or with one emitter and one of those (a build 2.5% faster than with the
// assignment on wavefront 3).
// TR: a test build whose back-substitution ring holds A.ring_cols columns
// (launched only when that option is set, so that the kernel of every
// other build keeps a ring length known at compile time).
template <typename T, int QM, bool TR>
__global__ void __launch_bounds__(kBuildThreads) k_build(BuildArgs A) {
  extern __shared__ __align__(16) uint8_t lds[];
  if (A.abort && *A.abort) return;  // same value for every thread
  const uint32_t lane = lane_id();
  const uint32_t wid = uniform(threadIdx.x >> 6);  // one value per wavefront
  uint8_t *const wbase = A.scratch + (uint64_t)blockIdx.x * A.scratch_stride;
  const uint64_t slot_bytes = slot_layout(nullptr, A.M, A.scr_V, A.scr_l, A.logcap, nullptr);
  auto bufs = [&](uint32_t s) {
    ShardBufs sb;
    slot_layout(wbase + (uint64_t)s * slot_bytes, A.M, A.scr_V, A.scr_l, A.logcap, &sb);
    return sb;
  };
  BandCtl *const ctl = band_ctl(lds, A.lds_bytes);
  PipeCtl *const pc = pipe_ctl(lds, A.lds_bytes);
  ShardRec *const rec = pc->rec;

  if (threadIdx.x < kSlots) rec[threadIdx.x].state = kRecFree;
  if (threadIdx.x == 0) {
    pc->quit = 0;
    pc->abort = 0;
    pc->bar[0] = pc->bar[1] = pc->bar[2] = 0;
    pc->pick = kSlots;
  }
  // the only workgroup barrier: from here on the stages meet through records
  __syncthreads();

  auto state = [&](uint32_t s) { return lds_load(&rec[s].state); };
  auto geo = [&](uint32_t s) {
    Geo G = A.G;
    G.V = uniform64(rec[s].V);
    G.vmask = uniform64(rec[s].vmask);
    G.l = uniform(rec[s].l);
    G.sigma = uniform(rec[s].sigma);
    G.b = uniform(rec[s].b);
    return G;
  };

  // ------------------------------------------------------------ peeling
  // Peeling of an item is done by wavefront 3, except for the workgroup's
  // first item, which all five wavefronts peel together (nothing else can
  // run before it).  The helpers below take the calling threads' index tid
  // in [0, nthr) and sync(), which orders their memory operations (the
  // workgroup barrier, or a wavefront fence when one wavefront calls).
  uint64_t *f_st;
  uint32_t *f_F0, *f_F1, *f_cc;
  uint8_t *f_pe;
  {
    FrontBufs fb;
    front_layout(wbase + (uint64_t)kSlots * slot_bytes, A.M, A.scr_V, A.scr_l, &fb);
    f_st = fb.st;
    f_F0 = fb.F0;
    f_F1 = fb.F1;
    f_cc = fb.cc;
    f_pe = fb.pe;
  }
  uint32_t *const fcnt = pc->fcnt;

  // edges, peeling order and grouped 2-core of attempt t; early = 1: two
  // 2-core rows contradict each other, 2: an MWHC hypergraph did not peel.
  // List appends count in LDS: fcnt[0] the degree-one vertices, fcnt[1]
  // the peeled edges, fcnt[2 + r mod 3] the vertices freed by round r (a
  // count is reset a round before its use, after everyone has read its
  // previous value), fcnt[5] the 2-core size, fcnt[6] a contradiction.
  auto front = [&](const Geo &G, const ShardBufs &sb, uint32_t m, uint64_t base, uint32_t t,
                   uint32_t tid, uint32_t nthr, auto &&sync, uint32_t &k_out,
                   uint32_t &rounds_out, uint32_t &early_out) {
    const uint64_t V = G.V;
    uint64_t *const E = sb.E;
    const uint64_t *const R = sb.R;
    uint32_t *const stk = sb.stack, *const rst = sb.rst;
    const uint32_t w0t = tid - lane;  // this wavefront's first thread
    const FrontBufs fb{f_st, f_pe, f_F0, f_F1, f_cc};
    uint32_t nrounds = 0;
    // The workgroup's first item (all wavefronts, nothing in the window's
    // LDS yet) counts the vertex state in LDS, kLdsChunk vertices per pass
    // over the edges, and stores it whole: every workgroup peels its first
    // item at the same time, when global atomics are the scarce resource.
    const uint32_t kLdsChunk = (A.lds_bytes - kLdsTail - ring_bytes<T>()) / 8u;
    const bool lds_inc = nthr == kBuildThreads && V <= 8ull * kLdsChunk;
    VF_CLK(pf0);
    if (tid == 0)
      for (int i = 0; i < 7; i++) fcnt[i] = 0;
    // edges of this attempt, cleared vertex state.  The passes over edges
    // and vertices keep kPU loads per lane in flight: a wavefront alone
    // would otherwise wait a memory round trip per 64 elements.
    for (uint32_t i0 = tid; i0 < m; i0 += nthr * kPU) {
      uint64_t key[kPU];
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++) {
        const uint32_t i = i0 + u * nthr;
        key[u] = i < m ? A.bkeys[base + i] : 0ull;
      }
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++) {
        const uint32_t i = i0 + u * nthr;
        if (i < m) {
          uint32_t v0, v1, v2;
          edge3(G, fin64(key[u] ^ G.khi), fin64(key[u] ^ G.klo), t, v0, v1, v2);
          E[i] = pack3(v0, v1, v2);
          fb.pe[i] = 0;
        }
      }
    }
    if (!lds_inc)
      for (uint64_t v = tid; v < V; v += nthr) fb.st[v] = 0;
    sync();
    VF_CLK(pf1);
    // incidence: degree and xor of incident edges
    for (uint64_t c0 = 0; lds_inc && c0 < V; c0 += kLdsChunk) {
      uint64_t *const lst = (uint64_t *)lds;
      const uint32_t cn = (uint32_t)min((uint64_t)kLdsChunk, V - c0);
      for (uint32_t j = tid; j < cn; j += nthr) lst[j] = 0;
      sync();
      for (uint32_t i0 = tid; i0 < m; i0 += nthr * kPU) {
        uint64_t e[kPU];
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          const uint32_t i = i0 + u * nthr;
          e[u] = i < m ? E[i] : 0ull;
        }
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          const uint32_t i = i0 + u * nthr;
          if (i < m) {
            uint32_t v[3];
            unpack3(e[u], v);
            for (int k = 0; k < 3; k++) {
              const uint64_t d = (uint64_t)v[k] - c0;
              if (d < cn) atomicAdd((unsigned long long *)&lst[d], kDegOne + i);
            }
          }
        }
      }
      sync();
      // stored whole, with the first frontier (the vertices of degree one)
      for (uint32_t j0 = w0t; j0 < cn; j0 += nthr) {
        const uint32_t j = j0 + lane;
        const uint64_t sv = j < cn ? lst[j] : 0ull;
        if (j < cn) fb.st[c0 + j] = sv;
        const bool one = j < cn && (sv >> 32) == 1;
        const uint32_t at = wave_append(one, &fcnt[0]);
        if (one) fb.F0[at] = (uint32_t)(c0 + j);
      }
      sync();
    }
    for (uint32_t i0 = tid; !lds_inc && i0 < m; i0 += nthr * kPU) {
      uint64_t e[kPU];
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++) {
        const uint32_t i = i0 + u * nthr;
        e[u] = i < m ? E[i] : 0ull;
      }
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++) {
        const uint32_t i = i0 + u * nthr;
        if (i < m) {
          uint32_t v[3];
          unpack3(e[u], v);
          for (int k = 0; k < 3; k++)
            atomicAdd((unsigned long long *)&fb.st[v[k]], kDegOne + i);
        }
      }
    }
    sync();
    VF_CLK(pf2);
    // round-synchronous peeling (the first frontier, unless found above)
    for (uint64_t v0 = w0t; !lds_inc && v0 < V; v0 += (uint64_t)nthr * kPU) {
      uint64_t sv[kPU];
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++) {
        const uint64_t v = v0 + (uint64_t)u * nthr + lane;
        sv[u] = v < V ? fb.st[v] : 0ull;
      }
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++) {
        const uint64_t v = v0 + (uint64_t)u * nthr + lane;
        const bool one = v < V && (sv[u] >> 32) == 1;
        const uint32_t at = wave_append(one, &fcnt[0]);
        if (one) fb.F0[at] = (uint32_t)v;
      }
    }
    sync();
    uint32_t nf = lds_load(&fcnt[0]), nst = 0;
    VF_CLK(pf3);
    uint32_t *cur = fb.F0, *nxt = fb.F1;
    if (tid == 0) rst[0] = 0;
    while (nf) {
      const uint32_t r0 = nst;
      uint32_t *const ncnt = &fcnt[2 + nrounds % 3];
      if (tid == 0) fcnt[2 + (nrounds + 1) % 3] = 0;
      // select with the degrees of the start of the round (kPU frontier
      // vertices per lane at a time, each step's loads in flight together)
      for (uint32_t i0 = w0t; i0 < nf; i0 += nthr * kPU) {
        uint32_t v[kPU], e[kPU], side[kPU];
        uint64_t sv[kPU], ev[kPU];
        bool take[kPU];
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          const uint32_t i = i0 + u * nthr + lane;
          v[u] = i < nf ? cur[i] : 0xFFFFFFFFu;
        }
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) sv[u] = v[u] != 0xFFFFFFFFu ? fb.st[v[u]] : 0ull;
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          take[u] = (sv[u] >> 32) == 1;
          e[u] = (uint32_t)sv[u];
          ev[u] = take[u] ? E[e[u]] : 0ull;
        }
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          side[u] = 0;
          if (take[u]) {
            uint32_t a[3];
            unpack3(ev[u], a);
            side[u] = a[0] == v[u] ? 0u : (a[1] == v[u] ? 1u : 2u);
            for (uint32_t k = 0; k < side[u]; k++)
              if ((fb.st[a[k]] >> 32) == 1) take[u] = false;
          }
        }
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          const uint32_t at = wave_append(take[u], &fcnt[1]);
          if (take[u]) {
            stk[at] = e[u] | (side[u] << 30);
            fb.pe[e[u]] = 1;
          }
        }
      }
      sync();
      nst = lds_load(&fcnt[1]);
      // remove the selected edges
      for (uint32_t i0 = r0 + w0t; i0 < nst; i0 += nthr * kPU) {
        uint32_t e[kPU];
        uint64_t ev[kPU];
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          const uint32_t i = i0 + u * nthr + lane;
          e[u] = i < nst ? stk[i] & 0x3FFFFFFFu : 0xFFFFFFFFu;
        }
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) ev[u] = e[u] != 0xFFFFFFFFu ? E[e[u]] : 0ull;
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          bool push[3] = {false, false, false};
          uint32_t a[3] = {0, 0, 0};
          if (e[u] != 0xFFFFFFFFu) {
            unpack3(ev[u], a);
            for (int k = 0; k < 3; k++) {
              const uint64_t old = atomicAdd((unsigned long long *)&fb.st[a[k]],
                                             (unsigned long long)(-(kDegOne + e[u])));
              push[k] = (old >> 32) == 2;
            }
          }
          for (int k = 0; k < 3; k++) {
            const uint32_t at = wave_append(push[k], ncnt);
            if (push[k]) nxt[at] = a[k];
          }
        }
      }
      nrounds++;
      if (tid == 0) rst[nrounds] = nst;
      sync();
      nf = lds_load(ncnt);
      uint32_t *tmp = cur;
      cur = nxt;
      nxt = tmp;
    }

    VF_CLK(pf4);
    // 2-core edges, grouped by the entry group of their top vertex (an
    // MWHC hypergraph is peel-only: only its unpeeled edges are counted)
    uint32_t k;
    if (G.mwhc) {
      uint32_t left = 0;
      for (uint32_t i = tid; i < m; i += nthr) left += fb.pe[i] ? 0u : 1u;
      left = wave_sum(left);
      if (lane == 0 && left) atomicAdd(&fcnt[5], left);
      sync();
      k = lds_load(&fcnt[5]);
    } else {
      const uint32_t gsh = entry_shift(G.sigma);
      const uint32_t ngroups = (uint32_t)((V - 1) >> gsh) + 2;
      for (uint32_t g = tid; g < ngroups; g += nthr) fb.cc[g] = 0;
      sync();
      for (uint32_t i0 = tid; i0 < m; i0 += nthr * kPU) {
        uint64_t e[kPU];
        uint8_t pe[kPU];
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          const uint32_t i = i0 + u * nthr;
          pe[u] = i < m ? fb.pe[i] : (uint8_t)1;
          e[u] = i < m ? E[i] : 0ull;
        }
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++)
          if (!pe[u]) atomicAdd(&fb.cc[(uint32_t)(e[u] >> 42) >> gsh], 1u);
      }
      sync();
      if (tid < 64) {  // one wavefront scans the group counts
        const uint32_t kk = wave_scan_array(fb.cc, sb.cb, ngroups);
        if (tid == 0) fcnt[5] = kk;
      }
      sync();
      k = lds_load(&fcnt[5]);
      for (uint32_t i0 = tid; i0 < m; i0 += nthr * kPU) {
        uint64_t e[kPU], r[kPU];
        uint8_t pe[kPU];
        uint32_t pos[kPU];
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++) {
          const uint32_t i = i0 + u * nthr;
          pe[u] = i < m ? fb.pe[i] : (uint8_t)1;
          e[u] = i < m ? E[i] : 0ull;
          r[u] = i < m ? R[i] : 0ull;
        }
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++)
          pos[u] = pe[u] ? 0u : atomicAdd(&fb.cc[(uint32_t)(e[u] >> 42) >> gsh], 1u);
#pragma unroll
        for (uint32_t u = 0; u < kPU; u++)
          if (!pe[u]) {
            sb.cE[pos[u]] = e[u];
            sb.cR[pos[u]] = r[u];
          }
      }
      sync();
    }
    // MWHC is peel-only: any unpeeled edge ends the attempt (kind 2).
    // Otherwise two 2-core rows with the same vertices and different right
    // sides (the usual reason for an inconsistent system) end the attempt
    // before the elimination: rows are listed by top vertex in the degree
    // array, which peeling no longer needs
    VF_CLK(pf5);
    const uint32_t kl = G.mwhc ? 0u : k;
    uint32_t *const head = (uint32_t *)fb.st, *const next = fb.F0;
    if (kl)
      for (uint64_t v = tid; v < V; v += nthr) head[v] = 0xFFFFFFFFu;
    sync();
    for (uint32_t i0 = tid; i0 < kl; i0 += nthr * kPU) {
      uint64_t e[kPU];
      uint32_t nx[kPU];
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++) {
        const uint32_t i = i0 + u * nthr;
        e[u] = i < kl ? sb.cE[i] : 0ull;
      }
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++) {
        const uint32_t i = i0 + u * nthr;
        nx[u] = i < kl ? atomicExch(&head[(uint32_t)(e[u] >> 42)], i) : 0u;
      }
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++)
        if (i0 + u * nthr < kl) next[i0 + u * nthr] = nx[u];
    }
    sync();
    bool clash = false;
    for (uint32_t i0 = tid; i0 < kl; i0 += nthr * kPU) {
      uint64_t e[kPU], r[kPU];
      uint32_t x[kPU];
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++) {
        const uint32_t i = i0 + u * nthr;
        e[u] = i < kl ? sb.cE[i] : 0ull;
        r[u] = i < kl ? sb.cR[i] : 0ull;
        x[u] = i < kl ? next[i] : 0xFFFFFFFFu;
      }
#pragma unroll
      for (uint32_t u = 0; u < kPU; u++)
        for (; x[u] != 0xFFFFFFFFu; x[u] = next[x[u]])
          clash |= sb.cE[x[u]] == e[u] && sb.cR[x[u]] != r[u];
    }
    if (__ballot(clash) != 0 && lane == 0) atomicOr(&fcnt[6], 1u);
    sync();
    const bool dup = lds_load(&fcnt[6]) != 0;
#ifdef VF_STAGE_CLOCKS
    if (tid == w0t && w0t == 0) {
      VF_CLK_ADD(kClkPeelPhases + 0, pf1 - pf0);
      VF_CLK_ADD(kClkPeelPhases + 1, pf2 - pf1);
      VF_CLK_ADD(kClkPeelPhases + 2, pf3 - pf2);
      VF_CLK_ADD(kClkPeelPhases + 3, pf4 - pf3);
      VF_CLK_ADD(kClkPeelPhases + 4, pf5 - pf4);
      VF_CLK_ADD(kClkPeelPhases + 5, wall_clock64() - pf5);
      VF_CLK_ADD(kClkPeelPhases + 6, 1);
      VF_CLK_ADD(kClkPeelPhases + 7, nrounds);
    }
#endif
    k_out = k;
    rounds_out = nrounds;
    early_out = G.mwhc && k ? 2u : (dup ? 1u : 0u);
  };

  // cells of a failed item are zero, its local seed 255
  auto clear = [&](uint32_t s, uint32_t tid, uint32_t nthr) {
    const uint64_t V = uniform64(rec[s].V);
    T *const wg = (T *)uniform64(rec[s].cells);
    for (uint64_t v = tid; v < V; v += nthr) wg[v] = (T)0;
    if (tid == 0) A.tseed[uniform(rec[s].shard)] = 255;
  };

  uint32_t order = 0;  // peeling wavefront: records made ready so far
  // attempts t, t + 1, ... of record s until one leaves a 2-core for the
  // elimination (ready) or none (solved); every attempt failing clears the
  // cells (free)
  auto attempts = [&](uint32_t s, uint32_t t, uint32_t tid, uint32_t nthr, auto &&sync) {
    const uint32_t j = uniform(rec[s].shard), m = uniform(rec[s].m);
    const uint64_t base = uniform64(rec[s].base);
    const ShardBufs sb = bufs(s);
    const Geo G = geo(s);
    for (; t < A.tmax; t++) {
      uint32_t k, nrounds, early;
      front(G, sb, m, base, t, tid, nthr, sync, k, nrounds, early);
      if (early) {
        if (tid == 0) {
          const uint32_t idx = atomicAdd(&A.work[kWorkFails], 1u);
          if (idx < A.fail_cap) A.fails[idx] = FailRec{j, t, early, k};
        }
        continue;
      }
      if (tid == 0) {
        rec[s].t = t;
        rec[s].core = k;
        rec[s].rounds = nrounds;
        rec[s].np = 0;
        rec[s].order = order;
      }
      order += k ? 1u : 0u;
      sync();
      if (tid < 64) lds_publish(&rec[s].state, k ? kRecReady : kRecSolved);
      return;
    }
    clear(s, tid, nthr);
    sync();
    if (tid < 64) lds_publish(&rec[s].state, kRecFree);
  };

  // the next work item and its first local seed (one lane); j = ~0: none
  auto next_item = [&](uint32_t &j, uint32_t &t0) {
    j = atomicAdd(&A.work[kWorkNext], 1u);
    t0 = 0;
    if (A.list) {
      if (j < (A.nlist_dev ? *A.nlist_dev : A.nlist)) {
        t0 = A.list[2 * j + 1];
        j = A.list[2 * j];
      } else {
        j = 0xFFFFFFFFu;
      }
    } else if (j >= A.G.S) {
      j = 0xFFFFFFFFu;
    }
  };
  // record s takes item j (one lane)
  auto fill = [&](uint32_t s, uint32_t j, uint32_t t0) {
    ShardRec &r = rec[s];
    r.state = kRecFront;
    r.shard = j;
    r.t = t0;
    if (A.items) {
      const BatchItem it = A.items[j];
      r.V = it.V;
      r.vmask = it.vmask;
      r.l = it.l;
      r.sigma = it.sigma;
      r.b = it.b;
      r.base = it.key_off;
      r.m = it.n;
      r.cells = (uint64_t)((uint8_t *)A.cells + it.cell_off);
    } else {
      r.V = A.G.V;
      r.vmask = A.G.vmask;
      r.l = A.G.l;
      r.sigma = A.G.sigma;
      r.b = A.G.b;
      r.base = A.offsets[j];
      r.m = (uint32_t)(A.offsets[j + 1] - A.offsets[j]);
      r.cells = (uint64_t)((T *)A.cells + (uint64_t)j * A.G.V);
    }
  };
  // right sides of record s: values (Problem 1) or fingerprints (Problem 2)
  auto rights = [&](uint32_t s, uint32_t tid, uint32_t nthr) {
    const Geo G = geo(s);
    const ShardBufs sb = bufs(s);
    const uint32_t m = uniform(rec[s].m);
    const uint64_t base = uniform64(rec[s].base);
    for (uint32_t i = tid; i < m; i += nthr) {
      const uint64_t key = A.bkeys[base + i];
      if (G.is_filter) {
        sb.R[i] = fingerprint(G, fin64(key ^ G.khi), fin64(key ^ G.klo));
      } else {
        sb.R[i] = A.bvals[base + i] & G.vmask;
      }
    }
  };

  // the workgroup's first item, peeled by all five wavefronts into record 0
  bool exhausted;
  VF_CLK(ck0);
  {
    auto bar = [] { __syncthreads(); };
    if (threadIdx.x == 0) {
      uint32_t j, t0;
      next_item(j, t0);
      pc->first[0] = j;
      pc->first[1] = t0;
      if (j != 0xFFFFFFFFu) fill(0, j, t0);
    }
    __syncthreads();
    const uint32_t j = lds_load(&pc->first[0]), t0 = lds_load(&pc->first[1]);
    exhausted = j == 0xFFFFFFFFu;
    if (!exhausted) {
      rights(0, threadIdx.x, kBuildThreads);
      __syncthreads();
      attempts(0, t0, threadIdx.x, kBuildThreads, bar);
    }
    __syncthreads();
    if (threadIdx.x == 0) VF_CLK_ADD(kClkFirst, wall_clock64() - ck0);
  }

  if (wid == 3) {
    // ------------------------------------------------ peeling (wavefront 3)
    auto wsync = [] { wave_sync_global(); };
    for (;;) {
      // failed eliminations first, then a new item into a free record once
      // no record waits for the elimination (taking items further ahead
      // would only leave other workgroups idle at the end)
      uint32_t s = kSlots, what = kRecFree;
      bool done = false;
      wait_for(pc, A.work, [&] {
        uint32_t fr = kSlots, nfree = 0, nready = 0;
        for (uint32_t i = 0; i < kSlots; i++) {
          const uint32_t st = state(i);
          if (st == kRecRetry || st == kRecGiveUp) {
            s = i;
            what = st;
            return true;
          }
          if (st == kRecFree) {
            nfree++;
            if (fr == kSlots) fr = i;
          }
          nready += st == kRecReady ? 1u : 0u;
        }
        if (!exhausted && fr < kSlots && nready == 0) {
          s = fr;
          what = kRecFree;
          return true;
        }
        done = exhausted && nfree == kSlots;
        return done;
      });
      acquire_wg();
      if (done) {
        lds_publish(&pc->quit, 1u);
        break;
      }
      if (what == kRecGiveUp) {
        clear(s, lane, 64);
        wave_sync_global();
        lds_publish(&rec[s].state, kRecFree);
        continue;
      }
      if (what == kRecRetry) {
        if (lane == 0) rec[s].state = kRecFront;
        VF_CLK(c0);
        attempts(s, uniform(rec[s].t) + 1u, lane, 64, wsync);
        VF_CLK_ADD(kClkPeel, wall_clock64() - c0);
        VF_CLK_ADD(kClkPeel + 1, 1);
        continue;
      }
      // the next work item
      uint32_t j = 0xFFFFFFFFu, t0 = 0;
      if (lane == 0) next_item(j, t0);
      j = uniform(j);
      t0 = uniform(t0);
      if (j == 0xFFFFFFFFu) {
        exhausted = true;
        continue;
      }
      if (lane == 0) fill(s, j, t0);
      wave_sync();
      rights(s, lane, 64);
      VF_CLK(c0);
      attempts(s, t0, lane, 64, wsync);
      VF_CLK_ADD(kClkPeel, wall_clock64() - c0);
      VF_CLK_ADD(kClkPeel + 1, 1);
    }
  } else if (wid != 4) {
    // -------------------------------------- elimination (wavefronts 0, 1, 2)
    const uint32_t bw = wid;  // 0: search, 1 and 2: emit
    // the SIMDs issue the elimination's instructions ahead of the peeling
    // and assigning wavefronts', the search's ahead of all
    if (bw == 0) __builtin_amdgcn_s_setprio(3);
    else __builtin_amdgcn_s_setprio(2);
    uint32_t gen = 0;
    for (;;) {
      if (bw == 0) {
        uint32_t s = kSlots;
        wait_for(pc, A.work, [&] {
          uint32_t best = 0xFFFFFFFFu;
          s = kSlots;
          for (uint32_t i = 0; i < kSlots; i++)
            if (state(i) == kRecReady) {
              const uint32_t o = lds_load(&rec[i].order);
              if (o < best) {
                best = o;
                s = i;
              }
            }
          return s < kSlots || lds_load(&pc->quit) != 0;
        });
        acquire_wg();
        if (lane == 0) {
          if (s < kSlots) rec[s].state = kRecBand;
          pc->pick = s;
        }
      }
      band_sync(pc, A.work, bw, gen);
      const uint32_t s = lds_load(&pc->pick);
      if (s >= kSlots) break;
      const ShardBufs sb = bufs(s);
      const Geo G = geo(s);
      const uint32_t W = min(A.wmax, window_slots_for(G.sigma, A.lds_bytes - ring_bytes<T>()));
      uint32_t np = 0;
      VF_CLK(c0b);
      const int st = band_solve<QM>(A, G, W, sb, lds, ctl, bw, &np, pc, gen);
      if (bw == 0) {
        VF_CLK_ADD(kClkBand, wall_clock64() - c0b);
        VF_CLK_ADD(kClkBand + 1, 1);
        VF_CLK_MAX(kClkElimEnd, wall_clock64() - ck0);
      }
      if (bw == 0) {
        const uint32_t j = uniform(rec[s].shard), t = uniform(rec[s].t);
        uint32_t next = kRecSolved;
        if (st == kSolveCapacity) {
          if (lane == 0) {
            if (A.overflow) {
              const uint32_t idx = atomicAdd(&A.work[kWorkCap], 1u);
              atomicAdd(&A.work[kWorkRelaunch], 1u);
              A.overflow[2 * idx] = j;
              A.overflow[2 * idx + 1] = t;
            } else {
              atomicOr(&A.work[kWorkStatus], kStatusCapacity);
            }
          }
          next = kRecGiveUp;
        } else if (st == kSolveInconsistent) {
          if (lane == 0) {
            const uint32_t idx = atomicAdd(&A.work[kWorkFails], 1u);
            if (idx < A.fail_cap) A.fails[idx] = FailRec{j, t, 1u, uniform(rec[s].core)};
          }
          next = kRecRetry;
        } else if (lane == 0) {
          rec[s].np = np;
        }
        lds_publish(&rec[s].state, next);
      }
    }
  } else {
    // ----------------------------------------------- assignment (wavefront 4)
    uint32_t *const bcol = (uint32_t *)(lds + A.lds_bytes - kBcolBytes);
    // the ring of the back-substitution sits between the window and the
    // control blocks at the end of the LDS
    T *const ring = ring_bytes<T>() ? (T *)(lds + A.lds_bytes - kLdsTail - ring_bytes<T>())
                                    : nullptr;
    for (;;) {
      uint32_t s = kSlots;
      wait_for(pc, A.work, [&] {
        s = kSlots;
        for (uint32_t i = 0; i < kSlots; i++)
          if (s == kSlots && state(i) == kRecSolved) s = i;
        return s < kSlots || lds_load(&pc->quit) != 0;
      });
      acquire_wg();
      if (s >= kSlots) break;
      // cells: zero, core values by back-substitution, then the peeled
      // edges in reverse round order
      const ShardBufs sb = bufs(s);
      const uint64_t V = uniform64(rec[s].V);
      T *const wg = (T *)uniform64(rec[s].cells);
      const uint32_t np = uniform(rec[s].np), nrounds = uniform(rec[s].rounds);
      for (uint64_t v = lane; v < V; v += 64) wg[v] = (T)0;
      wave_sync_global();
      VF_CLK(c0a);
      // (a test build's ring, of ring_cols columns, for every segment size)
      const bool use_ring = ring && (TR || 3u * (1u << uniform(rec[s].sigma)) + 64u <= kRing);
      if (np) back_substitute<T, TR>(sb, np, wg, bcol, use_ring ? ring : nullptr, A.ring_cols);
      VF_CLK_ADD(kClkBackSub, wall_clock64() - c0a);
      for (int r = (int)nrounds - 1; r >= 0; r--) {
        const uint32_t e0 = sb.rst[r], e1 = sb.rst[r + 1];
        for (uint32_t i = e0 + lane; i < e1; i += 64) {
          const uint32_t ent = sb.stack[i];
          const uint32_t e = ent & 0x3FFFFFFFu, side = ent >> 30;
          uint32_t a[3];
          unpack3(sb.E[e], a);
          uint64_t val = sb.R[e];
          for (uint32_t q = 0; q < 3; q++)
            if (q != side) val ^= (uint64_t)wg[a[q]];
          wg[a[side]] = (T)val;
        }
        wave_sync_global();
      }
      if (lane == 0) A.tseed[uniform(rec[s].shard)] = (uint8_t)uniform(rec[s].t);
      VF_CLK_ADD(kClkAssign, wall_clock64() - c0a);
      VF_CLK_ADD(kClkAssign + 1, 1);
      lds_publish(&rec[s].state, kRecFree);
    }
  }
  if (wid == 4) VF_CLK_ADD(kClkTotal, wall_clock64() - ck0);
}

// ------------------------------------------------- small instances (batches)
//
// An instance of at most kSmallKeys keys and kSmallCells cells is built by
// one wavefront, everything on chip: its edges sit in registers (two keys
// per lane), peeling keeps each vertex's degree and edge-index sum in LDS,
// the 2-core is eliminated densely in registers (each row an 8-word mask
// over the cells, one row per lane and register set), swept from the top
// column down with the first candidate row as pivot (the same canonical
// solution as any other choice: pivots are the highest columns, free
// variables zero), then back-substituted and the peeled edges assigned in
// reverse round order in LDS.  Failed attempts retry with the next local
// seed, exactly as the large-instance kernel does.
constexpr uint32_t kSmallKeys = 128;
constexpr uint32_t kSmallCells = 256;
constexpr uint32_t kSmallWaves = kSmallWavesPerGroup;

bool small_instance(uint64_t n, uint64_t V) { return n <= kSmallKeys && V <= kSmallCells; }

template <typename T>
__device__ __forceinline__ void small_store(uint8_t *cells, const uint64_t *x, uint64_t V,
                                            uint64_t vmask, uint32_t lane) {
  T *const c = (T *)cells;
  for (uint32_t v = lane; v < V; v += 64) c[v] = (T)(x[v] & vmask);
}

__global__ void __launch_bounds__(64 * kSmallWaves) k_small(BuildArgs A) {
  __shared__ uint64_t xs_all[kSmallWaves][kSmallCells];        // vertex state, then values
  __shared__ uint32_t prow_all[kSmallWaves][kSmallKeys][8];    // pivot rows
  __shared__ uint64_t prhs_all[kSmallWaves][kSmallKeys];       // their right sides
  __shared__ uint16_t pcol_all[kSmallWaves][kSmallKeys];       // their columns
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  uint64_t *const xs = xs_all[wv];
  uint32_t (*const prow)[8] = prow_all[wv];
  uint64_t *const prhs = prhs_all[wv];
  uint16_t *const pcol = pcol_all[wv];
  if (A.abort && *A.abort) return;
  const uint32_t nlist = A.nlist_dev ? *A.nlist_dev : A.nlist;
  for (uint32_t w = blockIdx.x * kSmallWaves + wv; w < nlist; w += gridDim.x * kSmallWaves) {
    const uint32_t q = A.list[2 * w], t0 = A.list[2 * w + 1];
    const BatchItem I = A.items[q];
    Geo g = A.G;
    g.V = I.V;
    g.vmask = I.vmask;
    g.l = I.l;
    g.sigma = I.sigma;
    g.b = I.b;
    g.h = 0;
    const uint32_t m = I.n, V = (uint32_t)I.V;
    uint8_t *const cells = (uint8_t *)A.cells + I.cell_off;
    uint64_t hi[2], lo[2], rhs[2];
    bool valid[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
      const uint32_t i = lane + 64 * r;
      valid[r] = i < m;
      const uint64_t key = valid[r] ? A.bkeys[I.key_off + i] : 0ull;
      hi[r] = fin64(key ^ g.khi);
      lo[r] = fin64(key ^ g.klo);
      rhs[r] = !valid[r] ? 0ull
               : g.is_filter ? fingerprint(g, hi[r], lo[r])
                             : A.bvals[I.key_off + i] & g.vmask;
    }
    uint32_t t = t0;
    bool ok = false;
    for (; t < A.tmax && !ok; t++) {
      uint32_t ev[2][3];
#pragma unroll
      for (int r = 0; r < 2; r++) {
        ev[r][0] = ev[r][1] = ev[r][2] = 0;
        if (valid[r]) edge3(g, hi[r], lo[r], t, ev[r][0], ev[r][1], ev[r][2]);
      }
      for (uint32_t v = lane; v < V; v += 64) xs[v] = 0;
      wave_sync();
#pragma unroll
      for (int r = 0; r < 2; r++)
        if (valid[r])
#pragma unroll
          for (int k = 0; k < 3; k++)
            atomicAdd((unsigned long long *)&xs[ev[r][k]], kDegOne + lane + 64 * r);
      wave_sync();
      // round-synchronous peeling: degrees as they stand when the round
      // starts, hinge = the edge's first degree-one vertex
      int32_t rnd[2] = {-1, -1};
      uint32_t side[2] = {0, 0};
      int32_t nrounds = 0;
      for (;;) {
        bool take[2] = {false, false};
#pragma unroll
        for (int r = 0; r < 2; r++) {
          if (valid[r] && rnd[r] < 0) {
#pragma unroll
            for (int k = 2; k >= 0; k--)
              if ((xs[ev[r][k]] >> 32) == 1) {
                take[r] = true;
                side[r] = (uint32_t)k;
              }
          }
        }
        wave_sync();
        if (!(__ballot(take[0]) | __ballot(take[1]))) break;
#pragma unroll
        for (int r = 0; r < 2; r++)
          if (take[r]) {
            rnd[r] = nrounds;
#pragma unroll
            for (int k = 0; k < 3; k++)
              atomicAdd((unsigned long long *)&xs[ev[r][k]],
                        (unsigned long long)(-(kDegOne + lane + 64 * r)));
          }
        wave_sync();
        nrounds++;
      }
      // the 2-core as rows over the cells
      uint32_t row[2][8];
      uint64_t rr[2];
      bool live[2];
#pragma unroll
      for (int r = 0; r < 2; r++) {
        live[r] = valid[r] && rnd[r] < 0;
        rr[r] = live[r] ? rhs[r] : 0ull;
#pragma unroll
        for (int d = 0; d < 8; d++) {
          uint32_t x = 0;
          if (live[r])
#pragma unroll
            for (int k = 0; k < 3; k++)
              if ((ev[r][k] >> 5) == (uint32_t)d) x ^= 1u << (ev[r][k] & 31);
          row[r][d] = x;
        }
      }
      const uint32_t ncore = (uint32_t)(__popcll(__ballot(live[0])) + __popcll(__ballot(live[1])));
      uint32_t np = 0;
      const int nwords = (int)((V + 31) >> 5);
#pragma unroll
      for (int d = 7; d >= 0; d--) {
        if (d >= nwords) continue;
        uint32_t colmask = wave_or((live[0] ? row[0][d] : 0u) | (live[1] ? row[1][d] : 0u));
        while (colmask) {
          const uint32_t b = 31 - __clz(colmask), bit = 1u << b;
          const uint64_t m0 = __ballot(live[0] && (row[0][d] & bit));
          const uint64_t m1 = __ballot(live[1] && (row[1][d] & bit));
          if (!(m0 | m1)) {
            colmask &= bit - 1u;
            continue;
          }
          const int pr = m0 ? 0 : 1;
          const int pl = (int)__ffsll((long long)(m0 ? m0 : m1)) - 1;
          uint32_t pw[8];
#pragma unroll
          for (int dd = 0; dd < 8; dd++) pw[dd] = readlane(pr == 0 ? row[0][dd] : row[1][dd], pl);
          const uint64_t prh = readlane64(pr == 0 ? rr[0] : rr[1], pl);
          if (lane == 0) {
#pragma unroll
            for (int dd = 0; dd < 8; dd++) prow[np][dd] = pw[dd];
            prhs[np] = prh;
            pcol[np] = (uint16_t)(d * 32 + b);
          }
#pragma unroll
          for (int r = 0; r < 2; r++) {
            const bool cand = live[r] && (row[r][d] & bit);
            if (r == pr && (int)lane == pl) {
              live[r] = false;  // the pivot row leaves
            } else if (cand) {
#pragma unroll
              for (int dd = 0; dd < 8; dd++) row[r][dd] ^= pw[dd];
              rr[r] ^= prh;
            }
          }
          np++;
          colmask = (colmask | pw[d]) & (bit - 1u);
        }
      }
      // rows left over are zero: a right side that is not zero is a
      // contradiction
      if (__ballot((live[0] && rr[0] != 0) || (live[1] && rr[1] != 0))) {
        if (lane == 0) {
          const uint32_t idx = atomicAdd(&A.work[kWorkFails], 1u);
          if (idx < A.fail_cap) A.fails[idx] = FailRec{q, t, 1u, ncore};
        }
        continue;
      }
      // values: pivots by increasing column (the last found is the lowest)
      for (uint32_t v = lane; v < V; v += 64) xs[v] = 0;
      wave_sync();
      for (int i = (int)np - 1; i >= 0; i--) {
        const uint32_t c = pcol[i];
        const uint32_t word = prow[i][lane >> 3];
        const uint32_t nib = (word >> ((lane & 7u) * 4)) & 0xFu;
        uint64_t acc = 0;
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
          const uint32_t v = lane * 4 + j;
          if (((nib >> j) & 1u) && v != c) acc ^= xs[v];
        }
        acc = wave_xor64(acc);
        if (lane == 0) xs[c] = acc ^ prhs[i];
        wave_sync();
      }
      for (int rd = nrounds - 1; rd >= 0; rd--) {
#pragma unroll
        for (int r = 0; r < 2; r++)
          if (rnd[r] == rd) {
            uint64_t val = rhs[r];
#pragma unroll
            for (int k = 0; k < 3; k++)
              if ((uint32_t)k != side[r]) val ^= xs[ev[r][k]];
            xs[ev[r][side[r]]] = val;
          }
        wave_sync();
      }
      switch (I.cell_bytes) {
        case 1: small_store<uint8_t>(cells, xs, V, g.vmask, lane); break;
        case 2: small_store<uint16_t>(cells, xs, V, g.vmask, lane); break;
        case 4: small_store<uint32_t>(cells, xs, V, g.vmask, lane); break;
        default: small_store<uint64_t>(cells, xs, V, g.vmask, lane); break;
      }
      if (lane == 0) A.tseed[q] = (uint8_t)t;
      ok = true;
    }
    if (!ok) {
      for (uint32_t v = lane; v < V; v += 64) xs[v] = 0;
      wave_sync();
      switch (I.cell_bytes) {
        case 1: small_store<uint8_t>(cells, xs, V, 0, lane); break;
        case 2: small_store<uint16_t>(cells, xs, V, 0, lane); break;
        case 4: small_store<uint32_t>(cells, xs, V, 0, lane); break;
        default: small_store<uint64_t>(cells, xs, V, 0, lane); break;
      }
      if (lane == 0) A.tseed[q] = 255;
    }
    wave_sync();
  }
}

hipError_t launch_small(const BuildArgs &a, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_small, dim3((uint32_t)nwg), dim3(64 * kSmallWaves), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ query

// Each thread answers QP queries that are a grid apart (coalesced per
// step): the loads of the QP independent queries are in flight together.
// The local seeds are copied to LDS when they fit (up to kSeedLds shards),
// which leaves the three cell probes as the only gathers from memory.
constexpr uint32_t kSeedLds = 16384;

template <typename T, int QP>
__global__ void __launch_bounds__(256) k_query(Geo G, const T *__restrict__ cells,
                                               const uint8_t *__restrict__ tseed,
                                               const uint64_t *__restrict__ keys, uint64_t n,
                                               void *__restrict__ out) {
  extern __shared__ uint8_t seeds_lds[];
  const bool lds_seeds = G.S <= kSeedLds;
  if (lds_seeds) {
    for (uint32_t i = threadIdx.x; i < G.S; i += blockDim.x) seeds_lds[i] = tseed[i];
    __syncthreads();
  }
  const uint8_t *const ts = lds_seeds ? seeds_lds : tseed;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i0 < n;
       i0 += stride * QP) {
    uint64_t hi[QP], lo[QP];
#pragma unroll
    for (int k = 0; k < QP; k++) {
      const uint64_t i = i0 + (uint64_t)k * stride;
      const uint64_t key = i < n ? keys[i] : 0ull;
      hi[k] = fin64(key ^ G.khi);
      lo[k] = fin64(key ^ G.klo);
    }
    uint32_t t[QP];
#pragma unroll
    for (int k = 0; k < QP; k++) t[k] = ts[shard_of(hi[k], G.h)];
    T x[QP];
#pragma unroll
    for (int k = 0; k < QP; k++) {
      uint32_t v0, v1, v2;
      edge3(G, hi[k], lo[k], t[k], v0, v1, v2);
      const T *w = cells + (uint64_t)shard_of(hi[k], G.h) * G.V;
      x[k] = w[v0] ^ w[v1] ^ w[v2];
    }
#pragma unroll
    for (int k = 0; k < QP; k++) {
      const uint64_t i = i0 + (uint64_t)k * stride;
      if (i < n) {
        if (G.is_filter) ((uint8_t *)out)[i] = (uint64_t)x[k] == fingerprint(G, hi[k], lo[k]);
        else ((T *)out)[i] = x[k];
      }
    }
  }
}

// ------------------------------------------------------------ packed cells
//
// A structure may keep its cells as one little-endian bit string of b-bit
// fields: cell i at bits [i b, i b + b) of consecutive 64-bit words (the
// paper's bit-array storage of values of any width, section 5).  The build
// works on byte-aligned cells in the workspace and packs them at the end.

__device__ __forceinline__ uint64_t packed_get(const uint64_t *__restrict__ w, uint64_t i,
                                               uint32_t b) {
  const uint64_t bit = i * b;
  const uint64_t q = bit >> 6;
  const uint32_t sh = (uint32_t)bit & 63u;
  uint64_t x = w[q] >> sh;
  if (sh + b > 64) x |= w[q + 1] << (64 - sh);
  return b >= 64 ? x : x & ((1ull << b) - 1);
}

// Word j of the packed string of count cells (each in[i] holds b bits).
template <typename T>
__device__ __forceinline__ uint64_t pack_word(const T *__restrict__ in, uint64_t count,
                                              uint32_t b, uint64_t j) {
  const uint64_t lo = j * 64, hi = lo + 64;
  const uint64_t mask = b >= 64 ? ~0ull : (1ull << b) - 1;
  uint64_t acc = 0;
  for (uint64_t i = lo / b; i < count && i * b < hi; i++) {
    const uint64_t v = (uint64_t)in[i] & mask;
    const uint64_t at = i * b;
    acc |= at >= lo ? v << (at - lo) : v >> (lo - at);
  }
  return acc;
}

template <typename T>
__global__ void __launch_bounds__(256) k_pack(const T *__restrict__ in, uint64_t count, uint32_t b,
                                              uint64_t *__restrict__ out, uint64_t nwords,
                                              const uint32_t *__restrict__ abort) {
  if (abort && *abort) return;
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < nwords;
       j += (uint64_t)gridDim.x * blockDim.x)
    out[j] = pack_word(in, count, b, j);
}

// Packing of a batch: instance i's cells at src[i].cell_off bytes of `in`
// (byte-aligned cells of src[i].cell_bytes) go to dst[i].cell_off bytes of
// `out` as a packed string of b bits each.
__global__ void __launch_bounds__(256) k_pack_batch(const BatchItem *__restrict__ src,
                                                    const BatchItem *__restrict__ dst,
                                                    uint64_t count, const uint8_t *__restrict__ in,
                                                    uint8_t *__restrict__ out,
                                                    const uint32_t *__restrict__ abort) {
  if (abort && *abort) return;
  for (uint64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const BatchItem I = src[it];
    uint64_t *const o = (uint64_t *)(out + dst[it].cell_off);
    const uint64_t nw = (I.V * I.b + 63) / 64;
    const uint8_t *const c = in + I.cell_off;
    for (uint64_t j = threadIdx.x; j < nw; j += blockDim.x) {
      uint64_t w;
      switch (I.cell_bytes) {
        case 1: w = pack_word((const uint8_t *)c, I.V, I.b, j); break;
        case 2: w = pack_word((const uint16_t *)c, I.V, I.b, j); break;
        case 4: w = pack_word((const uint32_t *)c, I.V, I.b, j); break;
        default: w = pack_word((const uint64_t *)c, I.V, I.b, j); break;
      }
      o[j] = w;
    }
  }
}

// k_query on packed cells (T: the answer type of a function).
template <typename T, int QP>
__global__ void __launch_bounds__(256) k_query_packed(Geo G, const uint64_t *__restrict__ words,
                                                      const uint8_t *__restrict__ tseed,
                                                      const uint64_t *__restrict__ keys,
                                                      uint64_t n, void *__restrict__ out) {
  extern __shared__ uint8_t seeds_lds[];
  const bool lds_seeds = G.S <= kSeedLds;
  if (lds_seeds) {
    for (uint32_t i = threadIdx.x; i < G.S; i += blockDim.x) seeds_lds[i] = tseed[i];
    __syncthreads();
  }
  const uint8_t *const ts = lds_seeds ? seeds_lds : tseed;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i0 < n;
       i0 += stride * QP) {
    uint64_t hi[QP], lo[QP];
#pragma unroll
    for (int k = 0; k < QP; k++) {
      const uint64_t i = i0 + (uint64_t)k * stride;
      const uint64_t key = i < n ? keys[i] : 0ull;
      hi[k] = fin64(key ^ G.khi);
      lo[k] = fin64(key ^ G.klo);
    }
    uint64_t x[QP];
#pragma unroll
    for (int k = 0; k < QP; k++) {
      const uint32_t j = shard_of(hi[k], G.h);
      uint32_t v0, v1, v2;
      edge3(G, hi[k], lo[k], ts[j], v0, v1, v2);
      const uint64_t base = (uint64_t)j * G.V;
      x[k] = packed_get(words, base + v0, G.b) ^ packed_get(words, base + v1, G.b) ^
             packed_get(words, base + v2, G.b);
    }
#pragma unroll
    for (int k = 0; k < QP; k++) {
      const uint64_t i = i0 + (uint64_t)k * stride;
      if (i < n) {
        if (G.is_filter) ((uint8_t *)out)[i] = x[k] == fingerprint(G, hi[k], lo[k]);
        else ((T *)out)[i] = (T)x[k];
      }
    }
  }
}

// Query of keys grouped by shard (section 4: a key's shard is fixed by its
// signature, so the queries of one shard need only that shard's cells).  A
// workgroup takes whole shards: it copies the shard's cells to LDS (the
// launcher only runs when they fit), then answers the shard's keys
// bkeys[off[j] .. off[j+1]) with three LDS probes each and writes each
// answer to its original position out[bidx[p]], or, with ans, in grouped
// order to ans[p] for k_place_rows to move.
constexpr uint32_t kGroupThreads = 1024;
constexpr int kGroupQP = 4;
constexpr uint64_t kGroupLdsMax = kLdsBudget - 256;

template <typename T, int MODE>
__global__ void __launch_bounds__(kGroupThreads) k_query_grouped(
    Geo G, const T *__restrict__ cells, const uint8_t *__restrict__ tseed,
    const uint64_t *__restrict__ off, const uint64_t *__restrict__ bkeys,
    const uint32_t *__restrict__ bidx, void *__restrict__ out, void *__restrict__ ans,
    uint32_t vb) {
  extern __shared__ uint4 cells_lds[];
  // V cells of a shard are a whole number of 16-byte words and start
  // 16-byte aligned (checked by the launcher)
  const uint32_t n16 = (uint32_t)((G.V * sizeof(T)) >> 4);
  const T *const w = (const T *)cells_lds;
  for (uint32_t j = blockIdx.x; j < G.S; j += gridDim.x) {
    const uint64_t p0 = off[j], p1 = off[j + 1];
    if (p0 == p1) continue;
    const uint4 *src = (const uint4 *)(cells + (uint64_t)j * G.V);
    for (uint32_t i = threadIdx.x; i < n16; i += kGroupThreads) cells_lds[i] = src[i];
    __syncthreads();
    if (MODE == 2) {
      // one word per query (k_scatter_rows<2>): segment, offsets, fingerprint
      const uint32_t sg = G.sigma, ss = 1u << sg;
      const uint64_t gm = (1ull << vb) - 1, om = ss - 1;
      const uint32_t fsh = vb + 3 * sg;
      const uint64_t fm = G.b >= 48 ? ~0ull : (1ull << G.b) - 1;
      for (uint64_t q0 = p0 + threadIdx.x; q0 < p1; q0 += (uint64_t)kGroupThreads * kGroupQP) {
        uint64_t pk[kGroupQP];
#pragma unroll
        for (int k = 0; k < kGroupQP; k++) {
          const uint64_t q = q0 + (uint64_t)k * kGroupThreads;
          pk[k] = q < p1 ? bkeys[q] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < kGroupQP; k++) {
          const uint64_t q = q0 + (uint64_t)k * kGroupThreads;
          if (q < p1) {
            const uint32_t g = (uint32_t)(pk[k] & gm);
            const uint32_t v0 = g * ss + (uint32_t)((pk[k] >> vb) & om);
            const uint32_t v1 = (g + 1) * ss + (uint32_t)((pk[k] >> (vb + sg)) & om);
            const uint32_t v2 = (g + 2) * ss + (uint32_t)((pk[k] >> (vb + 2 * sg)) & om);
            const T x = w[v0] ^ w[v1] ^ w[v2];
            if (G.is_filter) ((uint8_t *)ans)[q] = (uint64_t)x == ((pk[k] >> fsh) & fm);
            else ((T *)ans)[q] = x;
          }
        }
      }
      __syncthreads();
      continue;
    }
    if (MODE == 1) {
      // packed edges (k_scatter_rows<1>): no hashing here
      const uint64_t vm = (1ull << vb) - 1;
      for (uint64_t q0 = p0 + threadIdx.x; q0 < p1; q0 += (uint64_t)kGroupThreads * kGroupQP) {
        uint64_t pk[kGroupQP];
        uint32_t dst[kGroupQP];
#pragma unroll
        for (int k = 0; k < kGroupQP; k++) {
          const uint64_t q = q0 + (uint64_t)k * kGroupThreads;
          pk[k] = q < p1 ? bkeys[q] : 0ull;
          dst[k] = q < p1 && !ans ? bidx[q] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kGroupQP; k++) {
          const uint64_t q = q0 + (uint64_t)k * kGroupThreads;
          if (q < p1) {
            const T x = w[pk[k] & vm] ^ w[(pk[k] >> vb) & vm] ^ w[(pk[k] >> (2 * vb)) & vm];
            if (G.is_filter) {
              const uint8_t a = (uint64_t)x == (pk[k] >> (3 * vb));
              if (ans) ((uint8_t *)ans)[q] = a;
              else ((uint8_t *)out)[dst[k]] = a;
            } else {
              if (ans) ((T *)ans)[q] = x;
              else ((T *)out)[dst[k]] = x;
            }
          }
        }
      }
      __syncthreads();
      continue;
    }
    const uint32_t t = tseed[j];
    for (uint64_t q0 = p0 + threadIdx.x; q0 < p1; q0 += (uint64_t)kGroupThreads * kGroupQP) {
      uint64_t hi[kGroupQP], lo[kGroupQP];
      uint32_t dst[kGroupQP];
#pragma unroll
      for (int k = 0; k < kGroupQP; k++) {
        const uint64_t q = q0 + (uint64_t)k * kGroupThreads;
        const uint64_t key = q < p1 ? bkeys[q] : 0ull;
        dst[k] = q < p1 && !ans ? bidx[q] : 0u;
        hi[k] = fin64(key ^ G.khi);
        lo[k] = fin64(key ^ G.klo);
      }
#pragma unroll
      for (int k = 0; k < kGroupQP; k++) {
        const uint64_t q = q0 + (uint64_t)k * kGroupThreads;
        if (q < p1) {
          uint32_t v0, v1, v2;
          edge3(G, hi[k], lo[k], t, v0, v1, v2);
          const T x = w[v0] ^ w[v1] ^ w[v2];
          if (ans) {
            if (G.is_filter) ((uint8_t *)ans)[q] = (uint64_t)x == fingerprint(G, hi[k], lo[k]);
            else ((T *)ans)[q] = x;
          } else {
            if (G.is_filter) ((uint8_t *)out)[dst[k]] = (uint64_t)x == fingerprint(G, hi[k], lo[k]);
            else ((T *)out)[dst[k]] = x;
          }
        }
      }
    }
    __syncthreads();
  }
}

// Query of a batch of unsharded functions: instance inst[i]'s geometry
// comes from its descriptor; the answer is widened to 64 bits.
__global__ void __launch_bounds__(256) k_query_batch(Geo G, const BatchItem *__restrict__ items,
                                                     uint64_t count,
                                                     const uint8_t *__restrict__ cells,
                                                     const uint8_t *__restrict__ tseed,
                                                     const uint32_t *__restrict__ inst,
                                                     const uint64_t *__restrict__ keys, uint64_t n,
                                                     uint64_t *__restrict__ out, uint32_t packed) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t q = inst[i];
    if (q >= count) {
      out[i] = ~0ull;
      continue;
    }
    const BatchItem it = items[q];
    Geo g = G;
    g.V = it.V;
    g.l = it.l;
    g.sigma = it.sigma;
    g.h = 0;
    const uint64_t key = keys[i];
    const uint64_t hi = fin64(key ^ G.khi), lo = fin64(key ^ G.klo);
    uint32_t v0, v1, v2;
    edge3(g, hi, lo, tseed[q], v0, v1, v2);
    const uint8_t *w = cells + it.cell_off;
    uint64_t x;
    if (packed) {
      const uint64_t *pw = (const uint64_t *)w;
      out[i] = packed_get(pw, v0, it.b) ^ packed_get(pw, v1, it.b) ^ packed_get(pw, v2, it.b);
      continue;
    }
    switch (it.cell_bytes) {
      case 1: x = (uint64_t)(w[v0] ^ w[v1] ^ w[v2]); break;
      case 2: {
        const uint16_t *c = (const uint16_t *)w;
        x = (uint64_t)(c[v0] ^ c[v1] ^ c[v2]);
        break;
      }
      case 4: {
        const uint32_t *c = (const uint32_t *)w;
        x = (uint64_t)(c[v0] ^ c[v1] ^ c[v2]);
        break;
      }
      default: {
        const uint64_t *c = (const uint64_t *)w;
        x = c[v0] ^ c[v1] ^ c[v2];
        break;
      }
    }
    out[i] = x;
  }
}

// Build order: shards with more keys first.  A shard's 2-core, and with it
// its elimination time, grows quickly with its load, so handing out the
// largest shards first leaves the quick ones for the end of the launch.
// Shards are bucketed by M - count (deficits of 1023 or more share the last
// bucket); the order inside a bucket is arbitrary.
__global__ void __launch_bounds__(1024) k_order(const uint32_t *__restrict__ counts, uint32_t S,
                                                uint32_t M, uint32_t *__restrict__ list) {
  __shared__ uint32_t hist[1024];
  const uint32_t tid = threadIdx.x;
  hist[tid] = 0;
  __syncthreads();
  for (uint32_t j = tid; j < S; j += 1024) atomicAdd(&hist[min(M - counts[j], 1023u)], 1u);
  __syncthreads();
  // exclusive prefix sum over the 1024 buckets
  const uint32_t own = hist[tid];
  uint32_t inc = own;
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    __syncthreads();
    const uint32_t y = tid >= d ? hist[tid - d] : 0u;
    __syncthreads();
    inc += y;
    hist[tid] = inc;
  }
  __syncthreads();
  hist[tid] = inc - own;
  __syncthreads();
  for (uint32_t j = tid; j < S; j += 1024) {
    const uint32_t pos = atomicAdd(&hist[min(M - counts[j], 1023u)], 1u);
    list[2 * pos] = j;
    list[2 * pos + 1] = 0;
  }
}

// ----------------------------------------------------------------- launch

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  if (!n) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_pack_checked(const void *in, uint32_t cell_bytes, uint64_t count, uint32_t b,
                               uint64_t *out, const uint32_t *abort, hipStream_t s) {
  const uint64_t nw = (count * b + 63) / 64;
  if (!nw) return hipSuccess;
  uint64_t blocks = (nw + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  switch (cell_bytes) {
    case 1: hipLaunchKernelGGL(k_pack<uint8_t>, dim3((uint32_t)blocks), dim3(256), 0, s, (const uint8_t *)in, count, b, out, nw, abort); break;
    case 2: hipLaunchKernelGGL(k_pack<uint16_t>, dim3((uint32_t)blocks), dim3(256), 0, s, (const uint16_t *)in, count, b, out, nw, abort); break;
    case 4: hipLaunchKernelGGL(k_pack<uint32_t>, dim3((uint32_t)blocks), dim3(256), 0, s, (const uint32_t *)in, count, b, out, nw, abort); break;
    default: hipLaunchKernelGGL(k_pack<uint64_t>, dim3((uint32_t)blocks), dim3(256), 0, s, (const uint64_t *)in, count, b, out, nw, abort); break;
  }
  return hipGetLastError();
}

hipError_t launch_pack(const void *in, uint32_t cell_bytes, uint64_t count, uint32_t b,
                       uint64_t *out, hipStream_t s) {
  return launch_pack_checked(in, cell_bytes, count, b, out, nullptr, s);
}

hipError_t launch_pack_batch(const BatchItem *src, const BatchItem *dst, uint64_t count,
                             const uint8_t *in, uint8_t *out, const uint32_t *abort,
                             hipStream_t s) {
  if (!count) return hipSuccess;
  const uint64_t blocks = count < 65536 ? count : 65536;
  hipLaunchKernelGGL(k_pack_batch, dim3((uint32_t)blocks), dim3(256), 0, s, src, dst, count, in,
                     out, abort);
  return hipGetLastError();
}

// Bit 1 of meta[1] when the largest shard (meta[0], from k_scan) exceeds
// the bound the structure was sized for.
__global__ void k_check_bound(uint32_t *meta, uint32_t cap) {
  if (threadIdx.x == 0 && meta[0] > cap) atomicOr(&meta[1], 2u);
}

hipError_t launch_check_bound(uint32_t *meta, uint32_t cap, hipStream_t s) {
  hipLaunchKernelGGL(k_check_bound, dim3(1), dim3(64), 0, s, meta, cap);
  return hipGetLastError();
}

hipError_t launch_check_values(const uint64_t *vals, uint64_t n, uint32_t b, uint32_t *flag,
                              hipStream_t s) {
  if (!n || b >= 64) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_check_values, dim3((uint32_t)blocks), dim3(256), 0, s, vals, n, b, flag);
  return hipGetLastError();
}

hipError_t launch_check_batch_values(const BatchItem *items, uint64_t count, const uint64_t *vals,
                                    uint32_t *flag, hipStream_t s) {
  if (!count) return hipSuccess;
  const uint64_t blocks = count < 65536 ? count : 65536;
  hipLaunchKernelGGL(k_check_batch_values, dim3((uint32_t)blocks), dim3(256), 0, s, items, count,
                     vals, flag);
  return hipGetLastError();
}

hipError_t launch_count(const uint64_t *keys, uint64_t n, uint64_t khi, uint32_t h,
                        uint32_t S, uint32_t *counts, int ncu, hipStream_t s) {
  if (!n) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  uint64_t cap = (uint64_t)ncu * (S <= 1024 ? 8 : 4);
  if (blocks > cap) blocks = cap;
  size_t shm = S <= kLdsHistMax ? (size_t)S * 4 : 0;
  hipLaunchKernelGGL(k_count, dim3((uint32_t)blocks), dim3(256), shm, s, keys, n, khi, h, S,
                     counts);
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *counts, uint32_t S, uint64_t *offsets,
                       uint64_t *cursor, uint32_t *max_out, hipStream_t s,
                       uint32_t *clear) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, S, offsets, cursor, max_out,
                     clear);
  return hipGetLastError();
}

hipError_t launch_order(const uint32_t *counts, uint32_t S, uint32_t M, uint32_t *list,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, s, counts, S, M, list);
  return hipGetLastError();
}

hipError_t launch_scatter(const uint64_t *keys, const uint64_t *vals, uint64_t n,
                          uint64_t khi, uint32_t h, uint32_t S, uint64_t *cursor,
                          uint64_t *bkeys, uint64_t *bvals, uint32_t *bidx, int ncu,
                          hipStream_t s) {
  if (!n) return hipSuccess;
  const uint64_t chunk = (uint64_t)kScatterThreads * kScatterPer;
  uint64_t blocks = (n + chunk - 1) / chunk;
  uint64_t cap = (uint64_t)ncu * 4;
  if (blocks > cap) blocks = cap;
  size_t shm = S <= kScatterLdsMax ? (size_t)S * 12 : 0;
  hipLaunchKernelGGL(k_scatter, dim3((uint32_t)blocks), dim3(kScatterThreads), shm, s, keys, vals,
                     n, khi, h, S, (unsigned long long *)cursor, bkeys, bvals, bidx);
  return hipGetLastError();
}

template <typename T, int QM, bool TR = false>
static hipError_t set_build_lds(uint32_t lds_bytes) {
  // largest dynamic LDS set so far, per device: a launch within it makes no
  // attribute call (none is made while a stream is being captured then)
  constexpr int kDevs = 64;
  static std::atomic<uint32_t> done[kDevs];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  const bool cached = dev >= 0 && dev < kDevs;
  if (cached && done[dev].load(std::memory_order_relaxed) >= lds_bytes) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute((const void *)k_build<T, QM, TR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_bytes);
  if (e == hipSuccess && cached) {
    uint32_t cur = done[dev].load(std::memory_order_relaxed);
    while (cur < lds_bytes && !done[dev].compare_exchange_weak(cur, lds_bytes)) {
    }
  }
  return e;
}

template <typename T, int QM, bool TR = false>
static hipError_t launch_build_q(const BuildArgs &a, int nwg, hipStream_t s) {
  const hipError_t e = set_build_lds<T, QM, TR>(a.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_build<T, QM, TR>), dim3(nwg), dim3(kBuildThreads), a.lds_bytes, s, a);
  return hipGetLastError();
}

// The elimination keeps up to QM slot groups of 64 window rows in
// registers; fewer groups mean fewer instructions per column.
template <typename T>
static hipError_t launch_build_t(const BuildArgs &a, int nwg, hipStream_t s) {
  if (a.ring_cols) return launch_build_q<T, 8, true>(a, nwg, s);  // test builds
  return a.wmax <= 256   ? launch_build_q<T, 4>(a, nwg, s)
         : a.wmax <= 384 ? launch_build_q<T, 6>(a, nwg, s)
                         : launch_build_q<T, 8>(a, nwg, s);
}

template <typename T, int QM>
static int build_occ_q(uint32_t lds_bytes) {
  int nb = 0;
  if (set_build_lds<T, QM>(lds_bytes) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_build<T, QM, false>,
                                                  (int)kBuildThreads, lds_bytes) != hipSuccess)
    return 0;
  return nb;
}

template <typename T>
static int build_occ_t(uint32_t wmax, uint32_t lds_bytes) {
  return wmax <= 256   ? build_occ_q<T, 4>(lds_bytes)
         : wmax <= 384 ? build_occ_q<T, 6>(lds_bytes)
                       : build_occ_q<T, 8>(lds_bytes);
}

int build_blocks_per_cu(uint32_t cell_bytes, uint32_t wmax, uint32_t lds_bytes) {
  switch (cell_bytes) {
    case 1: return build_occ_t<uint8_t>(wmax, lds_bytes);
    case 2: return build_occ_t<uint16_t>(wmax, lds_bytes);
    case 4: return build_occ_t<uint32_t>(wmax, lds_bytes);
    default: return build_occ_t<uint64_t>(wmax, lds_bytes);
  }
}

template <typename T>
static hipError_t prepare_build_t(const BuildArgs &a) {
  if (a.ring_cols) return set_build_lds<T, 8, true>(a.lds_bytes);
  return a.wmax <= 256   ? set_build_lds<T, 4>(a.lds_bytes)
         : a.wmax <= 384 ? set_build_lds<T, 6>(a.lds_bytes)
                         : set_build_lds<T, 8>(a.lds_bytes);
}

hipError_t prepare_build(const BuildArgs &a) {
  switch (a.cell_bytes) {
    case 1: return prepare_build_t<uint8_t>(a);
    case 2: return prepare_build_t<uint16_t>(a);
    case 4: return prepare_build_t<uint32_t>(a);
    default: return prepare_build_t<uint64_t>(a);
  }
}

hipError_t launch_build(const BuildArgs &a, int nwg, hipStream_t s) {
  switch (a.cell_bytes) {
    case 1: return launch_build_t<uint8_t>(a, nwg, s);
    case 2: return launch_build_t<uint16_t>(a, nwg, s);
    case 4: return launch_build_t<uint32_t>(a, nwg, s);
    default: return launch_build_t<uint64_t>(a, nwg, s);
  }
}

// Query requests against several structures (functions and filters of any
// geometry, byte or packed cells) in one launch: a thread finds the request
// of its combined index by binary search over the request starts.
__global__ void __launch_bounds__(256) k_query_multi(MultiArgs A) {
  const uint64_t total = A.start[A.count];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total; i += stride) {
    uint32_t r = 0;
#pragma unroll
    for (uint32_t step = kMultiMax / 2; step; step >>= 1)
      if (r + step < A.count && A.start[r + step] <= i) r += step;
    const MultiReq &q = A.req[r];
    const uint64_t o = i - A.start[r];
    const uint64_t key = q.keys[o];
    const uint64_t hi = fin64(key ^ q.G.khi), lo = fin64(key ^ q.G.klo);
    const uint32_t j = shard_of(hi, q.G.h);
    uint32_t v0, v1, v2;
    edge3(q.G, hi, lo, q.tseed[j], v0, v1, v2);
    const uint64_t base = (uint64_t)j * q.G.V;
    uint64_t x;
    if (q.packed) {
      const uint64_t *w = (const uint64_t *)q.cells;
      x = packed_get(w, base + v0, q.G.b) ^ packed_get(w, base + v1, q.G.b) ^
          packed_get(w, base + v2, q.G.b);
    } else {
      switch (q.cell_bytes) {
        case 1: {
          const uint8_t *w = (const uint8_t *)q.cells + base;
          x = w[v0] ^ w[v1] ^ w[v2];
        } break;
        case 2: {
          const uint16_t *w = (const uint16_t *)q.cells + base;
          x = w[v0] ^ w[v1] ^ w[v2];
        } break;
        case 4: {
          const uint32_t *w = (const uint32_t *)q.cells + base;
          x = w[v0] ^ w[v1] ^ w[v2];
        } break;
        default: {
          const uint64_t *w = (const uint64_t *)q.cells + base;
          x = w[v0] ^ w[v1] ^ w[v2];
        } break;
      }
    }
    if (q.G.is_filter) {
      ((uint8_t *)q.out)[o] = x == fingerprint(q.G, hi, lo);
    } else {
      switch (q.cell_bytes) {
        case 1: ((uint8_t *)q.out)[o] = (uint8_t)x; break;
        case 2: ((uint16_t *)q.out)[o] = (uint16_t)x; break;
        case 4: ((uint32_t *)q.out)[o] = (uint32_t)x; break;
        default: ((uint64_t *)q.out)[o] = x; break;
      }
    }
  }
}

hipError_t launch_query_multi(const MultiArgs &a, int ncu, hipStream_t s) {
  const uint64_t total = a.start[a.count];
  if (!total) return hipSuccess;
  uint64_t blocks = (total + 255) / 256;
  const uint64_t cap = (uint64_t)ncu * 8;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(k_query_multi, dim3((uint32_t)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_query_batch(const Geo &G, const BatchItem *items, uint64_t count,
                              const uint8_t *cells, const uint8_t *tseed, const uint32_t *inst,
                              const uint64_t *keys, uint64_t n, uint64_t *out, int ncu,
                              hipStream_t s, bool packed) {
  if (!n) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  const uint64_t cap = (uint64_t)ncu * 16;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(k_query_batch, dim3((uint32_t)blocks), dim3(256), 0, s, G, items, count,
                     cells, tseed, inst, keys, n, out, packed ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_query(const Geo &G, const void *cells, uint32_t cell_bytes,
                        const uint8_t *tseed, const uint64_t *keys, uint64_t n,
                        void *out, int ncu, hipStream_t s, bool packed) {
  if (!n) return hipSuccess;
  constexpr int QP = 4;
  // 8 workgroups of 4 wavefronts per CU, each thread QP queries per step
  uint64_t blocks = (n + 256 * QP - 1) / (256 * QP);
  const uint64_t cap = (uint64_t)ncu * 8;
  if (blocks > cap) blocks = cap;
  dim3 g((uint32_t)blocks), b(256);
  const size_t shm = G.S <= kSeedLds ? G.S : 0;
  if (packed) {
    const uint64_t *w = (const uint64_t *)cells;
    switch (cell_bytes) {
      case 1: hipLaunchKernelGGL((k_query_packed<uint8_t, QP>), g, b, shm, s, G, w, tseed, keys, n, out); break;
      case 2: hipLaunchKernelGGL((k_query_packed<uint16_t, QP>), g, b, shm, s, G, w, tseed, keys, n, out); break;
      case 4: hipLaunchKernelGGL((k_query_packed<uint32_t, QP>), g, b, shm, s, G, w, tseed, keys, n, out); break;
      default: hipLaunchKernelGGL((k_query_packed<uint64_t, QP>), g, b, shm, s, G, w, tseed, keys, n, out); break;
    }
    return hipGetLastError();
  }
  switch (cell_bytes) {
    case 1: hipLaunchKernelGGL((k_query<uint8_t, QP>), g, b, shm, s, G, (const uint8_t *)cells, tseed, keys, n, out); break;
    case 2: hipLaunchKernelGGL((k_query<uint16_t, QP>), g, b, shm, s, G, (const uint16_t *)cells, tseed, keys, n, out); break;
    case 4: hipLaunchKernelGGL((k_query<uint32_t, QP>), g, b, shm, s, G, (const uint32_t *)cells, tseed, keys, n, out); break;
    default: hipLaunchKernelGGL((k_query<uint64_t, QP>), g, b, shm, s, G, (const uint64_t *)cells, tseed, keys, n, out); break;
  }
  return hipGetLastError();
}

bool group_rows_fit(uint32_t S) { return S <= kRowMaxS; }
uint64_t group_rows_words(uint32_t S) { return (uint64_t)kRowBlocksMax * S; }

static void group_rows_split(uint64_t n, uint64_t *nblk, uint64_t *seg) {
  uint64_t b = (n + kRowSub - 1) / kRowSub;
  if (b > kRowBlocksMax) b = kRowBlocksMax;
  *nblk = b;
  *seg = (n + b - 1) / b;
}

bool place_fits(uint32_t S, uint64_t n, uint32_t ob) {
  uint64_t nblk, seg;
  group_rows_split(n, &nblk, &seg);
  return S <= kRowMaxS && place_lds_bytes(S, seg, ob) != 0;
}

hipError_t launch_count_rows(const uint64_t *keys, uint64_t n, uint64_t khi, uint32_t h,
                             uint32_t S, uint32_t *rows, uint32_t *totals, hipStream_t s) {
  if (!n || S > kRowMaxS || n > 0xFFFFFFFFull) return hipErrorInvalidValue;
  uint64_t nblk, seg;
  group_rows_split(n, &nblk, &seg);
  hipLaunchKernelGGL(k_count_rows, dim3((uint32_t)nblk), dim3(kRowThreads), (size_t)S * 4, s,
                     keys, n, seg, khi, h, S, rows, totals);
  return hipGetLastError();
}

bool pack_fits(const Geo &G, uint32_t S, uint32_t *vb) {
  uint32_t w = 1;
  while (w < 21 && (1ull << w) < G.V) w++;
  *vb = w;
  return S <= kPackMaxS && (1ull << w) >= G.V && 3 * w + (G.is_filter ? G.b : 0u) <= 64;
}

bool pack_compact_fits(const Geo &G, uint32_t S, uint64_t n, uint32_t *gb) {
  uint32_t w = 1;
  while (w < 32 && (1ull << w) < G.l) w++;
  *gb = w;
  uint64_t nblk, seg;
  group_rows_split(n, &nblk, &seg);
  return !G.mwhc && S <= kPackMaxS && seg <= 65536 && (1ull << w) >= G.l &&
         w + 3 * G.sigma + (G.is_filter ? G.b : 0u) <= 48;
}

template <int MODE>
static hipError_t launch_scatter_rows_t(const uint64_t *keys, uint64_t n, uint64_t seg,
                                        uint64_t nblk, uint64_t khi, uint32_t h, uint32_t S,
                                        const uint32_t *rows, uint64_t *cursor, uint64_t *bkeys,
                                        uint32_t *bidx, uint32_t *starts, const Geo &G,
                                        const uint8_t *tseed, uint32_t vb, hipStream_t s) {
  const size_t shm = MODE == 2 ? (size_t)kRowSub2 * 10 + (size_t)S * 12
                               : (size_t)kRowSub * (MODE ? 14 : 12) + (size_t)S * 12;
  hipError_t e = hipFuncSetAttribute((const void *)k_scatter_rows<MODE>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter_rows<MODE>, dim3((uint32_t)nblk), dim3(kRowThreads), shm, s, keys,
                     n, seg, khi, h, S, rows, (unsigned long long *)cursor, bkeys, bidx, starts,
                     G, tseed, vb);
  return hipGetLastError();
}

hipError_t launch_scatter_rows(const uint64_t *keys, uint64_t n, uint64_t khi, uint32_t h,
                               uint32_t S, const uint32_t *rows, uint64_t *cursor,
                               uint64_t *bkeys, uint32_t *bidx, uint32_t *starts, hipStream_t s,
                               int mode, const Geo *G, const uint8_t *tseed, uint32_t vb) {
  if (!n || S > kRowMaxS || n > 0xFFFFFFFFull) return hipErrorInvalidValue;
  if (mode && (!G || !tseed || S > kPackMaxS)) return hipErrorInvalidValue;
  uint64_t nblk, seg;
  group_rows_split(n, &nblk, &seg);
  if (mode == 2 && seg > 65536) return hipErrorInvalidValue;
  const Geo g = G ? *G : Geo{};
  switch (mode) {
    case 0: return launch_scatter_rows_t<0>(keys, n, seg, nblk, khi, h, S, rows, cursor, bkeys, bidx, starts, g, tseed, 0u, s);
    case 1: return launch_scatter_rows_t<1>(keys, n, seg, nblk, khi, h, S, rows, cursor, bkeys, bidx, starts, g, tseed, vb, s);
    default: return launch_scatter_rows_t<2>(keys, n, seg, nblk, khi, h, S, rows, cursor, bkeys, bidx, starts, g, tseed, vb, s);
  }
}

hipError_t launch_group_rows(const uint64_t *keys, uint64_t n, uint64_t khi, uint32_t h,
                             uint32_t S, uint32_t *rows, uint32_t *totals, uint64_t *offsets,
                             uint64_t *cursor, uint32_t *meta, uint64_t *bkeys, uint32_t *bidx,
                             uint32_t *starts, hipStream_t s, int mode, const Geo *G,
                             const uint8_t *tseed, uint32_t vb) {
  hipError_t e = launch_count_rows(keys, n, khi, h, S, rows, totals, s);
  if (e != hipSuccess) return e;
  e = launch_scan(totals, S, offsets, cursor, meta, s, totals);
  if (e != hipSuccess) return e;
  return launch_scatter_rows(keys, n, khi, h, S, rows, cursor, bkeys, bidx, starts, s, mode, G,
                             tseed, vb);
}

template <typename T>
static hipError_t launch_place_t(const uint32_t *rows, const uint32_t *starts, uint32_t S,
                                 uint64_t n, uint64_t nblk, uint64_t seg, uint32_t lds,
                                 const void *ans, const uint32_t *bidx, const uint64_t *bwords,
                                 void *out, hipStream_t s) {
  const void *f = bwords ? (const void *)k_place_rows<T, true> : (const void *)k_place_rows<T, false>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (bwords)
    hipLaunchKernelGGL((k_place_rows<T, true>), dim3((uint32_t)nblk), dim3(kRowThreads), lds, s,
                       rows, starts, S, n, seg, (const T *)ans, bidx, bwords, (T *)out);
  else
    hipLaunchKernelGGL((k_place_rows<T, false>), dim3((uint32_t)nblk), dim3(kRowThreads), lds, s,
                       rows, starts, S, n, seg, (const T *)ans, bidx, bwords, (T *)out);
  return hipGetLastError();
}

hipError_t launch_place_rows(const uint32_t *rows, const uint32_t *starts, uint32_t S,
                             uint64_t n, uint32_t ob, const void *ans, const uint32_t *bidx,
                             const uint64_t *bwords, void *out, hipStream_t s) {
  uint64_t nblk, seg;
  group_rows_split(n, &nblk, &seg);
  const uint32_t lds = place_lds_bytes(S, seg, ob);
  if (!n || S > kRowMaxS || !lds) return hipErrorInvalidValue;
  switch (ob) {
    case 1: return launch_place_t<uint8_t>(rows, starts, S, n, nblk, seg, lds, ans, bidx, bwords, out, s);
    case 2: return launch_place_t<uint16_t>(rows, starts, S, n, nblk, seg, lds, ans, bidx, bwords, out, s);
    case 4: return launch_place_t<uint32_t>(rows, starts, S, n, nblk, seg, lds, ans, bidx, bwords, out, s);
    default: return launch_place_t<uint64_t>(rows, starts, S, n, nblk, seg, lds, ans, bidx, bwords, out, s);
  }
}

uint32_t query_grouped_lds_bytes(const Geo &G, const void *cells, uint32_t cell_bytes) {
  const uint64_t vb = G.V * cell_bytes;
  return vb <= kGroupLdsMax && (vb & 15) == 0 && ((uintptr_t)cells & 15) == 0 ? (uint32_t)vb
                                                                              : 0;
}

template <typename T, int MODE>
static hipError_t launch_query_grouped_t(const Geo &G, const void *cells, const uint8_t *tseed,
                                         const uint64_t *off, const uint64_t *bkeys,
                                         const uint32_t *bidx, void *out, void *ans,
                                         uint32_t vb, uint32_t lds, dim3 g, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void *)k_query_grouped<T, MODE>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_query_grouped<T, MODE>), g, dim3(kGroupThreads), lds, s, G,
                     (const T *)cells, tseed, off, bkeys, bidx, out, ans, vb);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_query_grouped_p(const Geo &G, const void *cells, const uint8_t *tseed,
                                         const uint64_t *off, const uint64_t *bkeys,
                                         const uint32_t *bidx, void *out, void *ans,
                                         uint32_t vb, int mode, uint32_t lds, dim3 g,
                                         hipStream_t s) {
  switch (mode) {
    case 0: return launch_query_grouped_t<T, 0>(G, cells, tseed, off, bkeys, bidx, out, ans, 0, lds, g, s);
    case 1: return launch_query_grouped_t<T, 1>(G, cells, tseed, off, bkeys, bidx, out, ans, vb, lds, g, s);
    default: return launch_query_grouped_t<T, 2>(G, cells, tseed, off, bkeys, bidx, out, ans, vb, lds, g, s);
  }
}

hipError_t launch_query_grouped(const Geo &G, const void *cells, uint32_t cell_bytes,
                                const uint8_t *tseed, const uint64_t *off, const uint64_t *bkeys,
                                const uint32_t *bidx, void *out, void *ans, uint32_t vb,
                                int mode, int ncu, hipStream_t s) {
  const uint32_t lds = query_grouped_lds_bytes(G, cells, cell_bytes);
  if (!lds || (mode == 2 && !ans)) return hipErrorInvalidValue;
  uint64_t blocks = G.S;
  const uint64_t cap = (uint64_t)ncu * 8;
  if (blocks > cap) blocks = cap;
  const dim3 g((uint32_t)blocks);
  switch (cell_bytes) {
    case 1: return launch_query_grouped_p<uint8_t>(G, cells, tseed, off, bkeys, bidx, out, ans, vb, mode, lds, g, s);
    case 2: return launch_query_grouped_p<uint16_t>(G, cells, tseed, off, bkeys, bidx, out, ans, vb, mode, lds, g, s);
    case 4: return launch_query_grouped_p<uint32_t>(G, cells, tseed, off, bkeys, bidx, out, ans, vb, mode, lds, g, s);
    default: return launch_query_grouped_p<uint64_t>(G, cells, tseed, off, bkeys, bidx, out, ans, vb, mode, lds, g, s);
  }
}

}  // namespace vfk
