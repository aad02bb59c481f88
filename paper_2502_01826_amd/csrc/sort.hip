// Steps a3-a4: splat emission into per-tile buckets and the per-tile depth
// sort (App. E: every splat carries the tile index and the distance key; the
// paper sorts them all at once by a 64-bit key, Alg. 1 sphericalSplatting and
// computeGridRange).  Here the tile part of the key is applied by bucketing
// (the tile ranges come from the counts made during projection) and the
// distance part by sorting each bucket in its own workgroup, which gives the
// same order -- (distance key, Gaussian index) within each tile -- with one
// pass over the splats instead of one per key byte.
//
// Each bucket is sorted by one MSD counting pass and a rank within the small
// sub-buckets it makes (below), in LDS for buckets of up to `chunk` entries
// and through global scratch for longer ones.  No workgroup ever waits on
// another, so every wave finishes.
#include <climits>

#include "gsrf_internal.h"

namespace gsrf {

// a3: one splat per covered tile.  The workgroup (RB records of one pair)
// counts its splats per tile in LDS, reserves each tile's share with one
// global atomic on its sub-bucket's cursor, then writes (key, Gaussian) at its
// reserved slots.  With 256 records and at most kEmitCache splats, the first
// pass keeps every splat's (tile, rank in the workgroup's share, record) in
// LDS, so the second pass neither searches nor counts again.
constexpr int kEmitCache = 2048;

template <int RB>
__global__ __launch_bounds__(RB) void k_emit(const gsrf_pair *__restrict__ pairs,
                                              const int64_t *__restrict__ scene_off,
                                              const int64_t *__restrict__ rec_base,
                                              const uint32_t *__restrict__ rec_key,
                                              const ushort4 *__restrict__ rec_rect, int32_t T, int32_t nta, int64_t PT,
                                              const int64_t *__restrict__ counters, uint32_t *__restrict__ tcur,
                                              uint2 *__restrict__ ekv) {
  if (counters[1] != 0) return;  // over capacity: every range is empty, nothing is emitted
  constexpr bool CACHE = RB == 256;   // tile < 2^16, rank < 2^8, record < 2^8
  extern __shared__ uint32_t sm[];
  uint32_t *cnt = sm;        // [T]
  uint32_t *base = sm + T;   // [T]
  __shared__ RectScan<RB> rs;
  __shared__ uint32_t keys[RB];
  __shared__ uint32_t cache[CACHE ? kEmitCache : 1];
  const int k = blockIdx.y;
  for (int t = threadIdx.x; t < T; t += blockDim.x) cnt[t] = 0;
  const int s = pairs[k].scene;
  const int64_t g0 = scene_off[s];
  const int64_t n = scene_off[s + 1] - g0;
  const int64_t j = (int64_t)blockIdx.x * RB + threadIdx.x;
  ushort4 rc = make_ushort4(0, 0, 0, 0);
  uint32_t key = 0;
  if (j < n) {
    const int64_t r = rec_base[k] + j;
    rc = rec_rect[r];
    key = rec_key[r];
  }
  keys[threadIdx.x] = key;
  rect_scan(rs, rc);
  const uint32_t total = rs.off[RB];
  const bool cached = CACHE && total <= (uint32_t)kEmitCache;
  for (uint32_t sp = threadIdx.x; sp < total; sp += RB) {
    int t;
    const int slot = rect_splat(rs, sp, nta, &t);
    const uint32_t rank = atomicAdd(&cnt[t], 1u);
    if (cached) cache[sp] = ((uint32_t)t << 16) | (rank << 8) | (uint32_t)slot;
  }
  __syncthreads();
  // reserve this workgroup's share of each touched tile in sub-bucket b % kSub
  // (four tiles per thread at a time, so that their atomics are in flight together)
  uint32_t *cur = tcur + (size_t)(blockIdx.x % kSub) * PT + (size_t)k * T;
  for (int t0 = threadIdx.x; t0 < T; t0 += 4 * RB) {
    uint32_t r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * RB;
      const uint32_t c = t < T ? cnt[t] : 0u;
      r[u] = c ? atomicAdd(cur + t, c) : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * RB;
      if (t < T) {
        base[t] = r[u];
        cnt[t] = 0;
      }
    }
  }
  __syncthreads();
  const uint32_t gbase = (uint32_t)(g0 + (int64_t)blockIdx.x * RB);
  if (cached) {
    for (uint32_t sp = threadIdx.x; sp < total; sp += RB) {
      const uint32_t c = cache[sp];
      const uint32_t slot = c & 0xFFu;
      ekv[base[c >> 16] + ((c >> 8) & 0xFFu)] = make_uint2(keys[slot], gbase + slot);
    }
  } else {
    for (uint32_t sp = threadIdx.x; sp < total; sp += RB) {
      int t;
      const int slot = rect_splat(rs, sp, nta, &t);
      const uint32_t pos = base[t] + atomicAdd(&cnt[t], 1u);
      ekv[pos] = make_uint2(keys[slot], gbase + (uint32_t)slot);
    }
  }
}

// ---------------------------------------------------------------------------
// a4: per-tile sort by (distance key, Gaussian index), one workgroup per tile.
//
// Each entry is the 64-bit composite c = key << 32 | index (unique within a
// tile).  One MSD counting pass splits the bucket into 2^b sub-buckets (about
// four entries each, b <= 11) by the key's D^2 value scaled linearly between
// the bucket's extremes: histogram, exclusive scan and scatter.  Each entry's final place is then its sub-bucket's start plus its
// rank among the sub-bucket's entries, found by comparing with all of them;
// sub-buckets are small, so this costs a few comparisons per entry and no
// further passes.  The scatter buffer is LDS for buckets of up to `chunk`
// entries; longer buckets scatter to global scratch and are ranked in LDS
// windows of whole sub-buckets.  The result does not depend on the (atomic)
// scatter order, so it is deterministic.
// ---------------------------------------------------------------------------
constexpr int kSortRegs = 8;              // entries per thread held in registers (LDS path)

// Workgroup shapes: 1024 threads (any bucket; up to 2^11 sub-buckets), 512
// threads (buckets of at most 8 x 512 entries, held in registers; 2^10) and 256
// threads (at most 8 x 256 entries; 2^9).
template <int NT>
struct SortShape {
  static constexpr int kWaves = NT / 64;
  static constexpr int kBitsMax = NT >= 1024 ? 11 : NT >= 512 ? 10 : 9;
  static constexpr int kBins = 1 << kBitsMax;
  static constexpr int kRedWords = 4 * kWaves;    // u64: wave min/max, totals, wave sums
};
constexpr int kSortWaves = kTileSortThreads / 64;
constexpr int kSortBitsMax = SortShape<kTileSortThreads>::kBitsMax;
constexpr int kSortBins = SortShape<kTileSortThreads>::kBins;
constexpr int kSmallSortThreads = 256;
constexpr int kSmallSortMax = kSortRegs * kSmallSortThreads;   // 2048 entries
constexpr int kMidSortThreads = 512;
// 3840 of the 4096 entries the registers hold: with 2^10 sub-buckets the
// workgroup's LDS stays under 40 KB, so four workgroups share a CU
constexpr int kMidSortMax = 3840;

__device__ __forceinline__ uint64_t composite(uint32_t k, uint32_t v) { return ((uint64_t)k << 32) | v; }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int d) {
  const uint32_t lo = __shfl_xor((uint32_t)x, d, 64), hi = __shfl_xor((uint32_t)(x >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}

// f(entry) for every entry of a bucket in global memory, kGlobalBatch loads
// per thread in flight at a time (a plain strided loop would wait for each load).
constexpr int kGlobalBatch = 4;

template <int NT, typename F>
__device__ __forceinline__ void for_each_global(const uint2 *__restrict__ ekv, int n, F f) {
  for (int b = 0; b < n; b += kGlobalBatch * NT) {
    uint2 x[kGlobalBatch];
#pragma unroll
    for (int e = 0; e < kGlobalBatch; ++e) {
      const int i = b + (int)threadIdx.x + e * NT;
      x[e] = i < n ? ekv[i] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int e = 0; e < kGlobalBatch; ++e)
      if (b + (int)threadIdx.x + e * NT < n) f(x[e]);
  }
}

// dst[i] = src[i] for i < len, kGlobalBatch loads per thread in flight.
template <int NT>
__device__ __forceinline__ void copy_window(const uint2 *__restrict__ src, uint2 *dst, int len) {
  for (int b = 0; b < len; b += kGlobalBatch * NT) {
    uint2 x[kGlobalBatch];
#pragma unroll
    for (int e = 0; e < kGlobalBatch; ++e) {
      const int i = b + (int)threadIdx.x + e * NT;
      x[e] = i < len ? src[i] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int e = 0; e < kGlobalBatch; ++e) {
      const int i = b + (int)threadIdx.x + e * NT;
      if (i < len) dst[i] = x[e];
    }
  }
}

// Exclusive scan of cnt[0, nbins) into start[0, nbins) by the NT threads;
// CURSOR: cnt is overwritten with the same starts (scatter cursors).
template <int NT, bool CURSOR = false>
__device__ void bins_scan(uint32_t *cnt, uint32_t *start, int nbins, uint32_t *wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (nbins + NT - 1) / NT;
  const int lo = min(nbins, tid * per), hi = min(nbins, lo + per);
  uint32_t local = 0;
  for (int i = lo; i < hi; ++i) local += cnt[i];
  uint32_t inc = local;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t off = 0;
  for (int w = 0; w < wave; ++w) off += wsum[w];
  uint32_t run = off + inc - local;
  for (int i = lo; i < hi; ++i) {
    const uint32_t c = cnt[i];
    start[i] = run;
    if (CURSOR) cnt[i] = run;
    run += c;
  }
}

// a3 for workgroups of RB = 1024 records with at most kEmitStagedTiles tiles:
// the splats are taken kEmitChunk at a time; each chunk is counted per tile
// (one search per splat), its tiles' shares are reserved with one global
// atomic each, and the chunk is placed in LDS in tile order, so that the
// stores to the buckets run over consecutive addresses of each tile's share
// instead of one cache line per lane.
constexpr int kEmitChunk = 4096;
constexpr int kEmitStagedTiles = 1536;

template <int RB>
__global__ __launch_bounds__(RB) void k_emit_staged(const gsrf_pair *__restrict__ pairs,
                                                     const int64_t *__restrict__ scene_off,
                                                     const int64_t *__restrict__ rec_base,
                                                     const uint32_t *__restrict__ rec_key,
                                                     const ushort4 *__restrict__ rec_rect, int32_t T, int32_t nta,
                                                     int64_t PT, const int64_t *__restrict__ counters,
                                                     uint32_t *__restrict__ tcur, uint2 *__restrict__ ekv) {
  if (counters[1] != 0) return;  // over capacity: every range is empty, nothing is emitted
  constexpr int E = kEmitChunk / RB;
  extern __shared__ uint32_t sm[];
  uint32_t *ccnt = sm;            // [T] splats of the chunk per tile
  uint32_t *cstart = sm + T;      // [T] their start in the staged chunk
  uint32_t *cbase = sm + 2 * T;   // [T] their reserved start in the bucket
  __shared__ RectScan<RB> rs;
  __shared__ uint32_t keys[RB];
  __shared__ uint2 stage[kEmitChunk];
  __shared__ uint16_t stile[kEmitChunk];
  __shared__ uint32_t wsum[RB / 64];
  const int tid = threadIdx.x;
  const int k = blockIdx.y;
  for (int t = tid; t < T; t += RB) ccnt[t] = 0;
  const int s = pairs[k].scene;
  const int64_t g0 = scene_off[s];
  const int64_t n = scene_off[s + 1] - g0;
  const int64_t j = (int64_t)blockIdx.x * RB + tid;
  ushort4 rc = make_ushort4(0, 0, 0, 0);
  uint32_t key = 0;
  if (j < n) {
    const int64_t r = rec_base[k] + j;
    rc = rec_rect[r];
    key = rec_key[r];
  }
  keys[tid] = key;
  rect_scan(rs, rc);   // (ends with a barrier: ccnt and keys are visible)
  const uint32_t total = rs.off[RB];
  const uint32_t gbase = (uint32_t)(g0 + (int64_t)blockIdx.x * RB);
  uint32_t *cur = tcur + (size_t)(blockIdx.x % kSub) * PT + (size_t)k * T;
  for (uint32_t c0 = 0; c0 < total; c0 += kEmitChunk) {
    int tt[E], slot[E];
    uint32_t rank[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t sp = c0 + (uint32_t)(tid + e * RB);
      tt[e] = -1;
      if (sp < total) {
        slot[e] = rect_splat(rs, sp, nta, &tt[e]);
        rank[e] = atomicAdd(&ccnt[tt[e]], 1u);
      }
    }
    __syncthreads();
    bins_scan<RB>(ccnt, cstart, T, wsum);
    for (int t = tid; t < T; t += RB) {
      const uint32_t c = ccnt[t];
      if (c) cbase[t] = atomicAdd(cur + t, c);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (tt[e] >= 0) {
        const uint32_t p = cstart[tt[e]] + rank[e];
        stage[p] = make_uint2(keys[slot[e]], gbase + (uint32_t)slot[e]);
        stile[p] = (uint16_t)tt[e];
      }
    __syncthreads();
    const uint32_t m = min((uint32_t)kEmitChunk, total - c0);
    for (uint32_t i = tid; i < m; i += RB) {
      const int t = stile[i];
      ekv[cbase[t] + (i - cstart[t])] = stage[i];
    }
    __syncthreads();
    for (int t = tid; t < T; t += RB) ccnt[t] = 0;
    __syncthreads();
  }
}

// Sort the n entries ekv = (key, value) by composite into (ok, ov) through the scatter
// buffer bkv; SH: the buffer is in LDS, else in global memory and ranked
// through the LDS window skv.  HREGS (global buffer only): the first HREGS * NT
// entries stay in registers across the extremes, histogram and scatter passes,
// and only the rest is read from global memory in each of them.
template <int NT, bool SH, int REGS = kSortRegs, int HREGS = 0>
__device__ __forceinline__ void msd_rank_sort(const uint2 *__restrict__ ekv, int n, uint2 *bkv, uint32_t *__restrict__ ok,
                              uint32_t *__restrict__ ov, uint32_t *hist, uint32_t *start, uint64_t *red, uint2 *skv,
                              int chunk) {
  constexpr int kSortWaves = SortShape<NT>::kWaves, kSortBitsMax = SortShape<NT>::kBitsMax;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // LDS path (n <= REGS * NT): each thread keeps its entries in registers
  // across the passes, so the bucket is read from global memory once
  constexpr int RR = SH ? REGS : HREGS;
  uint32_t rk[RR > 0 ? RR : 1], rv[RR > 0 ? RR : 1];
  const int nr = min(n, RR * NT);   // entries held in registers
#pragma unroll
  for (int e = 0; e < RR; ++e) {
    const int i = tid + e * NT;
    const uint2 x = i < nr ? ekv[i] : make_uint2(0u, 0u);
    rk[e] = x.x;
    rv[e] = x.y;
  }
  const uint2 *gkv = ekv + nr;      // the rest, read in every pass
  const int ng = n - nr;
  uint64_t cmin = ~0ull, cmax = 0;
#pragma unroll
  for (int e = 0; e < RR; ++e)
    if (tid + e * NT < nr) {
      const uint64_t c = composite(rk[e], rv[e]);
      cmin = c < cmin ? c : cmin;
      cmax = c > cmax ? c : cmax;
    }
  if constexpr (!SH) {
    for_each_global<NT>(gkv, ng, [&](uint2 x) {
      const uint64_t c = composite(x.x, x.y);
      cmin = c < cmin ? c : cmin;
      cmax = c > cmax ? c : cmax;
    });
  }
  int bits = 1;
  while (bits < kSortBitsMax && (4 << bits) < n) ++bits;
  const int nbins = 1 << bits;
  // the histogram is cleared before the one barrier of the extremes
  for (int i = tid; i < nbins; i += NT) hist[i] = 0;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t a = shfl_xor_u64(cmin, d), b = shfl_xor_u64(cmax, d);
    cmin = a < cmin ? a : cmin;
    cmax = b > cmax ? b : cmax;
  }
  if (lane == 0) {
    red[wave] = cmin;
    red[kSortWaves + wave] = cmax;
  }
  __syncthreads();
  if (wave == 0) {   // lanes 0..15 fold the wave results
    uint64_t a = lane < kSortWaves ? red[lane] : ~0ull, b = lane < kSortWaves ? red[kSortWaves + lane] : 0ull;
#pragma unroll
    for (int d = kSortWaves / 2; d >= 1; d >>= 1) {
      const uint64_t x = shfl_xor_u64(a, d), y = shfl_xor_u64(b, d);
      a = x < a ? x : a;
      b = y > b ? y : b;
    }
    if (lane == 0) {
      red[2 * kSortWaves] = a;
      red[2 * kSortWaves + 1] = b;
    }
  }
  __syncthreads();
  cmin = red[2 * kSortWaves];
  cmax = red[2 * kSortWaves + 1];
  // sub-bucket of an entry: its depth key's value (D^2) scaled linearly onto
  // [0, nbins) -- monotone in the key, so in the composite; the density of
  // splats grows slowly with D^2 (not like the key bits, which are
  // logarithmic in D^2), so the sub-buckets stay balanced
  const float dlo = __uint_as_float((uint32_t)(cmin >> 32)), dhi = __uint_as_float((uint32_t)(cmax >> 32));
  const float scale = dhi > dlo ? (float)nbins / (dhi - dlo) : 0.f;
  auto digit = [&](uint32_t k) -> uint32_t {   // (a NaN product, from an infinite scale, lands in the last bin)
    const float x = (__uint_as_float(k) - dlo) * scale;
    return x < (float)nbins ? (uint32_t)x : (uint32_t)(nbins - 1);
  };
#pragma unroll
  for (int e = 0; e < RR; ++e)
    if (tid + e * NT < nr) atomicAdd(&hist[digit(rk[e])], 1u);
  if constexpr (!SH) for_each_global<NT>(gkv, ng, [&](uint2 x) { atomicAdd(&hist[digit(x.x)], 1u); });
  __syncthreads();
  bins_scan<NT, true>(hist, start, nbins, (uint32_t *)(red + 2 * kSortWaves + 2));   // hist: scatter cursors
  __syncthreads();
#pragma unroll
  for (int e = 0; e < RR; ++e)
    if (tid + e * NT < nr) {
      const uint32_t p = atomicAdd(&hist[digit(rk[e])], 1u);
      bkv[p] = make_uint2(rk[e], rv[e]);
    }
  if constexpr (!SH) {
    for_each_global<NT>(gkv, ng, [&](uint2 x) {
      const uint32_t p = atomicAdd(&hist[digit(x.x)], 1u);
      bkv[p] = x;
    });
  }
  if (!SH) __threadfence_block();
  __syncthreads();
  // hist[d] is now the end of sub-bucket d
  if constexpr (SH) {
    for (int p = tid; p < n; p += NT) {
      const uint2 kv = bkv[p];
      const uint32_t k = kv.x, v = kv.y;
      const uint64_t c = composite(k, v);
      const uint32_t d = digit(k);
      const int a = (int)start[d], e = (int)hist[d];
      int rank = 0;
#pragma unroll 4
      for (int j = a; j < e; ++j) {
        const uint2 o = bkv[j];
        rank += composite(o.x, o.y) < c ? 1 : 0;
      }
      ok[a + rank] = k;
      ov[a + rank] = v;
    }
  } else {
    // rank in LDS windows of whole sub-buckets (at most `chunk` entries each);
    // a single sub-bucket longer than that is ranked in global memory
    int w0 = 0;
    while (w0 < n) {
      const int lim = min(n, w0 + chunk);
      // last sub-bucket end <= lim (ends are non-decreasing in the digit)
      int lo = 0, hi = nbins - 1, w1 = w0;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int e = (int)hist[mid];
        if (e <= lim) {
          w1 = max(w1, e);
          lo = mid + 1;
        } else {
          hi = mid - 1;
        }
      }
      if (w1 > w0) {
        copy_window<NT>(bkv + w0, skv, w1 - w0);
        __syncthreads();
        for (int p = tid; p < w1 - w0; p += NT) {
          const uint2 kv = skv[p];
          const uint32_t k = kv.x, v = kv.y;
          const uint64_t c = composite(k, v);
          const uint32_t d = digit(k);
          const int a = (int)start[d] - w0, e = (int)hist[d] - w0;
          int rank = 0;
#pragma unroll 4
          for (int j = a; j < e; ++j) {
            const uint2 o = skv[j];
            rank += composite(o.x, o.y) < c ? 1 : 0;
          }
          ok[w0 + a + rank] = k;
          ov[w0 + a + rank] = v;
        }
        __syncthreads();
      } else {
        // the sub-bucket starting at w0 exceeds the window
        const uint32_t d0 = digit(bkv[w0].x);
        w1 = (int)hist[d0];
        for (int p = w0 + tid; p < w1; p += NT) {
          const uint32_t k = bkv[p].x, v = bkv[p].y;
          const uint64_t c = composite(k, v);
          int rank = 0;
          for (int j = w0; j < w1; ++j) rank += composite(bkv[j].x, bkv[j].y) < c ? 1 : 0;
          ok[w0 + rank] = k;
          ov[w0 + rank] = v;
        }
      }
      w0 = w1;
    }
  }
}

// One bucket by the 1024-thread workgroup: in LDS up to `chunk` entries
// (REGS * 1024 at most), else through the global scratch tkv, with the first
// REGS * 1024 entries kept in registers when REGS exceeds kSortRegs.
template <int REGS = kSortRegs>
__device__ __forceinline__ void sort_bucket(const uint2 *__restrict__ ekv, uint32_t s0, int n, int chunk,
                                            uint32_t *__restrict__ klo, uint32_t *__restrict__ val,
                                            uint2 *__restrict__ tkv, uint32_t *hist, uint32_t *start,
                                            uint64_t *red, uint2 *skv) {
  if (n <= 0) return;
  if (n <= chunk)
    msd_rank_sort<kTileSortThreads, true, REGS>(ekv + s0, n, skv, klo + s0, val + s0, hist, start, red, skv, chunk);
  else
    msd_rank_sort<kTileSortThreads, false, REGS, (REGS > kSortRegs ? REGS : 0)>(ekv + s0, n, tkv + s0, klo + s0,
                                                                               val + s0, hist, start, red, skv, chunk);
}

// a4: sort every tile's bucket; writes the sorted depth keys and Gaussian ids.
__global__ __launch_bounds__(kTileSortThreads, 8) void k_tile_sort(const uint32_t *__restrict__ tstart,
                                                                const uint32_t *__restrict__ tend, int chunk,
                                                                const uint2 *__restrict__ ekv,
                                                                uint32_t *__restrict__ klo, uint32_t *__restrict__ val,
                                                                uint2 *__restrict__ tkv) {
  extern __shared__ uint64_t sm64[];
  uint64_t *red = sm64;                                     // wave min/max, totals, wave sums
  uint32_t *hist = (uint32_t *)(sm64 + 4 * kSortWaves);     // [kSortBins]
  uint32_t *start = hist + kSortBins;                       // [kSortBins]
  uint2 *skv = (uint2 *)(start + kSortBins);                // [chunk]
  const int gt = blockIdx.x;
  const uint32_t s0 = tstart[gt];
  const int n = (int)(tend[gt] - s0);
  sort_bucket(ekv, s0, n, chunk, klo, val, tkv, hist, start, red, skv);
}

// a4 for launches with many tiles, in four kernels by bucket length: one
// 256-thread workgroup per tile sorts the buckets of at most 2048 entries
// (seven per CU), one 512-thread workgroup per tile those of 2049-3840 (four
// per CU), a fixed grid of 1024-thread workgroups with 8 entries per thread
// (two per CU) those up to its LDS chunk, and a fixed grid of 1024-thread
// workgroups with 16 entries per thread (one per CU) the longer ones.  A
// bucket's sort is a chain of dependent steps (load, extremes, histogram,
// scan, scatter, rank, store) that one workgroup cannot overlap, so the
// shortest buckets get the most workgroups in flight.
__global__ __launch_bounds__(kSmallSortThreads) void k_tile_sort_small(const uint32_t *__restrict__ tstart,
                                                                      const uint32_t *__restrict__ tend,
                                                                      const uint2 *__restrict__ ekv,
                                                                      uint32_t *__restrict__ klo,
                                                                      uint32_t *__restrict__ val) {
  constexpr int NT = kSmallSortThreads, NB = SortShape<NT>::kBins;
  __shared__ uint64_t red[SortShape<NT>::kRedWords];
  __shared__ uint32_t hist[NB], start[NB];
  __shared__ uint2 skv[kSmallSortMax];
  const int gt = blockIdx.x;
  const uint32_t s0 = tstart[gt];
  const int n = (int)(tend[gt] - s0);
  if (n <= 0 || n > kSmallSortMax) return;
  msd_rank_sort<NT, true>(ekv + s0, n, skv, klo + s0, val + s0, hist, start, red, skv, kSmallSortMax);
}

__global__ __launch_bounds__(kMidSortThreads) void k_tile_sort_mid(const uint32_t *__restrict__ tstart,
                                                                  const uint32_t *__restrict__ tend,
                                                                  const uint2 *__restrict__ ekv,
                                                                  uint32_t *__restrict__ klo,
                                                                  uint32_t *__restrict__ val) {
  constexpr int NT = kMidSortThreads, NB = SortShape<NT>::kBins;
  __shared__ uint64_t red[SortShape<NT>::kRedWords];
  __shared__ uint32_t hist[NB], start[NB];
  __shared__ uint2 skv[kMidSortMax];
  const int gt = blockIdx.x;
  const uint32_t s0 = tstart[gt];
  const int n = (int)(tend[gt] - s0);
  if (n <= kSmallSortMax || n > kMidSortMax) return;
  msd_rank_sort<NT, true>(ekv + s0, n, skv, klo + s0, val + s0, hist, start, red, skv, kMidSortMax);
}

// The long buckets by 1024-thread workgroups: REGS = 8 (two workgroups per CU,
// 64 VGPRs) for buckets up to that kernel's LDS chunk, REGS = 16 (one per CU,
// a chunk of 16384 entries in 128 KB of LDS) for the longer ones, which beyond
// the chunk go through global memory.  A fixed grid takes the buckets of length
// classes [c_lo, c_hi) of the queue, longest class first, one bucket per
// atomic pop of its kernel's counter (`pop`), until the classes are exhausted.
// Thread 0 runs two buckets ahead: while the workgroup sorts bucket k, the
// (start, entries) of bucket k + 1 and the queue position of bucket k + 2 are
// in flight, so no dependent global access separates two sorts.
template <int REGS>
__global__ __launch_bounds__(kTileSortThreads, REGS == kSortRegs ? 8 : 4) void k_tile_sort_long(
    uint32_t *__restrict__ long_q, int64_t PT, int c_lo, int c_hi, int pop, int chunk,
    const uint2 *__restrict__ ekv, uint32_t *__restrict__ klo, uint32_t *__restrict__ val,
    uint2 *__restrict__ tkv) {
  extern __shared__ uint64_t sm64[];
  uint64_t *red = sm64;
  uint32_t *hist = (uint32_t *)(sm64 + 4 * kSortWaves);
  uint32_t *start = hist + kSortBins;
  uint2 *skv = (uint2 *)(start + kSortBins);
  __shared__ uint2 s_job;
  constexpr uint32_t kDone = 0xffffffffu;   // entries of the job past the queue's end
  const uint2 *lists = (const uint2 *)(long_q + kLongQueueHeader);
  uint32_t *ctr = long_q + kLongClasses + pop;
  uint32_t cnt[kLongClasses];
  uint32_t next = 0;
  uint2 job1 = make_uint2(0u, kDone);
  // queue position -> (start, entries), or kDone past the classes' end
  auto fetch = [&](uint32_t i) -> uint2 {
    int64_t slot = -1;
#pragma unroll
    for (int k = 0; k < kLongClasses; ++k)
      if (slot < 0 && k >= c_lo && k < c_hi) {
        if (i < cnt[k]) slot = (int64_t)k * PT + i;
        else i -= cnt[k];
      }
    return slot < 0 ? make_uint2(0u, kDone) : lists[slot];
  };
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kLongClasses; ++k) cnt[k] = long_q[k];
    const uint32_t p0 = atomicAdd(ctr, 1u);
    const uint32_t p1 = atomicAdd(ctr, 1u);
    s_job = fetch(p0);
    job1 = fetch(p1);
    next = atomicAdd(ctr, 1u);
  }
  for (;;) {
    __syncthreads();
    const uint2 job = s_job;
    if (job.y == kDone) return;   // the same for every thread of the workgroup
    sort_bucket<REGS>(ekv, job.x, (int)job.y, chunk, klo, val, tkv, hist, start, red, skv);
    __syncthreads();
    if (threadIdx.x == 0) {
      s_job = job1;
      job1 = fetch(next);
      next = atomicAdd(ctr, 1u);
    }
  }
}

static int g_sort_chunk = 0, g_long_chunk = 0, g_xl_chunk = 0, g_n_cu = 0;
static size_t g_sort_lds = 0, g_long_lds = 0, g_xl_lds = 0;
constexpr int kXlRegs = 16;

size_t max_lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return 65536;
  return (size_t)v;
}

// Largest LDS chunk that lets `per_cu` 1024-thread workgroups share a CU
// (static_bytes: the kernel's own LDS besides the dynamic part), at most
// regs * 1024 entries.
static int sort_chunk_for(size_t static_bytes, int per_cu, int regs, size_t *dyn) {
  const size_t fixed = (size_t)4 * kSortWaves * 8 + (size_t)2 * kSortBins * 4;
  size_t lds = max_lds_per_block();
  if (lds > (size_t)160 * 1024 / per_cu) lds = (size_t)160 * 1024 / per_cu;
  int chunk = (int)((lds - fixed - static_bytes) / 8);
  chunk = (chunk / 32) * 32;
  if (chunk > regs * kTileSortThreads) chunk = regs * kTileSortThreads;
  if (chunk < kTileSortThreads) chunk = kTileSortThreads;
  *dyn = fixed + (size_t)8 * chunk;
  return chunk;
}

static void set_lds(const void *f, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static void choose_sort_chunk() {
  if (g_sort_chunk) return;
  const size_t item_bytes = 16;   // s_item, rounded up
  g_sort_chunk = sort_chunk_for(0, 2, kSortRegs, &g_sort_lds);
  set_lds((const void *)k_tile_sort, g_sort_lds);
  g_long_chunk = sort_chunk_for(item_bytes, 2, kSortRegs, &g_long_lds);
  set_lds((const void *)k_tile_sort_long<kSortRegs>, g_long_lds);
  g_xl_chunk = sort_chunk_for(item_bytes, 1, kXlRegs, &g_xl_lds);
  set_lds((const void *)k_tile_sort_long<kXlRegs>, g_xl_lds);
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      n > 0)
    g_n_cu = n;
  else
    g_n_cu = 256;
}

// Classes of the long-bucket queue: above the 8-entry kernel's chunk, five
// classes bounded by 2, 1.5 and 1 times the 16-entry kernel's chunk and the
// midpoint of the two chunks; from kMidSortMax to the 8-entry chunk, two
// classes split at their midpoint.  Within a class the buckets' costs differ
// by at most a factor of about 1.5, so taking the classes in order gives each
// workgroup a nearly equal share.
LongClasses long_classes() {
  choose_sort_chunk();
  LongClasses lc{};
  int n = 0;
  lc.thr[n++] = INT_MAX;
  const int xl = g_xl_chunk, lg = g_long_chunk;
  for (const int t : {2 * xl, xl + xl / 2, xl, (xl + lg) / 2})
    if (t > lg && t < lc.thr[n - 1]) lc.thr[n++] = t;
  lc.thr[n++] = lg;
  lc.split = n - 1;
  const int mid = (lg + kMidSortMax) / 2;
  if (mid > kMidSortMax && mid < lg) lc.thr[n++] = mid;
  lc.thr[n++] = kMidSortMax;
  lc.n = n - 1;
  lc.lo = kMidSortMax;
  return lc;
}

hipError_t launch_bin_sort(const gsrf_problem *p, const Layout &lay, char *ws, hipStream_t s) {
  const int64_t PT = (int64_t)p->n_pairs * lay.T;
  if (lay.n_records == 0 || PT == 0) return hipSuccess;
  const int64_t *counters = (const int64_t *)(ws + lay.counters);
  const uint32_t *tstart = (const uint32_t *)(ws + lay.tile_start);
  const uint32_t *tend = (const uint32_t *)(ws + lay.tile_end);
  {
    const int RB = lay.rec_block;
    dim3 grid((unsigned)((lay.max_scene + RB - 1) / RB), (unsigned)p->n_pairs);
    if (RB == 1024 && lay.T <= kEmitStagedTiles)
      hipLaunchKernelGGL(k_emit_staged<1024>, grid, dim3(1024), (size_t)lay.T * 12, s, p->pairs, p->scene_offsets_dev,
                         (const int64_t *)(ws + lay.rec_base), (const uint32_t *)(ws + lay.rec_key),
                         (const ushort4 *)(ws + lay.rec_rect), lay.T, lay.nta, PT, counters,
                         (uint32_t *)(ws + lay.tile_cur), (uint2 *)(ws + lay.ekv));
    else if (RB == 1024)
      hipLaunchKernelGGL(k_emit<1024>, grid, dim3(1024), (size_t)lay.T * 8, s, p->pairs, p->scene_offsets_dev,
                         (const int64_t *)(ws + lay.rec_base), (const uint32_t *)(ws + lay.rec_key),
                         (const ushort4 *)(ws + lay.rec_rect), lay.T, lay.nta, PT, counters,
                         (uint32_t *)(ws + lay.tile_cur), (uint2 *)(ws + lay.ekv));
    else
      hipLaunchKernelGGL(k_emit<256>, grid, dim3(256), (size_t)lay.T * 8, s, p->pairs, p->scene_offsets_dev,
                         (const int64_t *)(ws + lay.rec_base), (const uint32_t *)(ws + lay.rec_key),
                         (const ushort4 *)(ws + lay.rec_rect), lay.T, lay.nta, PT, counters,
                         (uint32_t *)(ws + lay.tile_cur), (uint2 *)(ws + lay.ekv));
  }
  choose_sort_chunk();
  const uint2 *ekv = (const uint2 *)(ws + lay.ekv);
  uint32_t *klo = (uint32_t *)(ws + lay.klo), *val = (uint32_t *)(ws + lay.val);
  uint2 *tkv = (uint2 *)(ws + lay.tkv);
  if (PT <= kSortFewTiles) {
    hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)PT), dim3(kTileSortThreads), g_sort_lds, s, tstart, tend,
                       g_sort_chunk, ekv, klo, val, tkv);
  } else {
    hipLaunchKernelGGL(k_tile_sort_small, dim3((unsigned)PT), dim3(kSmallSortThreads), 0, s, tstart, tend, ekv, klo,
                       val);
    hipLaunchKernelGGL(k_tile_sort_mid, dim3((unsigned)PT), dim3(kMidSortThreads), 0, s, tstart, tend, ekv, klo, val);
    const LongClasses lc = long_classes();
    uint32_t *long_q = (uint32_t *)(ws + lay.long_q);   // filled by k_scan_apply
    const int64_t grid = 2 * (int64_t)g_n_cu < PT ? 2 * (int64_t)g_n_cu : PT;   // two workgroups per CU
    hipLaunchKernelGGL(k_tile_sort_long<kSortRegs>, dim3((unsigned)grid), dim3(kTileSortThreads), g_long_lds, s,
                       long_q, PT, lc.split, lc.n, 1, g_long_chunk, ekv, klo, val, tkv);
    const int64_t xgrid = (int64_t)g_n_cu < PT ? (int64_t)g_n_cu : PT;         // one workgroup per CU
    hipLaunchKernelGGL(k_tile_sort_long<kXlRegs>, dim3((unsigned)xgrid), dim3(kTileSortThreads), g_xl_lds, s,
                       long_q, PT, 0, lc.split, 0, g_xl_chunk, ekv, klo, val, tkv);
  }
  return hipGetLastError();
}

}  // namespace gsrf
