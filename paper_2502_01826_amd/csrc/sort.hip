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
  uint32_t *cur = tcur + (size_t)(blockIdx.x % kSub) * PT + (size_t)k * T;
  for (int t = threadIdx.x; t < T; t += blockDim.x) {
    const uint32_t c = cnt[t];
    if (c) base[t] = atomicAdd(cur + t, c);
    cnt[t] = 0;
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
// tile).  One MSD counting pass splits the bucket into 2^b sub-buckets of
// c - c_min (about four entries each, b <= 11): histogram, exclusive scan and
// scatter.  Each entry's final place is then its sub-bucket's start plus its
// rank among the sub-bucket's entries, found by comparing with all of them;
// sub-buckets are small, so this costs a few comparisons per entry and no
// further passes.  The scatter buffer is LDS for buckets of up to `chunk`
// entries; longer buckets scatter to global scratch and are ranked in LDS
// windows of whole sub-buckets.  The result does not depend on the (atomic)
// scatter order, so it is deterministic.
// ---------------------------------------------------------------------------
constexpr int kSortWaves = kTileSortThreads / 64;
constexpr int kSortRegs = 8;              // entries per thread held in registers (LDS path)
constexpr int kSortBitsMax = 11;
constexpr int kSortBins = 1 << kSortBitsMax;

__device__ __forceinline__ uint64_t composite(uint32_t k, uint32_t v) { return ((uint64_t)k << 32) | v; }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int d) {
  const uint32_t lo = __shfl_xor((uint32_t)x, d, 64), hi = __shfl_xor((uint32_t)(x >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Exclusive scan of cnt[0, nbins) into start[0, nbins) (nbins <= 2 * threads).
__device__ void bins_scan(const uint32_t *cnt, uint32_t *start, int nbins, uint32_t *wsum) {
  constexpr int NT = kTileSortThreads;
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
    start[i] = run;
    run += cnt[i];
  }
}

// Sort the n entries ekv = (key, value) by composite into (ok, ov) through the scatter
// buffer (bk, bv); SH: the buffer is in LDS.
template <bool SH>
__device__ void msd_rank_sort(const uint2 *__restrict__ ekv, int n, uint32_t *bk,
                              uint32_t *bv, uint32_t *__restrict__ ok, uint32_t *__restrict__ ov, uint32_t *hist,
                              uint32_t *start, uint64_t *red, uint32_t *sk, uint32_t *sv, int chunk) {
  constexpr int NT = kTileSortThreads;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // LDS path (n <= kSortRegs * NT): each thread keeps its entries in registers
  // across the passes, so the bucket is read from global memory once
  uint32_t rk[SH ? kSortRegs : 1], rv[SH ? kSortRegs : 1];
  if constexpr (SH) {
#pragma unroll
    for (int e = 0; e < kSortRegs; ++e) {
      const int i = tid + e * NT;
      const uint2 x = i < n ? ekv[i] : make_uint2(0u, 0u);
      rk[e] = x.x;
      rv[e] = x.y;
    }
  }
  uint64_t cmin = ~0ull, cmax = 0;
  if constexpr (SH) {
#pragma unroll
    for (int e = 0; e < kSortRegs; ++e)
      if (tid + e * NT < n) {
        const uint64_t c = composite(rk[e], rv[e]);
        cmin = c < cmin ? c : cmin;
        cmax = c > cmax ? c : cmax;
      }
  } else {
    for (int i = tid; i < n; i += NT) {
      const uint64_t c = composite(ekv[i].x, ekv[i].y);
      cmin = c < cmin ? c : cmin;
      cmax = c > cmax ? c : cmax;
    }
  }
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
  int bits = 1;
  while (bits < kSortBitsMax && (4 << bits) < n) ++bits;
  const uint64_t span = cmax - cmin;
  const int nbits = span ? 64 - __clzll(span) : 0;
  const int shift = nbits > bits ? nbits - bits : 0;
  const int nbins = 1 << bits;
  for (int i = tid; i < nbins; i += NT) hist[i] = 0;
  __syncthreads();
  if constexpr (SH) {
#pragma unroll
    for (int e = 0; e < kSortRegs; ++e)
      if (tid + e * NT < n) atomicAdd(&hist[(uint32_t)((composite(rk[e], rv[e]) - cmin) >> shift)], 1u);
  } else {
    for (int i = tid; i < n; i += NT) atomicAdd(&hist[(uint32_t)((composite(ekv[i].x, ekv[i].y) - cmin) >> shift)], 1u);
  }
  __syncthreads();
  bins_scan(hist, start, nbins, (uint32_t *)(red + 2 * kSortWaves + 2));
  __syncthreads();
  for (int i = tid; i < nbins; i += NT) hist[i] = start[i];     // scatter cursors
  __syncthreads();
  if constexpr (SH) {
#pragma unroll
    for (int e = 0; e < kSortRegs; ++e)
      if (tid + e * NT < n) {
        const uint32_t p = atomicAdd(&hist[(uint32_t)((composite(rk[e], rv[e]) - cmin) >> shift)], 1u);
        bk[p] = rk[e];
        bv[p] = rv[e];
      }
  } else {
    for (int i = tid; i < n; i += NT) {
      const uint32_t k = ekv[i].x, v = ekv[i].y;
      const uint32_t p = atomicAdd(&hist[(uint32_t)((composite(k, v) - cmin) >> shift)], 1u);
      bk[p] = k;
      bv[p] = v;
    }
  }
  if (!SH) __threadfence_block();
  __syncthreads();
  // hist[d] is now the end of sub-bucket d
  if constexpr (SH) {
    for (int p = tid; p < n; p += NT) {
      const uint32_t k = bk[p], v = bv[p];
      const uint64_t c = composite(k, v);
      const uint32_t d = (uint32_t)((c - cmin) >> shift);
      const int a = (int)start[d], e = (int)hist[d];
      int rank = 0;
#pragma unroll 2
      for (int j = a; j < e; ++j) rank += composite(bk[j], bv[j]) < c ? 1 : 0;
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
        for (int i = tid; i < w1 - w0; i += NT) {
          sk[i] = bk[w0 + i];
          sv[i] = bv[w0 + i];
        }
        __syncthreads();
        for (int p = tid; p < w1 - w0; p += NT) {
          const uint32_t k = sk[p], v = sv[p];
          const uint64_t c = composite(k, v);
          const uint32_t d = (uint32_t)((c - cmin) >> shift);
          const int a = (int)start[d] - w0, e = (int)hist[d] - w0;
          int rank = 0;
#pragma unroll 2
          for (int j = a; j < e; ++j) rank += composite(sk[j], sv[j]) < c ? 1 : 0;
          ok[w0 + a + rank] = k;
          ov[w0 + a + rank] = v;
        }
        __syncthreads();
      } else {
        // the sub-bucket starting at w0 exceeds the window
        const uint64_t c0 = composite(bk[w0], bv[w0]);
        const uint32_t d0 = (uint32_t)((c0 - cmin) >> shift);
        w1 = (int)hist[d0];
        for (int p = w0 + tid; p < w1; p += NT) {
          const uint32_t k = bk[p], v = bv[p];
          const uint64_t c = composite(k, v);
          int rank = 0;
          for (int j = w0; j < w1; ++j) rank += composite(bk[j], bv[j]) < c ? 1 : 0;
          ok[w0 + rank] = k;
          ov[w0 + rank] = v;
        }
      }
      w0 = w1;
    }
  }
}

// a4: sort every tile's bucket; writes the sorted depth keys and Gaussian ids.
__global__ __launch_bounds__(kTileSortThreads, 8) void k_tile_sort(const uint32_t *__restrict__ tstart,
                                                                const uint32_t *__restrict__ tend, int chunk,
                                                                const uint2 *__restrict__ ekv,
                                                                uint32_t *__restrict__ klo, uint32_t *__restrict__ val,
                                                                uint32_t *__restrict__ tkey, uint32_t *__restrict__ tval) {
  extern __shared__ uint64_t sm64[];
  uint64_t *red = sm64;                                     // wave min/max, totals, wave sums
  uint32_t *hist = (uint32_t *)(sm64 + 4 * kSortWaves);     // [kSortBins]
  uint32_t *start = hist + kSortBins;                       // [kSortBins]
  uint32_t *sk = start + kSortBins;                         // [chunk]
  uint32_t *sv = sk + chunk;                                // [chunk]
  const int gt = blockIdx.x;
  const uint32_t s0 = tstart[gt];
  const int n = (int)(tend[gt] - s0);
  if (n <= 0) return;
  if (n <= chunk)
    msd_rank_sort<true>(ekv + s0, n, sk, sv, klo + s0, val + s0, hist, start, red, sk, sv, chunk);
  else
    msd_rank_sort<false>(ekv + s0, n, tkey + s0, tval + s0, klo + s0, val + s0, hist, start, red, sk, sv, chunk);
}

static int g_sort_chunk = 0;
static size_t g_sort_lds = 0;

size_t max_lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return 65536;
  return (size_t)v;
}

// Largest LDS chunk that still lets two 1024-thread workgroups share a CU.
static void choose_sort_chunk() {
  if (g_sort_chunk) return;
  const size_t fixed = (size_t)4 * kSortWaves * 8 + (size_t)2 * kSortBins * 4;
  size_t lds = max_lds_per_block();
  if (lds > 160 * 1024) lds = 160 * 1024;
  int chunk = (int)((lds / 2 - fixed) / 8);
  chunk = (chunk / 32) * 32;
  if (chunk > kSortRegs * kTileSortThreads) chunk = kSortRegs * kTileSortThreads;
  if (chunk < kTileSortThreads) chunk = kTileSortThreads;
  g_sort_lds = fixed + (size_t)8 * chunk;
  if (g_sort_lds > 65536)
    (void)hipFuncSetAttribute((const void *)k_tile_sort, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g_sort_lds);
  g_sort_chunk = chunk;
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
    if (RB == 1024)
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
  hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)PT), dim3(kTileSortThreads), g_sort_lds, s, tstart, tend,
                     g_sort_chunk, (const uint2 *)(ws + lay.ekv),
                     (uint32_t *)(ws + lay.klo), (uint32_t *)(ws + lay.val), (uint32_t *)(ws + lay.tkey),
                     (uint32_t *)(ws + lay.tval));
  return hipGetLastError();
}

}  // namespace gsrf
