// Steps a3-a4: splat emission, stable LSD radix sort on 64-bit
// (tile | depth) keys, and per-tile ranges (App. E: one sort of all splats
// with the tile index in the high 32 bits and the distance key in the low 32;
// Alg. 1 sphericalSplatting and computeGridRange).
//
// The sort is a classic three-kernel LSD pass per 8-bit digit: per-block
// digit histograms, an exclusive scan over (digit, block), and a stable
// scatter whose in-block ranks come from wave64 ballots.  There is no
// cross-block spin-waiting, so every wave always finishes.
#include "gsrf_internal.h"

namespace gsrf {

// a3: one splat per tile of each record's rectangle, in (tile row, tile column)
// order; value = global Gaussian index.
__global__ void k_emit(const gsrf_pair *__restrict__ pairs, const int64_t *__restrict__ scene_off,
                       const int64_t *__restrict__ rec_base, const uint32_t *__restrict__ rec_key,
                       const ushort4 *__restrict__ rec_rect, const uint32_t *__restrict__ rec_cnt,
                       const int64_t *__restrict__ rec_off, int32_t T, int32_t nta, int64_t cap,
                       const int64_t *__restrict__ counters,
                       uint32_t *__restrict__ khi, uint32_t *__restrict__ klo, uint32_t *__restrict__ val) {
  if (counters[1] != 0) return;  // over capacity: nothing is emitted
  const int k = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = pairs[k].scene;
  const int64_t g0 = scene_off[s];
  const int64_t n = scene_off[s + 1] - g0;
  if (j >= n) return;
  const int64_t r = rec_base[k] + j;
  const uint32_t cnt = rec_cnt[r];
  if (cnt == 0) return;
  const int64_t off = rec_off[r];
  if (off + (int64_t)cnt > cap) return;  // over capacity: reported through the counters
  const ushort4 rc = rec_rect[r];
  const uint32_t key = rec_key[r];
  const uint32_t gid = (uint32_t)(g0 + j);
  const uint32_t tbase = (uint32_t)k * (uint32_t)T;
  int64_t o = off;
  for (int tv = rc.z; tv < rc.z + rc.w; ++tv) {
    int tu = rc.x;
    for (int c = 0; c < rc.y; ++c) {
      khi[o] = tbase + (uint32_t)(tv * nta + tu);
      klo[o] = key;
      val[o] = gid;
      ++o;
      if (++tu == nta) tu = 0;
    }
  }
}

// Number of valid splats; zero when the count overflowed the capacity, so an
// over-full workspace is never read past what emission wrote.
__device__ __forceinline__ int64_t splat_n(const int64_t *counters, int64_t cap) {
  return counters[1] != 0 ? 0 : min(counters[0], cap);
}

__device__ __forceinline__ uint32_t digit_of(uint32_t hi, uint32_t lo, int pass) {
  return pass < 4 ? (lo >> (8 * pass)) & 255u : (hi >> (8 * (pass - 4))) & 255u;
}

__global__ void k_radix_hist(const uint32_t *__restrict__ khi, const uint32_t *__restrict__ klo,
                             const int64_t *__restrict__ counters, int64_t cap, int pass, int nblk,
                             uint32_t *__restrict__ hist) {
  __shared__ uint32_t cnt[256];
  const int tid = threadIdx.x;
  cnt[tid] = 0;
  __syncthreads();
  const int64_t n = splat_n(counters, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t i = base + it * kSortThreads + tid;
    if (i < n) atomicAdd(&cnt[digit_of(khi[i], klo[i], pass)], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * nblk + blockIdx.x] = cnt[tid];
}

// Stable scatter.  Items are visited in index order (iteration-major, then
// wave, then lane); each wave finds the lanes sharing its digit with eight
// ballots, and per-digit running offsets carry order across waves/iterations.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *__restrict__ khi_in, const uint32_t *__restrict__ klo_in, const uint32_t *__restrict__ val_in,
    uint32_t *__restrict__ khi_out, uint32_t *__restrict__ klo_out, uint32_t *__restrict__ val_out,
    const int64_t *__restrict__ counters, int64_t cap, int pass, int nblk, const uint32_t *__restrict__ hist_scan) {
  __shared__ uint32_t goff[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  __shared__ uint32_t wpre[4][256];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  goff[tid] = hist_scan[(int64_t)tid * nblk + blockIdx.x];
  run[tid] = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const int64_t n = splat_n(counters, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t i = base + it * kSortThreads + tid;
    const bool valid = i < n;
    uint32_t hi = 0, lo = 0, vv = 0, d = 0;
    if (valid) {
      hi = khi_in[i];
      lo = klo_in[i];
      vv = val_in[i];
      d = digit_of(hi, lo, pass);
    }
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    {
      uint32_t r = run[tid];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        wpre[w][tid] = r;
        r += wcnt[w][tid];
        wcnt[w][tid] = 0;
      }
      run[tid] = r;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = goff[d] + wpre[wave][d] + rank;
      khi_out[pos] = hi;
      klo_out[pos] = lo;
      val_out[pos] = vv;
    }
  }
}

// computeGridRange: [start, end) of each global tile in the sorted array.
__global__ void k_ranges(const uint32_t *__restrict__ khi, const int64_t *__restrict__ counters, int64_t cap,
                         uint32_t *__restrict__ tstart, uint32_t *__restrict__ tend) {
  const int64_t n = splat_n(counters, cap);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const uint32_t t = khi[i];
    if (i == 0 || khi[i - 1] != t) tstart[t] = (uint32_t)i;
    if (i == n - 1 || khi[i + 1] != t) tend[t] = (uint32_t)(i + 1);
  }
}

hipError_t launch_bin_sort(const gsrf_problem *p, const Layout &lay, char *ws, hipStream_t s) {
  const int64_t PT = (int64_t)p->n_pairs * lay.T;
  uint32_t *tstart = (uint32_t *)(ws + lay.tile_start);
  uint32_t *tend = (uint32_t *)(ws + lay.tile_end);
  hipError_t e = fill<uint32_t>(tstart, 0u, PT, s);
  if (e != hipSuccess) return e;
  e = fill<uint32_t>(tend, 0u, PT, s);
  if (e != hipSuccess) return e;
  if (lay.n_records == 0 || lay.cap == 0) return hipGetLastError();
  const int64_t *counters = (const int64_t *)(ws + lay.counters);
  uint32_t *khi[2] = {(uint32_t *)(ws + lay.khi[0]), (uint32_t *)(ws + lay.khi[1])};
  uint32_t *klo[2] = {(uint32_t *)(ws + lay.klo[0]), (uint32_t *)(ws + lay.klo[1])};
  uint32_t *val[2] = {(uint32_t *)(ws + lay.val[0]), (uint32_t *)(ws + lay.val[1])};
  {
    dim3 grid((unsigned)((lay.max_scene + 255) / 256), (unsigned)p->n_pairs);
    hipLaunchKernelGGL(k_emit, grid, dim3(256), 0, s, p->pairs, p->scene_offsets_dev,
                       (const int64_t *)(ws + lay.rec_base), (const uint32_t *)(ws + lay.rec_key),
                       (const ushort4 *)(ws + lay.rec_rect), (const uint32_t *)(ws + lay.rec_cnt),
                       (const int64_t *)(ws + lay.rec_off), lay.T, lay.nta, lay.cap, counters, khi[0], klo[0],
                       val[0]);
  }
  uint32_t *hist = (uint32_t *)(ws + lay.hist);
  uint32_t *hist_scan = (uint32_t *)(ws + lay.hist_scan);
  uint32_t *hist_tmp = (uint32_t *)(ws + lay.hist_tmp);
  const int nblk = lay.n_sort_blocks;
  int cur = 0;
  for (int pass = 0; pass < lay.sort_passes; ++pass) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, s, khi[cur], klo[cur], counters, lay.cap,
                       pass, nblk, hist);
    e = scan_u32_to_u32(hist, (int64_t)256 * nblk, hist_scan, hist_tmp, lay.n_hist_blocks, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0, s, khi[cur], klo[cur], val[cur],
                       khi[cur ^ 1], klo[cur ^ 1], val[cur ^ 1], counters, lay.cap, pass, nblk, hist_scan);
    cur ^= 1;
  }
  {
    int64_t blocks = (lay.cap + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, s, khi[cur], counters, lay.cap, tstart, tend);
  }
  return hipGetLastError();
}

}  // namespace gsrf
