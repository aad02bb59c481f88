// Steps a3-a4: splat emission into per-tile buckets and the per-tile depth
// sort (App. E: every splat carries the tile index and the distance key; the
// paper sorts them all at once by a 64-bit key, Alg. 1 sphericalSplatting and
// computeGridRange).  Here the tile part of the key is applied by bucketing
// (the tile ranges come from the counts made during projection) and the
// distance part by sorting each bucket in its own workgroup, which gives the
// same order -- (distance key, Gaussian index) within each tile -- with one
// pass over the splats instead of one per key byte.
//
// A bucket of up to `chunk` entries is sorted in LDS by a four-pass stable LSD
// radix sort on the 32-bit distance key (wave64 ballots rank equal digits),
// after which runs of equal keys are ordered by Gaussian index.  A longer
// bucket is sorted chunk by chunk and the sorted runs are merged pairwise in
// global memory (merge-path partitioning across the workgroup).  No
// workgroup ever waits on another, so every wave finishes.
#include "gsrf_internal.h"

namespace gsrf {

// a3: one splat per covered tile.  The workgroup (256 records of one pair)
// counts its splats per tile in LDS, reserves each tile's share with one
// global atomic on its sub-bucket's cursor, then writes (key, Gaussian) at its
// reserved slots.
__global__ __launch_bounds__(256) void k_emit(const gsrf_pair *__restrict__ pairs,
                                              const int64_t *__restrict__ scene_off,
                                              const int64_t *__restrict__ rec_base,
                                              const uint32_t *__restrict__ rec_key,
                                              const ushort4 *__restrict__ rec_rect, int32_t T, int32_t nta, int64_t PT,
                                              const int64_t *__restrict__ counters, uint32_t *__restrict__ tcur,
                                              uint32_t *__restrict__ ekey, uint32_t *__restrict__ eval) {
  if (counters[1] != 0) return;  // over capacity: every range is empty, nothing is emitted
  extern __shared__ uint32_t sm[];
  uint32_t *cnt = sm;        // [T]
  uint32_t *base = sm + T;   // [T]
  __shared__ RectScan rs;
  __shared__ uint32_t keys[256];
  const int k = blockIdx.y;
  for (int t = threadIdx.x; t < T; t += blockDim.x) cnt[t] = 0;
  const int s = pairs[k].scene;
  const int64_t g0 = scene_off[s];
  const int64_t n = scene_off[s + 1] - g0;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  ushort4 rc = make_ushort4(0, 0, 0, 0);
  uint32_t key = 0;
  if (j < n) {
    const int64_t r = rec_base[k] + j;
    rc = rec_rect[r];
    key = rec_key[r];
  }
  keys[threadIdx.x] = key;
  rect_scan(rs, rc);
  const uint32_t total = rs.off[256];
  for (uint32_t sp = threadIdx.x; sp < total; sp += 256) {
    int t;
    rect_splat(rs, sp, nta, &t);
    atomicAdd(&cnt[t], 1u);
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
  const uint32_t gbase = (uint32_t)(g0 + (int64_t)blockIdx.x * 256);
  for (uint32_t sp = threadIdx.x; sp < total; sp += 256) {
    int t;
    const int slot = rect_splat(rs, sp, nta, &t);
    const uint32_t pos = base[t] + atomicAdd(&cnt[t], 1u);
    ekey[pos] = keys[slot];
    eval[pos] = gbase + (uint32_t)slot;
  }
}

// ---------------------------------------------------------------------------
// Workgroup-level pieces of the tile sort (kTileSortThreads threads).
// ---------------------------------------------------------------------------
constexpr int kSortWaves = kTileSortThreads / 64;

struct SortLds {
  uint32_t *ak, *av, *bk, *bv;    // ping-pong buffers [chunk]
  uint32_t *hist, *run;           // [256] each
  uint32_t *wcnt, *wpre;          // [kSortWaves][256] each
};

__device__ __forceinline__ SortLds sort_lds_of(uint32_t *sm, int chunk) {
  SortLds L;
  L.ak = sm;
  L.av = sm + chunk;
  L.bk = sm + 2 * chunk;
  L.bv = sm + 3 * chunk;
  L.hist = sm + 4 * chunk;
  L.run = L.hist + 256;
  L.wcnt = L.run + 256;
  L.wpre = L.wcnt + kSortWaves * 256;
  return L;
}

// One stable counting pass on the byte at `shift` of the keys: src -> dst.
__device__ void lsd_pass(const uint32_t *sk, const uint32_t *sv, uint32_t *dk, uint32_t *dv, int n, int shift,
                         const SortLds &L) {
  constexpr int NT = kTileSortThreads;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid < 256) L.hist[tid] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += NT) atomicAdd(&L.hist[(sk[i] >> shift) & 255u], 1u);
  __syncthreads();
  // exclusive scan of the 256 digit counts by the first wave (4 bins per lane)
  if (wave == 0) {
    const uint32_t a0 = L.hist[4 * lane], a1 = L.hist[4 * lane + 1], a2 = L.hist[4 * lane + 2],
                   a3 = L.hist[4 * lane + 3];
    const uint32_t sum = a0 + a1 + a2 + a3;
    uint32_t inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d, 64);
      if (lane >= d) inc += y;
    }
    const uint32_t ex = inc - sum;
    L.run[4 * lane] = ex;
    L.run[4 * lane + 1] = ex + a0;
    L.run[4 * lane + 2] = ex + a0 + a1;
    L.run[4 * lane + 3] = ex + a0 + a1 + a2;
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int b0 = 0; b0 < n; b0 += NT) {
    const int i = b0 + tid;
    const bool valid = i < n;
    uint32_t key = 0, val = 0, d = 0;
    if (valid) {
      key = sk[i];
      val = sv[i];
      d = (key >> shift) & 255u;
    }
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) L.wcnt[wave * 256 + d] = __popcll(peers);
    __syncthreads();
    if (tid < 256) {
      uint32_t r = L.run[tid];
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) {
        L.wpre[w * 256 + tid] = r;
        r += L.wcnt[w * 256 + tid];
        L.wcnt[w * 256 + tid] = 0;
      }
      L.run[tid] = r;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = L.wpre[wave * 256 + d] + rank;
      dk[pos] = key;
      dv[pos] = val;
    }
  }
  __syncthreads();
}

// Sort n <= chunk entries held in (L.ak, L.av) by (key, value); result in place.
__device__ void lds_sort(int n, const SortLds &L) {
  lsd_pass(L.ak, L.av, L.bk, L.bv, n, 0, L);
  lsd_pass(L.bk, L.bv, L.ak, L.av, n, 8, L);
  lsd_pass(L.ak, L.av, L.bk, L.bv, n, 16, L);
  lsd_pass(L.bk, L.bv, L.ak, L.av, n, 24, L);
  // equal keys: order by Gaussian index (runs are short; the run's first
  // element's thread insertion-sorts it)
  for (int i = threadIdx.x; i < n; i += kTileSortThreads) {
    const uint32_t k0 = L.ak[i];
    if ((i > 0 && L.ak[i - 1] == k0) || i + 1 >= n || L.ak[i + 1] != k0) continue;
    int e = i + 1;
    while (e < n && L.ak[e] == k0) ++e;
    for (int a = i + 1; a < e; ++a) {
      const uint32_t v = L.av[a];
      int b = a - 1;
      while (b >= i && L.av[b] > v) {
        L.av[b + 1] = L.av[b];
        --b;
      }
      L.av[b + 1] = v;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ bool kv_less(uint32_t ka, uint32_t va, uint32_t kb, uint32_t vb) {
  return ka < kb || (ka == kb && va < vb);
}

// Merge sorted runs A[0, la) and B[0, lb) (given as key/value arrays) into
// out[0, la + lb); the workgroup splits the output by merge-path diagonals.
__device__ void merge_runs(const uint32_t *Ak, const uint32_t *Av, int la, const uint32_t *Bk, const uint32_t *Bv,
                           int lb, uint32_t *ok, uint32_t *ov) {
  const int total = la + lb;
  const int per = (total + kTileSortThreads - 1) / kTileSortThreads;
  const int d0 = min(total, (int)threadIdx.x * per);
  const int d1 = min(total, d0 + per);
  if (d0 >= d1) return;
  // number of A elements among the d0 smallest
  int lo = max(0, d0 - lb), hi = min(d0, la);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;     // take mid from A, d0 - mid from B
    const int jb = d0 - mid - 1;
    if (jb < 0 || kv_less(Bk[jb], Bv[jb], Ak[mid], Av[mid]))
      hi = mid;
    else
      lo = mid + 1;
  }
  int i = lo, j = d0 - lo;
  for (int d = d0; d < d1; ++d) {
    const bool takeA = (j >= lb) || (i < la && kv_less(Ak[i], Av[i], Bk[j], Bv[j]));
    if (takeA) {
      ok[d] = Ak[i];
      ov[d] = Av[i];
      ++i;
    } else {
      ok[d] = Bk[j];
      ov[d] = Bv[j];
      ++j;
    }
  }
}

// a4: sort every tile's bucket; writes the sorted depth keys and Gaussian ids.
__global__ __launch_bounds__(kTileSortThreads) void k_tile_sort(const uint32_t *__restrict__ tstart,
                                                                const uint32_t *__restrict__ tend, int chunk,
                                                                const uint32_t *__restrict__ ekey,
                                                                const uint32_t *__restrict__ eval,
                                                                uint32_t *__restrict__ klo, uint32_t *__restrict__ val,
                                                                uint32_t *__restrict__ tkey, uint32_t *__restrict__ tval) {
  extern __shared__ uint32_t sm[];
  const SortLds L = sort_lds_of(sm, chunk);
  const int gt = blockIdx.x;
  const uint32_t s0 = tstart[gt];
  const int n = (int)(tend[gt] - s0);
  if (n <= 0) return;
  for (int i = threadIdx.x; i < kSortWaves * 256; i += kTileSortThreads) L.wcnt[i] = 0;
  const int nruns = (n + chunk - 1) / chunk;
  int passes = 0;
  while ((1 << passes) < nruns) ++passes;
  // runs go to the buffer from which an even number of merge passes ends in (klo, val)
  uint32_t *rk = (passes & 1) ? tkey : klo, *rv = (passes & 1) ? tval : val;
  uint32_t *ok_ = (passes & 1) ? klo : tkey, *ov_ = (passes & 1) ? val : tval;
  for (int c = 0; c < nruns; ++c) {
    const int b = c * chunk;
    const int m = min(chunk, n - b);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += kTileSortThreads) {
      L.ak[i] = ekey[s0 + b + i];
      L.av[i] = eval[s0 + b + i];
    }
    __syncthreads();
    lds_sort(m, L);
    for (int i = threadIdx.x; i < m; i += kTileSortThreads) {
      rk[s0 + b + i] = L.ak[i];
      rv[s0 + b + i] = L.av[i];
    }
  }
  for (int w = chunk; w < n; w *= 2) {
    __syncthreads();   // the previous pass's (or the runs') writes are visible to the workgroup
    __threadfence_block();
    for (int a0 = 0; a0 < n; a0 += 2 * w) {
      const int la = min(w, n - a0);
      const int lb = max(0, min(w, n - a0 - la));
      merge_runs(rk + s0 + a0, rv + s0 + a0, la, rk + s0 + a0 + la, rv + s0 + a0 + la, lb, ok_ + s0 + a0,
                 ov_ + s0 + a0);
    }
    uint32_t *t1 = rk, *t2 = rv;
    rk = ok_; rv = ov_;
    ok_ = t1; ov_ = t2;
  }
}

static int g_sort_chunk = 0;
static size_t g_sort_lds = 0;

size_t max_lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return 65536;
  return (size_t)v;
}

static void choose_sort_chunk() {
  if (g_sort_chunk) return;
  const size_t fixed = (2 * 256 + 2 * kSortWaves * 256) * 4;
  size_t lds = max_lds_per_block();
  if (lds > 160 * 1024) lds = 160 * 1024;
  int chunk = (int)((lds - fixed) / 16);
  chunk = (chunk / 512) * 512;
  if (chunk > 8192) chunk = 8192;
  if (chunk < kTileSortThreads) chunk = kTileSortThreads;
  g_sort_lds = fixed + (size_t)16 * chunk;
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
    dim3 grid((unsigned)((lay.max_scene + 255) / 256), (unsigned)p->n_pairs);
    hipLaunchKernelGGL(k_emit, grid, dim3(256), (size_t)lay.T * 8, s, p->pairs, p->scene_offsets_dev,
                       (const int64_t *)(ws + lay.rec_base), (const uint32_t *)(ws + lay.rec_key),
                       (const ushort4 *)(ws + lay.rec_rect), lay.T, lay.nta, PT, counters,
                       (uint32_t *)(ws + lay.tile_cur), (uint32_t *)(ws + lay.ekey), (uint32_t *)(ws + lay.eval));
  }
  choose_sort_chunk();
  hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)PT), dim3(kTileSortThreads), g_sort_lds, s, tstart, tend,
                     g_sort_chunk, (const uint32_t *)(ws + lay.ekey), (const uint32_t *)(ws + lay.eval),
                     (uint32_t *)(ws + lay.klo), (uint32_t *)(ws + lay.val), (uint32_t *)(ws + lay.tkey),
                     (uint32_t *)(ws + lay.tval));
  return hipGetLastError();
}

}  // namespace gsrf
