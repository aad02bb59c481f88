// Paper-literal variants of the forward render (a5 + a6):
//   * per-Gaussian FLE and chord transmittance: the two-phase traversal with
//     its runtime switches on (render_two_phase.h, VAR kernels);
//   * per-ray midpoint order (App. A.3: the Gaussians a ray meets are taken
//     in increasing t_mid, not in the per-tile distance order): four steps,
//       count     phase-1 tests over each tile's whole list (no termination,
//                 which depends on the order), entry masks and hits per ray;
//       scan      exclusive scan of the hits per ray -> each ray's records;
//       collect   from the masks, one record per hit: key (t_mid in 2^-24 m
//                 steps << 24 | rank in list order) and the order-free terms (the
//                 transmittance factor rho and p psi e^{-j phi});
//       composite one wave per ray sorts its keys (bitonic, ascending
//                 compare-exchanges only, so the padding to a power of two
//                 never moves) and accumulates front to back with the same
//                 termination rule: a hit counts iff the product of the
//                 earlier factors is >= t_min.
//     S_hat and the RSSI are summed over the rays per pair in FP64, fixed order.
#include "render_two_phase.h"

namespace gsrf {

// ---- scan of the hits per ray (three launches, like the tile-count scan) ----
__global__ __launch_bounds__(256) void k_tmid_scan_reduce(const uint32_t *__restrict__ cnt, int64_t n,
                                                          uint64_t *__restrict__ blk) {
  __shared__ uint64_t sh[256];
  const int64_t i0 = (int64_t)blockIdx.x * kTmidScan;
  uint64_t local = 0;
  for (int i = threadIdx.x; i < kTmidScan; i += 256)
    if (i0 + i < n) {
      const uint32_t c = cnt[i0 + i];
      // a ray with more hits than the key's rank holds counts as over any capacity
      local += c > kTmidRankMask ? ((uint64_t)1 << 40) : c;
    }
  sh[threadIdx.x] = local;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) blk[blockIdx.x] = sh[0];
}

// exclusive scan of the block sums; counters[2] = total records,
// counters[3] = total if it exceeds the capacity, else 0
__global__ __launch_bounds__(1024) void k_tmid_scan_blocks(uint64_t *__restrict__ blk, int64_t nblk, int64_t cap,
                                                           int64_t *__restrict__ counters) {
  __shared__ uint64_t sh[1024];
  const int tid = threadIdx.x;
  uint64_t carry = 0;
  for (int64_t c0 = 0; c0 < nblk; c0 += 1024) {
    const int64_t i = c0 + tid;
    const uint64_t x = i < nblk ? blk[i] : 0;
    sh[tid] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const uint64_t y = tid >= off ? sh[tid - off] : 0;
      __syncthreads();
      sh[tid] += y;
      __syncthreads();
    }
    if (i < nblk) blk[i] = carry + sh[tid] - x;
    carry += sh[1023];
    __syncthreads();
  }
  if (tid == 0) {
    const uint64_t sat = (uint64_t)1 << 62;
    const int64_t tot = (int64_t)(carry > sat ? sat : carry);
    counters[2] = tot;
    counters[3] = carry > (uint64_t)cap ? tot : 0;
  }
}

__global__ __launch_bounds__(256) void k_tmid_scan_apply(const uint32_t *__restrict__ cnt, int64_t n,
                                                         const uint64_t *__restrict__ blk,
                                                         uint64_t *__restrict__ off_out) {
  __shared__ uint64_t sh[256];
  constexpr int PER = kTmidScan / 256;
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kTmidScan + (int64_t)tid * PER;
  uint32_t c[PER];
  uint64_t local = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    c[i] = (i0 + i < n) ? cnt[i0 + i] : 0u;
    local += c[i];
  }
  sh[tid] = local;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint64_t y = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += y;
    __syncthreads();
  }
  uint64_t run = blk[blockIdx.x] + sh[tid] - local;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (i0 + i < n) off_out[i0 + i] = run;
    run += c[i];
  }
}

// ---- per-ray sort and composite ----
constexpr int kTmidLdsKeys = 2048;   // keys sorted in LDS; longer rays sort in place in the workspace

// Ascending sort of k[0, n) by a bitonic network over the next power of two
// N2 >= n whose every compare-exchange puts the smaller key first (the first
// step of each merge compares mirrored positions).  Positions >= n stand for
// +infinity: a pair (a, b), a < b, with b >= n never swaps, so they are
// neither read nor written.  All 64 lanes of the (one-wave) workgroup call it.
__device__ void bitonic_sort_asc(uint64_t *k, uint32_t n) {
  uint32_t n2 = 1;
  while (n2 < n) n2 <<= 1;
  const int lane = threadIdx.x;
  for (uint32_t size = 2; size <= n2; size <<= 1) {
    const uint32_t half = size >> 1;
    for (uint32_t i = lane; i < n2 / 2; i += 64) {
      const uint32_t blk = i / half, o = i - blk * half;
      const uint32_t a = blk * size + o, b = blk * size + size - 1 - o;
      if (b < n) {
        const uint64_t x = k[a], y = k[b];
        if (y < x) {
          k[a] = y;
          k[b] = x;
        }
      }
    }
    __syncthreads();
    for (uint32_t stride = half >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = lane; i < n2 / 2; i += 64) {
        const uint32_t blk = i / stride, o = i - blk * stride;
        const uint32_t a = blk * 2 * stride + o, b = a + stride;
        if (b < n) {
          const uint64_t x = k[a], y = k[b];
          if (y < x) {
            k[a] = y;
            k[b] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(64) void k_tmid_composite(const uint32_t *__restrict__ ray_cnt,
                                                       const uint64_t *__restrict__ ray_off, uint64_t *hit_key,
                                                       const float4 *__restrict__ hit_val,
                                                       const int64_t *__restrict__ counters, float t_min,
                                                       float2 *__restrict__ signal) {
  __shared__ uint64_t sk[kTmidLdsKeys];
  const int64_t ray = blockIdx.x;
  const int lane = threadIdx.x;
  if (counters[3] != 0) {   // records over capacity: nothing was collected
    if (lane == 0) signal[ray] = make_float2(0.f, 0.f);
    return;
  }
  const uint32_t n = ray_cnt[ray];
  const uint64_t off = ray_off[ray];
  uint64_t *k = hit_key + off;
  if (n <= (uint32_t)kTmidLdsKeys) {
    for (uint32_t i = lane; i < n; i += 64) sk[i] = k[i];
    __syncthreads();
    k = sk;
  }
  bitonic_sort_asc(k, n);
  float T = 1.f, Sr = 0.f, Si = 0.f;
  for (uint32_t b0 = 0; b0 < n; b0 += 64) {
    const uint32_t i = b0 + lane;
    float keep = 1.f, cr = 0.f, ci = 0.f;
    if (i < n) {
      const float4 hv = hit_val[off + (uint32_t)(k[i] & kTmidRankMask)];
      keep = hv.x;
      cr = hv.y;
      ci = hv.z;
    }
    // exclusive product of the factors over the lanes (the earlier hits of this chunk)
    float incl = keep;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const float y = __shfl_up(incl, d, 64);
      if (lane >= d) incl *= y;
    }
    float excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 1.f;
    const float total = __shfl(incl, 63, 64);
    const float Tj = T * excl;
    const bool proc = (i < n) && (Tj >= t_min);
    float wr = proc ? Tj * cr : 0.f, wi = proc ? Tj * ci : 0.f;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      wr += __shfl_xor(wr, d, 64);
      wi += __shfl_xor(wi, d, 64);
    }
    Sr += wr;
    Si += wi;
    T *= total;
    if (T < t_min) break;
  }
  if (lane == 0) signal[ray] = make_float2(Sr, Si);
}

// S_hat per pair from the rays (FP64, fixed order) and RSSI.
__global__ __launch_bounds__(256) void k_ray_sum(const float2 *__restrict__ signal, int64_t n_rays,
                                                 float *__restrict__ signal_sum, float *__restrict__ rssi) {
  __shared__ double sr[256], si[256];
  const int k = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t t = threadIdx.x; t < n_rays; t += 256) {
    const float2 v = signal[(size_t)k * n_rays + t];
    a += v.x;
    b += v.y;
  }
  sr[threadIdx.x] = a;
  si[threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      sr[threadIdx.x] += sr[threadIdx.x + off];
      si[threadIdx.x] += si[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    signal_sum[2 * k] = (float)sr[0];
    signal_sum[2 * k + 1] = (float)si[0];
    if (rssi) {
      const double pw = sr[0] * sr[0] + si[0] * si[0];
      rssi[k] = pw > 0.0 ? (float)(10.0 * log10(pw)) : -INFINITY;
    }
  }
}

template <int MODE>
static hipError_t var_any(int L, int area, const RenderArgs &a, const TpIO &io, int64_t nblocks, hipStream_t s) {
  switch (L) {
    case 0: return tp_dispatch_var<0, MODE>(area, a, io, nblocks, s);
    case 1: return tp_dispatch_var<1, MODE>(area, a, io, nblocks, s);
    case 2: return tp_dispatch_var<2, MODE>(area, a, io, nblocks, s);
    case 3: return tp_dispatch_var<3, MODE>(area, a, io, nblocks, s);
    case 4: return tp_dispatch_var<4, MODE>(area, a, io, nblocks, s);
    case 5: return tp_dispatch_var<5, MODE>(area, a, io, nblocks, s);
    default: return tp_dispatch_var<6, MODE>(area, a, io, nblocks, s);
  }
}

hipError_t launch_render_fwd_variant(const gsrf_problem *p, const Layout &lay, char *ws, float *signal,
                                     float *signal_sum, float *rssi_dbm, hipStream_t s) {
  const RenderArgs a = make_render_args(p, lay, ws);
  const int64_t nblocks = (int64_t)p->n_pairs * lay.T;
  const int area = p->grid.tile_w * p->grid.tile_h;
  const int L = p->grid.fle_L;
  const int64_t n_rays = (int64_t)p->grid.n_az * p->grid.n_el;
  hipError_t e;
  if (p->grid.depth_order == 0) {
    TpIO io{};
    io.signal = (float2 *)signal;
    io.tile_sum = (float2 *)(ws + lay.tile_sum);
    mark_kernel_event(0, s);
    e = var_any<kTpFwd>(L, area, a, io, nblocks, s);
    mark_kernel_event(1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ray_sum, dim3(p->n_pairs), dim3(256), 0, s, (const float2 *)signal, n_rays, signal_sum,
                       rssi_dbm);
    return hipGetLastError();
  }
  // per-ray midpoint order
  TpIO io{};
  io.ray_cnt = (uint32_t *)(ws + lay.ray_cnt);
  io.ray_off = (const uint64_t *)(ws + lay.ray_off);
  io.hit_key = (uint64_t *)(ws + lay.hit_key);
  io.hit_val = (float4 *)(ws + lay.hit_val);
  io.counters = (const int64_t *)(ws + lay.counters);
  const int64_t n_all = n_rays * p->n_pairs;
  mark_kernel_event(0, s);
  e = var_any<kTpCount>(L, area, a, io, nblocks, s);
  if (e != hipSuccess) return e;
  const int64_t nblk = (n_all + kTmidScan - 1) / kTmidScan;
  uint64_t *blk = (uint64_t *)(ws + lay.tmid_blk);
  hipLaunchKernelGGL(k_tmid_scan_reduce, dim3((unsigned)nblk), dim3(256), 0, s, (const uint32_t *)io.ray_cnt, n_all,
                     blk);
  hipLaunchKernelGGL(k_tmid_scan_blocks, dim3(1), dim3(1024), 0, s, blk, nblk, lay.hit_cap,
                     (int64_t *)(ws + lay.counters));
  hipLaunchKernelGGL(k_tmid_scan_apply, dim3((unsigned)nblk), dim3(256), 0, s, (const uint32_t *)io.ray_cnt, n_all,
                     (const uint64_t *)blk, (uint64_t *)(ws + lay.ray_off));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = var_any<kTpCollect>(L, area, a, io, nblocks, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tmid_composite, dim3((unsigned)n_all), dim3(64), 0, s, (const uint32_t *)io.ray_cnt,
                     io.ray_off, io.hit_key, (const float4 *)io.hit_val, io.counters, p->grid.t_min,
                     (float2 *)signal);
  mark_kernel_event(1, s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_ray_sum, dim3(p->n_pairs), dim3(256), 0, s, (const float2 *)signal, n_rays, signal_sum,
                     rssi_dbm);
  return hipGetLastError();
}

}  // namespace gsrf
