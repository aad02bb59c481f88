// Steps a5-a6: complex front-to-back ray accumulation (Sec. 3.4 eq. rendering;
// App. A; Alg. 1 Blend) and the single-antenna sum (Sec. 3.4).
//
// One workgroup renders one (pair, tile).  The tile's depth-sorted Gaussian
// list is staged through LDS in batches; rays stop individually when their
// transmittance falls below t_min and the workgroup stops when all of its rays
// have.  Two traversals of a batch: the two-phase one (render_two_phase.h,
// lanes_per_ray = 0) and the direct one below, where each ray is served by G
// lanes that test and process consecutive entries.  Tile partials of S_hat are
// reduced in a fixed order, so the forward pass is deterministic.
#include "render_two_phase.h"

namespace gsrf {

template <int L, int NT, int G, bool STATS>
__global__ __launch_bounds__(NT) void k_render_fwd(RenderArgs a, float2 *__restrict__ signal,
                                                   double2 *__restrict__ sig64, float2 *__restrict__ tile_sum,
                                                   unsigned long long *__restrict__ stats) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int B = lds_batch(L, NT, false);
  constexpr int RAYS = NT / G;
  extern __shared__ float4 smem[];
  float4 *sgeo = smem;                          // [B][kGeo]
  float *scf = (float *)(smem + kGeo * B);      // [B][2K]
  const int gt = blockIdx.x;
  const int k = gt / a.T;
  const int tile = gt - k * a.T;
  const int tv = tile / a.nta, tu = tile - tv * a.nta;
  const int r = (int)threadIdx.x / G, q = (int)threadIdx.x % G;
  const int th_ = RAYS / a.tw;
  const int u = tu * a.tw + r % a.tw;
  const int v = tv * th_ + r / a.tw;
  const bool valid = (u < a.n_az) && (v < a.n_el);
  const gsrf_pair pr = a.pairs[k];
  const double inv_lam = pr.freq_hz / kC0;
  float vx = 0.f, vy = 0.f, vz = 1.f, Yr[K], Yi[K];
  ray_load<L>(valid ? u : 0, valid ? v : 0, a, vx, vy, vz, Yr, Yi);
  const uint32_t s0 = a.tstart[gt], s1 = a.tend[gt];
  float T = 1.f;
  double Sr = 0.0, Si = 0.0;   // FP64 sums of the exact products T_j c~_j (the adjoint's remainders need them)
  bool done = !valid || (1.0f < a.t_min);
  unsigned long long n_test = 0, n_hit = 0, n_staged = 0, n_tile_tests = 0;
  for (uint32_t base = s0; base < s1; base += B) {
    const int nb = (int)min((uint32_t)B, s1 - base);
    __syncthreads();
    if ((int)threadIdx.x < nb)
      stage_entry<K>(a, a.val[base + threadIdx.x], pr.rx[0], pr.rx[1], pr.rx[2], pr.tx[0], pr.tx[1], pr.tx[2], inv_lam,
                     sgeo + kGeo * threadIdx.x, scf + 2 * K * threadIdx.x);
    if (STATS && threadIdx.x == 0) {
      n_staged += nb;
      n_tile_tests += (unsigned long long)nb * min(a.tw, a.n_az - tu * a.tw) * min(th_, a.n_el - tv * th_);
    }
    __syncthreads();
    if (__ballot(!done) != 0) {              // wave-uniform
      for (int m = 0; m < nb; m += G) {
        const int j = m + q;
        Terms h;
        bool hit = false;
        float f = 1.f, ctr = 0.f, cti = 0.f;
        if (!done && j < nb) {
          if (STATS) ++n_test;
          hit = test_hit(vx, vy, vz, sgeo + kGeo * j, a.r_rx, h);
          if (hit) {
            hit_terms<K>(sgeo + kGeo * j, scf + 2 * K * j, Yr, Yi, a.amax, h);
            f = h.keep;
            ctr = h.p * h.pzr;
            cti = h.p * h.pzi;
          }
        }
        float excl, total;
        group_prod<G>(f, q, excl, total);
        const float Tj = T * excl;
        if (hit && Tj >= a.t_min) {
          Sr = fma((double)Tj, (double)ctr, Sr);
          Si = fma((double)Tj, (double)cti, Si);
          if (STATS) ++n_hit;
        }
        T = T * total;
        done = done || (T < a.t_min);
        if (__ballot(!done) == 0) break;
      }
    }
    if (__syncthreads_and(done ? 1 : 0)) break;
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      Sr += __shfl_xor(Sr, d, G);
      Si += __shfl_xor(Si, d, G);
    }
  }
  if (STATS) {
    // instrumentation: tests, processed hits, staged entries, rays, tile tests
    if (n_test) atomicAdd(stats + 0, n_test);
    if (n_hit) atomicAdd(stats + 1, n_hit);
    if (n_staged) atomicAdd(stats + 2, n_staged);
    if (valid && q == 0) atomicAdd(stats + 3, 1ull);
    if (n_tile_tests) atomicAdd(stats + 4, n_tile_tests);
    return;
  }
  if (valid && q == 0) {
    const size_t ri = ((size_t)k * a.n_el + v) * a.n_az + u;
    signal[ri] = make_float2((float)Sr, (float)Si);
    sig64[ri] = make_double2(Sr, Si);
  }
  // deterministic tile partial of S_hat (fixed tree order)
  __syncthreads();
  float *red = (float *)smem;
  red[threadIdx.x] = (q == 0) ? (float)Sr : 0.f;
  red[NT + threadIdx.x] = (q == 0) ? (float)Si : 0.f;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[threadIdx.x] += red[threadIdx.x + off];
      red[NT + threadIdx.x] += red[NT + threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_sum[gt] = make_float2(red[0], red[NT]);
}


// a6: S_hat per pair (tiles summed in fixed order, FP64) and RSSI in dBm: thread t
// takes partials t, t + 256, ... (four loads in flight), then wave butterflies and
// the four wave totals in wave order.
__global__ __launch_bounds__(256) void k_rssi(const float2 *__restrict__ tile_sum, int32_t T,
                                              float *__restrict__ signal_sum, float *__restrict__ rssi) {
  __shared__ double wr[4], wi[4];
  const int k = blockIdx.x, tid = threadIdx.x;
  const float2 *src = tile_sum + (size_t)k * T;
  double a = 0.0, b = 0.0;
  int t = tid;
  for (; t + 3 * 256 < T; t += 4 * 256) {
    const float2 x0 = src[t], x1 = src[t + 256], x2 = src[t + 512], x3 = src[t + 768];
    a += (double)x0.x;
    b += (double)x0.y;
    a += (double)x1.x;
    b += (double)x1.y;
    a += (double)x2.x;
    b += (double)x2.y;
    a += (double)x3.x;
    b += (double)x3.y;
  }
  for (; t < T; t += 256) {
    const float2 v = src[t];
    a += (double)v.x;
    b += (double)v.y;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    a += __shfl_xor(a, d, 64);
    b += __shfl_xor(b, d, 64);
  }
  if ((tid & 63) == 0) {
    wr[tid >> 6] = a;
    wi[tid >> 6] = b;
  }
  __syncthreads();
  if (tid == 0) {
    const double sr = (wr[0] + wr[1]) + (wr[2] + wr[3]), si = (wi[0] + wi[1]) + (wi[2] + wi[3]);
    signal_sum[2 * k] = (float)sr;
    signal_sum[2 * k + 1] = (float)si;
    if (rssi) {
      const double pw = sr * sr + si * si;
      rssi[k] = pw > 0.0 ? (float)(10.0 * log10(pw)) : -INFINITY;
    }
  }
}

template <int L, int NT, int G>
static hipError_t fwd_launch(const RenderArgs &a, int64_t nblocks, float2 *sig, double2 *sig64, float2 *tsum,
                             unsigned long long *stats, hipStream_t s) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int B = lds_batch(L, NT, false);
  size_t lds = (size_t)B * (kGeo * 16 + 2 * K * 4);
  if (lds < (size_t)NT * 8) lds = (size_t)NT * 8;
  if (stats)
    hipLaunchKernelGGL((k_render_fwd<L, NT, G, true>), dim3((unsigned)nblocks), dim3(NT), lds, s, a, sig, sig64, tsum,
                       stats);
  else
    hipLaunchKernelGGL((k_render_fwd<L, NT, G, false>), dim3((unsigned)nblocks), dim3(NT), lds, s, a, sig, sig64,
                       tsum, stats);
  return hipGetLastError();
}


template <int L>
static hipError_t fwd_dispatch(int area, int G, const RenderArgs &a, int64_t nblocks, float2 *sig, double2 *sig64,
                               float2 *tsum, unsigned long long *stats, hipStream_t s) {
  if (G == 0) {
    TpIO io{};
    io.signal = sig;
    io.sig64 = sig64;
    io.tile_sum = tsum;
    io.stats = stats;
    return stats ? tp_dispatch<L, kTpFwdStats>(area, a, io, nblocks, s) : tp_dispatch<L, kTpFwd>(area, a, io, nblocks, s);
  }
  switch (area * 8 + G) {
    case 64 * 8 + 1: return fwd_launch<L, 64, 1>(a, nblocks, sig, sig64, tsum, stats, s);
    case 64 * 8 + 2: return fwd_launch<L, 128, 2>(a, nblocks, sig, sig64, tsum, stats, s);
    case 64 * 8 + 4: return fwd_launch<L, 256, 4>(a, nblocks, sig, sig64, tsum, stats, s);
    case 128 * 8 + 1: return fwd_launch<L, 128, 1>(a, nblocks, sig, sig64, tsum, stats, s);
    case 128 * 8 + 2: return fwd_launch<L, 256, 2>(a, nblocks, sig, sig64, tsum, stats, s);
    case 128 * 8 + 4: return fwd_launch<L, 512, 4>(a, nblocks, sig, sig64, tsum, stats, s);
    case 256 * 8 + 1: return fwd_launch<L, 256, 1>(a, nblocks, sig, sig64, tsum, stats, s);
    case 256 * 8 + 2: return fwd_launch<L, 512, 2>(a, nblocks, sig, sig64, tsum, stats, s);
    default: return fwd_launch<L, 1024, 4>(a, nblocks, sig, sig64, tsum, stats, s);
  }
}

static hipError_t fwd_any(const gsrf_problem *p, const RenderArgs &a, int64_t nblocks, float2 *sig, double2 *sig64,
                          float2 *tsum, unsigned long long *stats, hipStream_t s) {
  const int area = p->grid.tile_w * p->grid.tile_h;
  const int G = p->grid.lanes_per_ray;   // 0: two-phase traversal
  switch (p->grid.fle_L) {
    case 0: return fwd_dispatch<0>(area, G, a, nblocks, sig, sig64, tsum, stats, s);
    case 1: return fwd_dispatch<1>(area, G, a, nblocks, sig, sig64, tsum, stats, s);
    case 2: return fwd_dispatch<2>(area, G, a, nblocks, sig, sig64, tsum, stats, s);
    case 3: return fwd_dispatch<3>(area, G, a, nblocks, sig, sig64, tsum, stats, s);
    case 4: return fwd_dispatch<4>(area, G, a, nblocks, sig, sig64, tsum, stats, s);
    case 5: return fwd_dispatch<5>(area, G, a, nblocks, sig, sig64, tsum, stats, s);
    default: return fwd_dispatch<6>(area, G, a, nblocks, sig, sig64, tsum, stats, s);
  }
}

RenderArgs make_render_args(const gsrf_problem *p, const Layout &lay, char *ws) {
  RenderArgs a;
  a.pairs = p->pairs;
  a.prep = (const float *)(ws + lay.prep);
  a.coeffs = p->coeffs;
  a.val = (const uint32_t *)(ws + lay.val);
  a.tstart = (const uint32_t *)(ws + lay.tile_start);
  a.tend = (const uint32_t *)(ws + lay.tile_end);
  a.hitmask = (uint32_t *)(ws + lay.hitmask);
  a.mask_end = (uint32_t *)(ws + lay.mask_end);
  a.rays = (const float *)(ws + lay.rays);
  a.logits = p->opacity_logits;
  a.fle_g = p->grid.fle_eval;
  a.chord = p->grid.transmittance;
  a.T = lay.T;
  a.nta = lay.nta;
  a.n_az = p->grid.n_az;
  a.n_el = p->grid.n_el;
  a.tw = p->grid.tile_w;
  a.el_lo = p->grid.el_lo;
  a.el_hi = p->grid.el_hi;
  a.r_rx = p->grid.r_rx;
  a.t_min = p->grid.t_min;
  a.amax = p->grid.alpha_max;
  return a;
}

hipError_t launch_render_fwd(const gsrf_problem *p, const Layout &lay, char *ws, float *signal, float *signal_sum,
                             float *rssi_dbm, hipStream_t s) {
  if (p->n_pairs == 0) return hipSuccess;
  if (has_variant(p->grid)) return launch_render_fwd_variant(p, lay, ws, signal, signal_sum, rssi_dbm, s);
  const RenderArgs a = make_render_args(p, lay, ws);
  const int64_t nblocks = (int64_t)p->n_pairs * lay.T;
  float2 *tsum = (float2 *)(ws + lay.tile_sum);
  mark_kernel_event(0, s);
  hipError_t e = fwd_any(p, a, nblocks, (float2 *)signal, (double2 *)(ws + lay.sig64), tsum, nullptr, s);
  mark_kernel_event(1, s);
  if (e != hipSuccess) return e;
  // partials per pair: one per render workgroup of the pair's tiles
  const int split = p->grid.lanes_per_ray == 0 ? tp_split(p->grid.tile_w * p->grid.tile_h, nblocks, p->grid.tile_h) : 1;
  hipLaunchKernelGGL(k_rssi, dim3(p->n_pairs), dim3(256), 0, s, tsum, lay.T * split, signal_sum, rssi_dbm);
  return hipGetLastError();
}

// S_hat of every (pair, carrier) of a multi-carrier render: one workgroup of
// 1024 threads sums the carrier's spectrum in FP64 in a fixed order (thread t
// takes rays t, t + 1024, ... with four loads in flight, then the threads'
// sums are reduced by wave butterflies and the 16 wave sums in wave order).
constexpr int kSumThreads = 1024;
__global__ __launch_bounds__(kSumThreads) void k_sum_multi(const float2 *__restrict__ multi, int64_t n_rays,
                                                           int n_freq, float *__restrict__ signal_sum) {
  __shared__ double wr[kSumThreads / 64], wi[kSumThreads / 64];
  const int f = blockIdx.x, k = blockIdx.y, tid = threadIdx.x;
  const float2 *src = multi + ((size_t)k * n_freq + f) * n_rays;
  double a = 0.0, b = 0.0;
  int64_t i = tid;
  for (; i + 3 * kSumThreads < n_rays; i += 4 * kSumThreads) {
    const float2 x0 = src[i], x1 = src[i + kSumThreads], x2 = src[i + 2 * kSumThreads], x3 = src[i + 3 * kSumThreads];
    a += (double)x0.x;
    b += (double)x0.y;
    a += (double)x1.x;
    b += (double)x1.y;
    a += (double)x2.x;
    b += (double)x2.y;
    a += (double)x3.x;
    b += (double)x3.y;
  }
  for (; i < n_rays; i += kSumThreads) {
    const float2 x = src[i];
    a += (double)x.x;
    b += (double)x.y;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    a += __shfl_xor(a, d, 64);
    b += __shfl_xor(b, d, 64);
  }
  if ((tid & 63) == 0) {
    wr[tid >> 6] = a;
    wi[tid >> 6] = b;
  }
  __syncthreads();
  if (tid == 0) {
    double x = 0.0, y = 0.0;
    for (int w = 0; w < kSumThreads / 64; ++w) {
      x += wr[w];
      y += wi[w];
    }
    signal_sum[2 * ((size_t)k * n_freq + f)] = (float)x;
    signal_sum[2 * ((size_t)k * n_freq + f) + 1] = (float)y;
  }
}

hipError_t launch_render_fwd_multi(const gsrf_problem *p, const Layout &lay, char *ws, int32_t n_freq, double f_step,
                                   float *signal, float *signal_sum, hipStream_t s) {
  if (p->n_pairs == 0 || n_freq == 0) return hipSuccess;
  const RenderArgs a = make_render_args(p, lay, ws);
  const int64_t nblocks = (int64_t)p->n_pairs * lay.T;
  const int area = p->grid.tile_w * p->grid.tile_h;
  TpIO io{};
  io.multi = (float2 *)signal;
  io.n_freq = n_freq;
  io.f_step = f_step;
  hipError_t e = hipSuccess;
  mark_kernel_event(0, s);
  for (int f0 = 0; f0 < n_freq && e == hipSuccess;) {   // one traversal per chunk of carriers
    io.f_first = f0;
    const bool wide = n_freq - f0 > kMultiChunk;
    switch (p->grid.fle_L) {
      case 0: e = wide ? tp_dispatch<0, kTpFwdMultiWide>(area, a, io, nblocks, s)
                       : tp_dispatch<0, kTpFwdMulti>(area, a, io, nblocks, s); break;
      case 1: e = wide ? tp_dispatch<1, kTpFwdMultiWide>(area, a, io, nblocks, s)
                       : tp_dispatch<1, kTpFwdMulti>(area, a, io, nblocks, s); break;
      case 2: e = wide ? tp_dispatch<2, kTpFwdMultiWide>(area, a, io, nblocks, s)
                       : tp_dispatch<2, kTpFwdMulti>(area, a, io, nblocks, s); break;
      case 3: e = wide ? tp_dispatch<3, kTpFwdMultiWide>(area, a, io, nblocks, s)
                       : tp_dispatch<3, kTpFwdMulti>(area, a, io, nblocks, s); break;
      case 4: e = wide ? tp_dispatch<4, kTpFwdMultiWide>(area, a, io, nblocks, s)
                       : tp_dispatch<4, kTpFwdMulti>(area, a, io, nblocks, s); break;
      case 5: e = wide ? tp_dispatch<5, kTpFwdMultiWide>(area, a, io, nblocks, s)
                       : tp_dispatch<5, kTpFwdMulti>(area, a, io, nblocks, s); break;
      default: e = wide ? tp_dispatch<6, kTpFwdMultiWide>(area, a, io, nblocks, s)
                        : tp_dispatch<6, kTpFwdMulti>(area, a, io, nblocks, s); break;
    }
    f0 += wide ? kMultiChunkWide : kMultiChunk;
  }
  if (e != hipSuccess) return e;
  mark_kernel_event(1, s);
  hipLaunchKernelGGL(k_sum_multi, dim3((unsigned)n_freq, (unsigned)p->n_pairs), dim3(kSumThreads), 0, s,
                     (const float2 *)signal, (int64_t)p->grid.n_el * p->grid.n_az, n_freq, signal_sum);
  return hipGetLastError();
}

hipError_t launch_render_stats(const gsrf_problem *p, const Layout &lay, char *ws, int64_t *counts, hipStream_t s) {
  hipError_t e = fill<int64_t>(counts, 0, 6, s);
  if (e != hipSuccess || p->n_pairs == 0) return e;
  const RenderArgs a = make_render_args(p, lay, ws);
  const int64_t nblocks = (int64_t)p->n_pairs * lay.T;
  return fwd_any(p, a, nblocks, nullptr, nullptr, nullptr, (unsigned long long *)counts, s);
}

}  // namespace gsrf
