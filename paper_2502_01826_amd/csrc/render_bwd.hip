// Steps a7-a8: the adjoint of the renderer (App. C backward kernel; App. D)
// and the per-Gaussian chain rule through Sigma^-1 = R diag(s^-2) R^T (the
// covariance gradient App. D.3 omits).
//
// Same traversal as the forward (render_common.h), recomputing each ray's
// transmittance front to back; the remainder R_j = sum_{i>j} T_i c~_i comes
// from the forward's S minus the running prefix, both FP64 sums of the same
// exact products T_i c~_i, so it is accurate to the size of the remainder
// itself (zero after a ray's last hit) and only S is kept between the passes.  Per processed hit a lane forms its contribution
// to the Gaussian's accumulators; the rays of a wave are summed by a
// reduce-scatter (recursive halving over lanes), the waves meet in LDS, and
// one burst of global atomics per (tile, Gaussian) flushes them.
#include "render_two_phase.h"

namespace gsrf {

template <int L, int NT, int G>
__global__ __launch_bounds__(NT) void k_render_bwd(RenderArgs a, const double2 *__restrict__ sig64,
                                                   const float2 *__restrict__ grad_signal,
                                                   const float2 *__restrict__ grad_sum, float *__restrict__ acc,
                                                   int acc_stride) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int B = lds_batch(L, NT, true);
  constexpr int NACC = n_acc(L);               // 12 + 2K
  constexpr int NV = pow2_at_least(NACC);
  constexpr int RAYS = NT / G;
  extern __shared__ float4 smem[];
  float4 *sgeo = smem;                          // [B][kGeo]
  float4 *stx = smem + kGeo * B;                // [B] TX leg, Gaussian id
  float *scf = (float *)(stx + B);              // [B][2K]
  float *sacc = scf + 2 * K * B;                // [B][NACC]
  uint32_t *sflag = (uint32_t *)(sacc + NACC * B);   // [B]
  const int gt = blockIdx.x;
  const int k = gt / a.T;
  const int tile = gt - k * a.T;
  const int tv = tile / a.nta, tu = tile - tv * a.nta;
  const int r = (int)threadIdx.x / G, q = (int)threadIdx.x % G;
  const int th_ = RAYS / a.tw;
  const int u = tu * a.tw + r % a.tw;
  const int v = tv * th_ + r / a.tw;
  const bool valid = (u < a.n_az) && (v < a.n_el);
  const int lane = threadIdx.x & 63;
  const gsrf_pair pr = a.pairs[k];
  const double lam = kC0 / pr.freq_hz, inv_lam = pr.freq_hz / kC0;
  const float twopi_lam = (float)(2.0 * 3.14159265358979323846 / lam);
  float vx = 0.f, vy = 0.f, vz = 1.f, Yr[K], Yi[K];
  ray_load<L>(valid ? u : 0, valid ? v : 0, a, vx, vy, vz, Yr, Yi);
  float Gr = 0.f, Gi = 0.f;
  double Sfr = 0.0, Sfi = 0.0;   // the forward's FP64 S
  if (valid) {
    const size_t ri = ((size_t)k * a.n_el + v) * a.n_az + u;
    const double2 sf = sig64[ri];
    const float2 gg = grad_signal[ri];
    Sfr = sf.x; Sfi = sf.y; Gr = gg.x; Gi = gg.y;
    if (grad_sum) {
      const float2 gs = grad_sum[k];
      Gr += gs.x;
      Gi += gs.y;
    }
  }
  for (int i = threadIdx.x; i < NACC * B; i += NT) sacc[i] = 0.f;
  for (int i = threadIdx.x; i < B; i += NT) sflag[i] = 0u;
  const uint32_t s0 = a.tstart[gt], s1 = a.tend[gt];
  float T = 1.f;
  double Pr = 0.0, Pi = 0.0;     // FP64 prefix of the exact products T_j c~_j, as the forward summed them
  bool done = !valid || (1.0f < a.t_min);
  for (uint32_t base = s0; base < s1; base += B) {
    const int nb = (int)min((uint32_t)B, s1 - base);
    __syncthreads();
    if ((int)threadIdx.x < nb)
      stage_entry<K>(a, a.val[base + threadIdx.x], pr.rx[0], pr.rx[1], pr.rx[2], pr.tx[0], pr.tx[1], pr.tx[2], inv_lam,
                     sgeo + kGeo * threadIdx.x, scf + 2 * K * threadIdx.x, stx + threadIdx.x);
    for (int i = threadIdx.x; i < nb; i += NT) {   // what the previous batch's flush left
      sflag[i] = 0u;
      sacc[NACC * i + NACC - 1] = 0.f;
    }
    __syncthreads();
    if (__ballot(!done) != 0) {              // wave-uniform
      for (int m = 0; m < nb; m += G) {
        const int j = m + q;
        const float4 *geo = sgeo + kGeo * j;
        Terms h;
        bool hit = false;
        float f = 1.f, ctr = 0.f, cti = 0.f;
        if (!done && j < nb) {
          hit = test_hit(vx, vy, vz, geo, a.r_rx, h);
          if (hit) {
            hit_terms<K>(geo, scf + 2 * K * j, Yr, Yi, a.amax, h);
            f = h.keep;
            ctr = h.p * h.pzr;
            cti = h.p * h.pzi;
          }
        }
        float excl, total;
        group_prod<G>(f, q, excl, total);
        const float Tj = T * excl;
        const bool proc = hit && (Tj >= a.t_min);
        const double wr = proc ? (double)Tj * (double)ctr : 0.0, wi = proc ? (double)Tj * (double)cti : 0.0;
        double wr_in, wi_in, wr_tot, wi_tot;
        group_sum64<G>(wr, q, wr_in, wr_tot);
        group_sum64<G>(wi, q, wi_in, wi_tot);
        T = T * total;
        done = done || (T < a.t_min);
        if (__ballot(proc) != 0) {
          float c[NV];
#pragma unroll
          for (int i = 0; i < NV; ++i) c[i] = 0.f;
          if (proc) {
            const float Rr = (float)(Sfr - (Pr + wr_in)), Ri = (float)(Sfi - (Pi + wi_in));
            hit_adjoint<K, NV>(h, geo, Tj, ctr, cti, Rr, Ri, Gr, Gi, vx, vy, vz, Yr, Yi, twopi_lam, c);
            sflag[j] = 1;
          }
          int first;
          bool writer;
          reduce_scatter<NV, G>(c, lane, &first, &writer);
          constexpr int NF = (NV * G >= 64) ? NV * G / 64 : 1;
          if (writer && j < nb) {
            float *dst = sacc + NACC * j;
#pragma unroll
            for (int i = 0; i < NF; ++i)
              if (first + i < NACC) atomicAdd(dst + first + i, c[i]);
          }
        }
        Pr += wr_tot;
        Pi += wi_tot;
        if (__ballot(!done) == 0) break;
      }
    }
    __syncthreads();
    // flush the staged Gaussians with any processed hit in this tile
    flush_batch<K, NT>(nb, sacc, sflag, stx, acc, acc_stride);
    if (__syncthreads_and(done ? 1 : 0)) break;
  }
}


// ---------------------------------------------------------------------------
// a8: chain rule per Gaussian from (dL/dM, dL/dmu, dL/dN, dL/do, dL/dc) to the
// stored parameters.  M = R D R^T with D = diag(exp(-2 log s)):
//   dL/dD_ii = (R^T G R)_ii, dL/dR = 2 G R D (G = symmetric dL/dM),
//   N = (2 pi)^-3/2 exp(-sum log s) gives dN/dlog s_i = -N,
//   q_hat = q / |q| gives dL/dq = (g - q_hat (q_hat . g)) / |q|,
//   o = sigmoid(a) gives do/da = o (1 - o).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chain(const float *__restrict__ log_scales, const float *__restrict__ quats,
                                               const float *__restrict__ logits, const float *__restrict__ acc,
                                               int32_t S, int32_t K, int64_t G, float *__restrict__ d_means,
                                               float *__restrict__ d_ls, float *__restrict__ d_q,
                                               float *__restrict__ d_a, float *__restrict__ d_c) {
  const int64_t g0 = (int64_t)blockIdx.x * 256;
  const int64_t g = g0 + threadIdx.x;
  // coefficient gradients: coalesced writes of this block's contiguous [256][2K] slab;
  // element e = l * 2K + c of the slab, (l, c) advanced without a division per element
  {
    const int two_k = 2 * K;
    const int total = (int)min((int64_t)256, G - g0) * two_k;
    const int step_l = 256 / two_k, step_c = 256 - step_l * two_k;
    int l = (int)threadIdx.x / two_k, c = (int)threadIdx.x - l * two_k;
    const float *src = acc + (size_t)g0 * S + 11;
    float *dst = d_c + (size_t)g0 * two_k;
    for (int e = threadIdx.x; e < total; e += 256) {
      dst[e] = src[(size_t)l * S + c];
      l += step_l;
      c += step_c;
      if (c >= two_k) {
        c -= two_k;
        ++l;
      }
    }
  }
  if (g >= G) return;
  const float4 *row4 = (const float4 *)(acc + (size_t)g * S);   // rows are 64-byte aligned
  const float4 r0 = row4[0], r1 = row4[1], r2 = row4[2];
  const float rv[12] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w};
  auto A = [&](int f) { return rv[f]; };
  const float Gm[3][3] = {{A(0), A(3), A(4)}, {A(3), A(1), A(5)}, {A(4), A(5), A(2)}};
  d_means[3 * g + 0] = A(6);
  d_means[3 * g + 1] = A(7);
  d_means[3 * g + 2] = A(8);
  const float dN = A(9), dO = A(10);
  float qw = quats[4 * g + 0], qx = quats[4 * g + 1], qy = quats[4 * g + 2], qz = quats[4 * g + 3];
  const float qn = sqrtf(fmaf(qw, qw, fmaf(qx, qx, fmaf(qy, qy, qz * qz))));
  qw /= qn; qx /= qn; qy /= qn; qz /= qn;
  float R[3][3];
  R[0][0] = 1.f - 2.f * (qy * qy + qz * qz); R[0][1] = 2.f * (qx * qy - qw * qz); R[0][2] = 2.f * (qx * qz + qw * qy);
  R[1][0] = 2.f * (qx * qy + qw * qz); R[1][1] = 1.f - 2.f * (qx * qx + qz * qz); R[1][2] = 2.f * (qy * qz - qw * qx);
  R[2][0] = 2.f * (qx * qz - qw * qy); R[2][1] = 2.f * (qy * qz + qw * qx); R[2][2] = 1.f - 2.f * (qx * qx + qy * qy);
  const float l0 = log_scales[3 * g + 0], l1 = log_scales[3 * g + 1], l2 = log_scales[3 * g + 2];
  const float d[3] = {expf(-2.f * l0), expf(-2.f * l1), expf(-2.f * l2)};
  const float Nn = (float)0.063493635934240969 * expf(-(l0 + l1 + l2));
  float GR[3][3];
  for (int a_ = 0; a_ < 3; ++a_)
    for (int i = 0; i < 3; ++i) GR[a_][i] = fmaf(Gm[a_][0], R[0][i], fmaf(Gm[a_][1], R[1][i], Gm[a_][2] * R[2][i]));
  for (int i = 0; i < 3; ++i) {
    const float gd = fmaf(R[0][i], GR[0][i], fmaf(R[1][i], GR[1][i], R[2][i] * GR[2][i]));
    d_ls[3 * g + i] = fmaf(-2.f * d[i], gd, -Nn * dN);
  }
  float gR[3][3];
  for (int a_ = 0; a_ < 3; ++a_)
    for (int i = 0; i < 3; ++i) gR[a_][i] = 2.f * GR[a_][i] * d[i];
  const float gw = 2.f * (-qz * gR[0][1] + qy * gR[0][2] + qz * gR[1][0] - qx * gR[1][2] - qy * gR[2][0] + qx * gR[2][1]);
  const float gx = 2.f * (qy * gR[0][1] + qz * gR[0][2] + qy * gR[1][0] - 2.f * qx * gR[1][1] - qw * gR[1][2] +
                          qz * gR[2][0] + qw * gR[2][1] - 2.f * qx * gR[2][2]);
  const float gy = 2.f * (-2.f * qy * gR[0][0] + qx * gR[0][1] + qw * gR[0][2] + qx * gR[1][0] + qz * gR[1][2] -
                          qw * gR[2][0] + qz * gR[2][1] - 2.f * qy * gR[2][2]);
  const float gz = 2.f * (-2.f * qz * gR[0][0] - qw * gR[0][1] + qx * gR[0][2] + qw * gR[1][0] - 2.f * qz * gR[1][1] +
                          qy * gR[1][2] + qx * gR[2][0] + qy * gR[2][1]);
  const float dot = fmaf(qw, gw, fmaf(qx, gx, fmaf(qy, gy, qz * gz)));
  d_q[4 * g + 0] = (gw - qw * dot) / qn;
  d_q[4 * g + 1] = (gx - qx * dot) / qn;
  d_q[4 * g + 2] = (gy - qy * dot) / qn;
  d_q[4 * g + 3] = (gz - qz * dot) / qn;
  const float o = 1.f / (1.f + expf(-logits[g]));
  d_a[g] = dO * o * (1.f - o);
}

template <int L, int NT, int G>
static hipError_t bwd_launch(const RenderArgs &a, int64_t nblocks, const double2 *sig, const float2 *gsig,
                             const float2 *gsum, float *acc, int S, hipStream_t s) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int B = lds_batch(L, NT, true);
  const size_t lds = (size_t)B * (kGeo * 16 + 16 + 2 * K * 4 + n_acc(L) * 4 + 4);
  hipLaunchKernelGGL((k_render_bwd<L, NT, G>), dim3((unsigned)nblocks), dim3(NT), lds, s, a, sig, gsig, gsum, acc, S);
  return hipGetLastError();
}


template <int L>
static hipError_t bwd_dispatch(int area, int G, const RenderArgs &a, int64_t nblocks, const double2 *sig,
                               const float2 *gsig, const float2 *gsum, float *acc, int S, hipStream_t s) {
  if (G == 0) {
    TpIO io{};
    io.sig64 = const_cast<double2 *>(sig);
    io.grad_signal = gsig;
    io.grad_sum = gsum;
    io.acc = acc;
    io.acc_stride = S;
    return tp_dispatch<L, kTpBwd>(area, a, io, nblocks, s);
  }
  switch (area * 8 + G) {
    case 64 * 8 + 1: return bwd_launch<L, 64, 1>(a, nblocks, sig, gsig, gsum, acc, S, s);
    case 64 * 8 + 2: return bwd_launch<L, 128, 2>(a, nblocks, sig, gsig, gsum, acc, S, s);
    case 64 * 8 + 4: return bwd_launch<L, 256, 4>(a, nblocks, sig, gsig, gsum, acc, S, s);
    case 128 * 8 + 1: return bwd_launch<L, 128, 1>(a, nblocks, sig, gsig, gsum, acc, S, s);
    case 128 * 8 + 2: return bwd_launch<L, 256, 2>(a, nblocks, sig, gsig, gsum, acc, S, s);
    case 128 * 8 + 4: return bwd_launch<L, 512, 4>(a, nblocks, sig, gsig, gsum, acc, S, s);
    case 256 * 8 + 1: return bwd_launch<L, 256, 1>(a, nblocks, sig, gsig, gsum, acc, S, s);
    case 256 * 8 + 2: return bwd_launch<L, 512, 2>(a, nblocks, sig, gsig, gsum, acc, S, s);
    default: return bwd_launch<L, 1024, 4>(a, nblocks, sig, gsig, gsum, acc, S, s);
  }
}

hipError_t launch_render_bwd(const gsrf_problem *p, const Layout &lay, char *ws, const float *signal,
                             const float *grad_signal, const float *grad_sum, float *d_means, float *d_log_scales,
                             float *d_quats, float *d_logits, float *d_coeffs, hipStream_t s) {
  float *acc = (float *)(ws + lay.grad_acc);
  hipError_t e = fill<float>(acc, 0.f, p->n_gauss * lay.acc_stride, s);
  if (e != hipSuccess) return e;
  if (p->n_pairs > 0) {
    const RenderArgs a = make_render_args(p, lay, ws);
    const int area = p->grid.tile_w * p->grid.tile_h;
    const int G = p->grid.lanes_per_ray;   // 0: two-phase traversal
    const int64_t nb = (int64_t)p->n_pairs * lay.T;
    // S of the preceding gsrf_render_fwd in FP64 (its workspace copy; `signal` is that
    // forward's FP32 output and is not read here)
    const double2 *sg = (const double2 *)(ws + lay.sig64);
    const float2 *gs = (const float2 *)grad_signal, *gm = (const float2 *)grad_sum;
    mark_kernel_event(2, s);
    switch (p->grid.fle_L) {
      case 0: e = bwd_dispatch<0>(area, G, a, nb, sg, gs, gm, acc, lay.acc_stride, s); break;
      case 1: e = bwd_dispatch<1>(area, G, a, nb, sg, gs, gm, acc, lay.acc_stride, s); break;
      case 2: e = bwd_dispatch<2>(area, G, a, nb, sg, gs, gm, acc, lay.acc_stride, s); break;
      case 3: e = bwd_dispatch<3>(area, G, a, nb, sg, gs, gm, acc, lay.acc_stride, s); break;
      case 4: e = bwd_dispatch<4>(area, G, a, nb, sg, gs, gm, acc, lay.acc_stride, s); break;
      case 5: e = bwd_dispatch<5>(area, G, a, nb, sg, gs, gm, acc, lay.acc_stride, s); break;
      default: e = bwd_dispatch<6>(area, G, a, nb, sg, gs, gm, acc, lay.acc_stride, s); break;
    }
    mark_kernel_event(3, s);
    if (e != hipSuccess) return e;
  }
  if (p->n_gauss > 0) {
    hipLaunchKernelGGL(k_chain, dim3((unsigned)((p->n_gauss + 255) / 256)), dim3(256), 0, s, p->log_scales, p->quats,
                       p->opacity_logits, (const float *)acc, lay.acc_stride, lay.K, p->n_gauss, d_means, d_log_scales, d_quats,
                       d_logits, d_coeffs);
  }
  return hipGetLastError();
}

}  // namespace gsrf

namespace gsrf {

// Several carriers (OFDM subcarriers, Sec. 4): per chunk of kGcChunk carriers a
// total pass and an adjoint pass over the forward's hit masks (the carriers
// share every hit decision); every chunk adds into the same accumulators and
// the chain rule runs once.
template <int L>
static hipError_t bwd_multi_chunks(int area, const RenderArgs &a, int64_t nblocks, int32_t n_freq, double f_step,
                                   const float2 *gsig, const float2 *gsum, double *wtot, float *acc, int S,
                                   hipStream_t s) {
  for (int32_t f0 = 0; f0 < n_freq; f0 += kGcChunk) {
    TpIO io{};
    io.n_freq = n_freq;
    io.f_first = f0;
    io.f_step = f_step;
    io.grad_multi = gsig;
    io.grad_sum_multi = gsum;
    io.wtot = wtot;
    io.acc = acc;
    io.acc_stride = S;
    hipError_t e = tp_dispatch<L, kTpMultiTotal>(area, a, io, nblocks, s);
    if (e != hipSuccess) return e;
    e = tp_dispatch<L, kTpBwdMulti>(area, a, io, nblocks, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_render_bwd_multi(const gsrf_problem *p, const Layout &lay, char *ws, int32_t n_freq, double f_step,
                                   const float *grad_signal, const float *grad_sum, float *d_means,
                                   float *d_log_scales, float *d_quats, float *d_logits, float *d_coeffs,
                                   hipStream_t s) {
  float *acc = (float *)(ws + lay.grad_acc);
  hipError_t e = fill<float>(acc, 0.f, p->n_gauss * lay.acc_stride, s);
  if (e != hipSuccess) return e;
  if (p->n_pairs > 0) {
    const RenderArgs a = make_render_args(p, lay, ws);
    const int area = p->grid.tile_w * p->grid.tile_h;
    const int64_t nb = (int64_t)p->n_pairs * lay.T;
    const float2 *gs = (const float2 *)grad_signal, *gm = (const float2 *)grad_sum;
    double *wt = (double *)(ws + lay.wtot);    // the per-ray totals of a chunk
    mark_kernel_event(2, s);
    switch (p->grid.fle_L) {
      case 0: e = bwd_multi_chunks<0>(area, a, nb, n_freq, f_step, gs, gm, wt, acc, lay.acc_stride, s); break;
      case 1: e = bwd_multi_chunks<1>(area, a, nb, n_freq, f_step, gs, gm, wt, acc, lay.acc_stride, s); break;
      case 2: e = bwd_multi_chunks<2>(area, a, nb, n_freq, f_step, gs, gm, wt, acc, lay.acc_stride, s); break;
      case 3: e = bwd_multi_chunks<3>(area, a, nb, n_freq, f_step, gs, gm, wt, acc, lay.acc_stride, s); break;
      case 4: e = bwd_multi_chunks<4>(area, a, nb, n_freq, f_step, gs, gm, wt, acc, lay.acc_stride, s); break;
      case 5: e = bwd_multi_chunks<5>(area, a, nb, n_freq, f_step, gs, gm, wt, acc, lay.acc_stride, s); break;
      default: e = bwd_multi_chunks<6>(area, a, nb, n_freq, f_step, gs, gm, wt, acc, lay.acc_stride, s); break;
    }
    mark_kernel_event(3, s);
    if (e != hipSuccess) return e;
  }
  if (p->n_gauss > 0) {
    hipLaunchKernelGGL(k_chain, dim3((unsigned)((p->n_gauss + 255) / 256)), dim3(256), 0, s, p->log_scales, p->quats,
                       p->opacity_logits, (const float *)acc, lay.acc_stride, lay.K, p->n_gauss, d_means, d_log_scales,
                       d_quats, d_logits, d_coeffs);
  }
  return hipGetLastError();
}

}  // namespace gsrf
