// Steps a1-a2: per-Gaussian activation and orthographic splatting of every
// (pair, Gaussian) record, plus the exclusive scans used by binning.
//
// Activation follows the covariance factorisation Sigma = R S S^T R^T
// (Sec. 2 3DGS preliminaries; App. B) and the normalised pdf of App. A.3.
// Splatting follows Sec. 3.3 (splatting process) with a conservative cap in
// place of the linearised 3 sqrt(lambda_max) footprint: the Gaussian's 3-sigma
// ellipsoid lies inside a sphere of radius 3 max(s), whose directions from the
// receiver form a cap of half-angle asin(3 max(s) / D).
#include "gsrf_internal.h"

namespace gsrf {

// ---------------------------------------------------------------------------
// a1: activation.  prep[g] = {mu, N, M (6 unique), o}.
//   M = Sigma^-1 = R diag(exp(-2 log s)) R^T, N = (2 pi)^-3/2 exp(-sum log s),
//   o = sigmoid(logit).  The quaternion (w,x,y,z) is normalised first.
// ---------------------------------------------------------------------------
__global__ void k_activate(const float *__restrict__ means, const float *__restrict__ log_scales,
                           const float *__restrict__ quats, const float *__restrict__ logits, int64_t G,
                           float *__restrict__ prep) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  float qw = quats[4 * g + 0], qx = quats[4 * g + 1], qy = quats[4 * g + 2], qz = quats[4 * g + 3];
  float qn = sqrtf(fmaf(qw, qw, fmaf(qx, qx, fmaf(qy, qy, qz * qz))));
  qw /= qn; qx /= qn; qy /= qn; qz /= qn;
  float R[3][3];
  R[0][0] = 1.f - 2.f * (qy * qy + qz * qz); R[0][1] = 2.f * (qx * qy - qw * qz); R[0][2] = 2.f * (qx * qz + qw * qy);
  R[1][0] = 2.f * (qx * qy + qw * qz); R[1][1] = 1.f - 2.f * (qx * qx + qz * qz); R[1][2] = 2.f * (qy * qz - qw * qx);
  R[2][0] = 2.f * (qx * qz - qw * qy); R[2][1] = 2.f * (qy * qz + qw * qx); R[2][2] = 1.f - 2.f * (qx * qx + qy * qy);
  float l0 = log_scales[3 * g + 0], l1 = log_scales[3 * g + 1], l2 = log_scales[3 * g + 2];
  float d[3] = {expf(-2.f * l0), expf(-2.f * l1), expf(-2.f * l2)};
  float M[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      M[a][b] = fmaf(R[a][0] * d[0], R[b][0], fmaf(R[a][1] * d[1], R[b][1], R[a][2] * d[2] * R[b][2]));
  const float inv_2pi_15 = (float)0.063493635934240969;  // (2 pi)^(-3/2)
  float *o = prep + kPrep * g;
  o[0] = means[3 * g + 0];
  o[1] = means[3 * g + 1];
  o[2] = means[3 * g + 2];
  o[3] = inv_2pi_15 * expf(-(l0 + l1 + l2));
  o[4] = M[0][0]; o[5] = M[1][1]; o[6] = M[2][2];
  o[7] = 0.5f * (M[0][1] + M[1][0]); o[8] = 0.5f * (M[0][2] + M[2][0]); o[9] = 0.5f * (M[1][2] + M[2][1]);
  o[10] = 1.f / (1.f + expf(-logits[g]));
  o[11] = 0.f; o[12] = 0.f; o[13] = 0.f; o[14] = 0.f; o[15] = 0.f;
}

// Record base of each pair: rec_base[k] = sum_{k'<k} |scene(k')|, rec_base[P] = R.
__global__ void k_rec_base(const gsrf_pair *__restrict__ pairs, const int64_t *__restrict__ scene_off,
                           int32_t P, int64_t *__restrict__ rec_base) {
  __shared__ int64_t sh[1024];
  const int tid = threadIdx.x;
  const int per = (P + 1023) / 1024;
  const int lo = tid * per, hi = min(P, lo + per);
  int64_t local = 0;
  for (int k = lo; k < hi; ++k) {
    int s = pairs[k].scene;
    local += scene_off[s + 1] - scene_off[s];
  }
  sh[tid] = local;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += v;
    __syncthreads();
  }
  int64_t run = sh[tid] - local;
  for (int k = lo; k < hi; ++k) {
    rec_base[k] = run;
    int s = pairs[k].scene;
    run += scene_off[s + 1] - scene_off[s];
  }
  if (tid == 1023) rec_base[P] = sh[1023];
}

// ---------------------------------------------------------------------------
// a2: per (pair, Gaussian) depth key and conservative tile rectangle, FP64.
//   e = mu - r, D^2 = (ex ex + ey ey) + ez ez (no FMA), key = bits(fp32(D^2)).
//   Culled if D + Rb < r_rx (1 - 1e-6) with Rb = 3 max(s).  If D <= Rb (1+1e-6)
//   every row and column is covered.  Otherwise theta = asin(Rb/D) + slack,
//   rows with centre elevation in [beta_c - theta, beta_c + theta], and columns
//   with centre azimuth within asin(sin theta / cos beta_c) of alpha_c unless
//   the band reaches a pole.  Columns wrap at the azimuth seam.
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
__global__ void k_project(const gsrf_pair *__restrict__ pairs, const int64_t *__restrict__ scene_off,
                          const int64_t *__restrict__ rec_base, const float *__restrict__ means,
                          const float *__restrict__ log_scales, gsrf_grid grid, int32_t nta,
                          uint32_t *__restrict__ rec_key, ushort4 *__restrict__ rec_rect,
                          uint32_t *__restrict__ rec_cnt) {
  const int k = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const gsrf_pair pr = pairs[k];
  const int64_t g0 = scene_off[pr.scene];
  const int64_t n = scene_off[pr.scene + 1] - g0;
  if (j >= n) return;
  const int64_t g = g0 + j;
  const int64_t r = rec_base[k] + j;
  const double ex = (double)means[3 * g + 0] - (double)pr.rx[0];
  const double ey = (double)means[3 * g + 1] - (double)pr.rx[1];
  const double ez = (double)means[3 * g + 2] - (double)pr.rx[2];
  const double D2 = (ex * ex + ey * ey) + ez * ez;
  rec_key[r] = __float_as_uint((float)D2);
  const double D = sqrt(D2);
  const double lmax = fmax(fmax((double)log_scales[3 * g + 0], (double)log_scales[3 * g + 1]),
                           (double)log_scales[3 * g + 2]);
  const double Rb = 3.0 * exp(lmax);
  const int n_az = grid.n_az, n_el = grid.n_el, tw = grid.tile_w, th = grid.tile_h;
  const double el_lo = (double)grid.el_lo, el_hi = (double)grid.el_hi;
  const double pi = 3.14159265358979323846;
  ushort4 rect = make_ushort4(0, 0, 0, 0);
  uint32_t cnt = 0;
  bool visible = !(D + Rb < (double)grid.r_rx * (1.0 - 1e-6));
  if (visible) {
    const bool inside = D <= Rb * (1.0 + 1e-6);
    long v_lo, v_hi, u_lo, u_hi;
    bool full;
    if (inside) {
      v_lo = 0; v_hi = n_el - 1; full = true; u_lo = 0; u_hi = n_az - 1;
    } else {
      const double theta = asin(fmin(Rb / D, 1.0)) + kCapSlack;
      const double bc = atan2(ez, sqrt(ex * ex + ey * ey));
      const double lo = bc - theta, hi = bc + theta;
      const double dbeta = (el_hi - el_lo) / n_el;
      v_lo = (long)ceil((lo - el_lo) / dbeta - 0.5);
      v_hi = (long)floor((hi - el_lo) / dbeta - 0.5);
      if (v_lo < 0) v_lo = 0;
      if (v_hi > n_el - 1) v_hi = n_el - 1;
      full = (hi >= pi / 2) || (lo <= -pi / 2);
      if (!full) {
        const double dalpha = 2.0 * pi / n_az;
        const double ac = atan2(ey, ex);
        const double da = asin(fmin(sin(theta) / cos(bc), 1.0));
        u_lo = (long)ceil((ac - da) / dalpha - 0.5);
        u_hi = (long)floor((ac + da) / dalpha - 0.5);
        if (u_hi - u_lo + 1 >= n_az) full = true;
      }
      if (full) { u_lo = 0; u_hi = n_az - 1; }
    }
    visible = (v_lo <= v_hi) && (full || u_hi >= u_lo);
    if (visible) {
      if (u_lo < 0) { u_lo += n_az; u_hi += n_az; }
      long tu0 = u_lo / tw;
      long ntu = (u_hi < n_az) ? (u_hi / tw - tu0 + 1) : ((nta - tu0) + (u_hi - n_az) / tw + 1);
      if (ntu >= nta) { tu0 = 0; ntu = nta; }
      const long tv0 = v_lo / th;
      const long ntv = v_hi / th - tv0 + 1;
      rect = make_ushort4((unsigned short)tu0, (unsigned short)ntu, (unsigned short)tv0, (unsigned short)ntv);
      cnt = (uint32_t)(ntu * ntv);
    }
  }
  rec_rect[r] = rect;
  rec_cnt[r] = cnt;
}
#pragma clang fp contract(on)

// ---------------------------------------------------------------------------
// Exclusive scans (three phases: per-block reduce, single-block scan of the
// block sums, per-block scan with the block offset).
// ---------------------------------------------------------------------------
template <typename T>
__device__ T block_excl_scan(T v, T *sh, T *total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    T x = tid >= off ? sh[tid - off] : (T)0;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  T incl = sh[tid];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

template <typename TO>
__global__ void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n, TO *__restrict__ tmp) {
  __shared__ TO sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TO s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += (TO)in[base + i];
  TO tot;
  block_excl_scan<TO>(s, sh, &tot);
  if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

// Single block: in-place exclusive scan of tmp[0..nb).  Writes the total to
// *total and, if it exceeds cap, also to *flag (else 0).
template <typename TO>
__global__ void k_scan_top(TO *__restrict__ tmp, int32_t nb, int64_t *__restrict__ total, int64_t cap,
                           int64_t *__restrict__ flag) {
  __shared__ TO sh[kScanThreads];
  const int per = (nb + kScanThreads - 1) / kScanThreads;
  const int lo = threadIdx.x * per, hi = min(nb, lo + per);
  TO s = 0;
  for (int i = lo; i < hi; ++i) s += tmp[i];
  TO tot;
  TO run = block_excl_scan<TO>(s, sh, &tot);
  for (int i = lo; i < hi; ++i) {
    TO x = tmp[i];
    tmp[i] = run;
    run += x;
  }
  if (threadIdx.x == 0) {
    if (total) *total = (int64_t)tot;
    if (flag) *flag = ((int64_t)tot > cap) ? (int64_t)tot : 0;
  }
}

template <typename TO>
__global__ void k_scan_down(const uint32_t *__restrict__ in, int64_t n, const TO *__restrict__ tmp,
                            TO *__restrict__ out) {
  __shared__ TO sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TO v[kScanItems];
  TO s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? (TO)in[base + i] : (TO)0;
    s += v[i];
  }
  TO tot;
  TO run = block_excl_scan<TO>(s, sh, &tot) + tmp[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

hipError_t scan_u32_to_i64(const uint32_t *in, int64_t n, int64_t *out, int64_t *tmp, int32_t nblocks,
                           int64_t *total, int64_t cap, int64_t *flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_reduce<int64_t>, dim3(nblocks), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_top<int64_t>, dim3(1), dim3(kScanThreads), 0, s, tmp, nblocks, total, cap, flag);
  hipLaunchKernelGGL(k_scan_down<int64_t>, dim3(nblocks), dim3(kScanThreads), 0, s, in, n, tmp, out);
  return hipGetLastError();
}

hipError_t scan_u32_to_u32(const uint32_t *in, int64_t n, uint32_t *out, uint32_t *tmp, int32_t nblocks,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_reduce<uint32_t>, dim3(nblocks), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_top<uint32_t>, dim3(1), dim3(kScanThreads), 0, s, tmp, nblocks,
                     (int64_t *)nullptr, (int64_t)0, (int64_t *)nullptr);
  hipLaunchKernelGGL(k_scan_down<uint32_t>, dim3(nblocks), dim3(kScanThreads), 0, s, in, n, tmp, out);
  return hipGetLastError();
}

__global__ void k_zero_counters(int64_t *c) {
  if (threadIdx.x < 4) c[threadIdx.x] = 0;
}

hipError_t launch_project(const gsrf_problem *p, const Layout &lay, char *ws, hipStream_t s) {
  float *prep = (float *)(ws + lay.prep);
  int64_t *rec_base = (int64_t *)(ws + lay.rec_base);
  int64_t *counters = (int64_t *)(ws + lay.counters);
  if (p->n_gauss > 0) {
    hipLaunchKernelGGL(k_activate, dim3((unsigned)((p->n_gauss + 255) / 256)), dim3(256), 0, s, p->means,
                       p->log_scales, p->quats, p->opacity_logits, p->n_gauss, prep);
  }
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, counters);
  if (p->n_pairs > 0) {
    hipLaunchKernelGGL(k_rec_base, dim3(1), dim3(1024), 0, s, p->pairs, p->scene_offsets_dev, p->n_pairs,
                       rec_base);
  }
  if (lay.n_records > 0) {
    dim3 grid((unsigned)((lay.max_scene + 255) / 256), (unsigned)p->n_pairs);
    hipLaunchKernelGGL(k_project, grid, dim3(256), 0, s, p->pairs, p->scene_offsets_dev, rec_base, p->means,
                       p->log_scales, p->grid, lay.nta, (uint32_t *)(ws + lay.rec_key),
                       (ushort4 *)(ws + lay.rec_rect), (uint32_t *)(ws + lay.rec_cnt));
    hipError_t e = scan_u32_to_i64((const uint32_t *)(ws + lay.rec_cnt), lay.n_records,
                                   (int64_t *)(ws + lay.rec_off), (int64_t *)(ws + lay.scan_tmp),
                                   lay.n_rec_blocks, counters + 0, lay.cap, counters + 1, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace gsrf
