// Adaptive density control (App. number of Gaussian updating; the parameter
// table gives eps_mu = 0.0002, eps_r = 10, eps_rho = 0.004, phi = 1.6): the
// per-Gaussian mean-gradient statistics of a window of iterations, and one
// pass that clones, splits and prunes with a stable compaction.
#include <math.h>

#include "gsrf_internal.h"

namespace gsrf {

// acc += dL/dmu (one FP32 add per component), count += 1 where the gradient is
// not zero (the Gaussian was hit in this iteration).
__global__ void k_grad_accum(const float *__restrict__ d_means, int64_t n, float *__restrict__ acc,
                             int32_t *__restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gx = d_means[3 * i], gy = d_means[3 * i + 1], gz = d_means[3 * i + 2];
  acc[3 * i] = acc[3 * i] + gx;
  acc[3 * i + 1] = acc[3 * i + 1] + gy;
  acc[3 * i + 2] = acc[3 * i + 2] + gz;
  if (gx != 0.f || gy != 0.f || gz != 0.f) cnt[i] += 1;
}

hipError_t launch_grad_accum(int64_t n, const float *d_means, float *acc, int32_t *cnt, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_accum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_means, n, acc, cnt);
  return hipGetLastError();
}

enum DcAction { kDcPrune = 0, kDcKeep = 1, kDcClone = 2, kDcSplit = 3 };
constexpr int kDcThreads = 256, kDcPer = 4, kDcBlock = kDcThreads * kDcPer;

struct DcArgs {
  const float *means, *log_scales, *quats, *logits, *coeffs, *acc, *z;
  const int32_t *cnt;
  int64_t n;
  int k2;                          // floats per coefficient row (2K)
  double eps_mu, eps_r, eps_rho, clone_step;
  float ln_phi;
  int densify, prune;
  float *o_means, *o_log_scales, *o_quats, *o_logits, *o_coeffs, *o_acc;
  int32_t *o_cnt;
  int64_t *blk;                    // per-block output counts, then their exclusive scan
  int64_t *counts;                 // n_out, clones, splits, pruned
};

// The action for Gaussian i; every discrete decision is taken in FP64.
__device__ int dc_action(const DcArgs &a, int64_t i) {
  if (a.prune && 1.0 / (1.0 + exp(-(double)a.logits[i])) < a.eps_rho) return kDcPrune;
  const int n = a.cnt[i];
  if (!a.densify || n <= 0) return kDcKeep;
  const double ax = a.acc[3 * i], ay = a.acc[3 * i + 1], az = a.acc[3 * i + 2];
  const double en = a.eps_mu * (double)n;
  if (!((ax * ax + ay * ay) + az * az > en * en)) return kDcKeep;    // |sum g| / n > eps_mu
  // radius: the mean of the diagonal of R S S^T R^T, which is the mean of s_k^2
  double r = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double sk = exp((double)a.log_scales[3 * i + k]);
    r += sk * sk;
  }
  return (r / 3.0 > a.eps_r) ? kDcSplit : kDcClone;
}

__device__ __forceinline__ int dc_outputs(int act) { return act == kDcPrune ? 0 : (act == kDcKeep ? 1 : 2); }

// Output counts per block of kDcBlock Gaussians.
__global__ void __launch_bounds__(kDcThreads) k_dc_count(DcArgs a) {
  __shared__ int64_t part[kDcThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kDcBlock + (int64_t)threadIdx.x * kDcPer;
  int64_t c = 0;
  for (int j = 0; j < kDcPer; ++j)
    if (base + j < a.n) c += dc_outputs(dc_action(a, base + j));
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kDcThreads / 64; ++w) t += part[w];
    a.blk[blockIdx.x] = t;
  }
}

// Exclusive scan of the block counts (one workgroup, chunks of 1024 with a
// carry); counts[0] = total, counts[1..3] cleared for the apply pass.
__global__ void __launch_bounds__(1024) k_dc_scan(int64_t *__restrict__ blk, int64_t nb, int64_t *__restrict__ counts) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
    const int64_t i = c0 + tid;
    const int64_t v = i < nb ? blk[i] : 0;
    int64_t x = v;                                   // inclusive scan within the wave
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t before = carry;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (i < nb) blk[i] = before + x - v;
    __syncthreads();
    if (tid == 1023) carry = before + x;
    __syncthreads();
  }
  if (tid == 0) {
    counts[0] = carry;
    counts[1] = counts[2] = counts[3] = 0;
  }
}

__device__ void dc_copy(const DcArgs &a, int64_t i, int64_t o) {
  for (int k = 0; k < 3; ++k) {
    a.o_means[3 * o + k] = a.means[3 * i + k];
    a.o_log_scales[3 * o + k] = a.log_scales[3 * i + k];
    a.o_acc[3 * o + k] = 0.f;
  }
  for (int k = 0; k < 4; ++k) a.o_quats[4 * o + k] = a.quats[4 * i + k];
  a.o_logits[o] = a.logits[i];
  for (int k = 0; k < a.k2; ++k) a.o_coeffs[(int64_t)a.k2 * o + k] = a.coeffs[(int64_t)a.k2 * i + k];
  a.o_cnt[o] = 0;
}

// Writes the survivors of each block's Gaussians at the scanned offsets, in
// index order (a clone's original before its copy, a split's first child
// before its second).
__global__ void __launch_bounds__(kDcThreads) k_dc_apply(DcArgs a) {
  __shared__ int64_t wsum[kDcThreads / 64];
  __shared__ int stat[3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < 3) stat[tid] = 0;
  const int64_t base = (int64_t)blockIdx.x * kDcBlock + (int64_t)tid * kDcPer;
  int act[kDcPer];
  int64_t c = 0;
  for (int j = 0; j < kDcPer; ++j) {
    act[j] = base + j < a.n ? dc_action(a, base + j) : kDcPrune;
    c += dc_outputs(act[j]);
  }
  int64_t x = c;
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int64_t o = a.blk[blockIdx.x] + x - c;
  for (int w = 0; w < wave; ++w) o += wsum[w];
  int n_clone = 0, n_split = 0, n_prune = 0;
  for (int j = 0; j < kDcPer; ++j) {
    const int64_t i = base + j;
    if (i >= a.n) break;
    if (act[j] == kDcPrune) {
      ++n_prune;
      continue;
    }
    dc_copy(a, i, o);
    if (act[j] == kDcClone) {
      ++n_clone;
      dc_copy(a, i, o + 1);
      const double inv = (double)a.cnt[i];
      for (int k = 0; k < 3; ++k)
        a.o_means[3 * (o + 1) + k] =
            (float)((double)a.means[3 * i + k] - a.clone_step * ((double)a.acc[3 * i + k] / inv));
    } else if (act[j] == kDcSplit) {
      ++n_split;
      dc_copy(a, i, o + 1);
      double qw = a.quats[4 * i], qx = a.quats[4 * i + 1], qy = a.quats[4 * i + 2], qz = a.quats[4 * i + 3];
      const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
      qw /= qn; qx /= qn; qy /= qn; qz /= qn;
      const double R[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                              {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
                              {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
      double sv[3];
      for (int k = 0; k < 3; ++k) sv[k] = exp((double)a.log_scales[3 * i + k]);
      for (int ch = 0; ch < 2; ++ch) {
        const float *zz = a.z + 6 * i + 3 * ch;
        const double w0 = sv[0] * zz[0], w1 = sv[1] * zz[1], w2 = sv[2] * zz[2];
        for (int k = 0; k < 3; ++k) {
          a.o_means[3 * (o + ch) + k] = (float)((double)a.means[3 * i + k] + (R[k][0] * w0 + R[k][1] * w1 + R[k][2] * w2));
          a.o_log_scales[3 * (o + ch) + k] = a.log_scales[3 * i + k] - a.ln_phi;
        }
      }
    }
    o += dc_outputs(act[j]);
  }
  if (n_clone) atomicAdd(&stat[0], n_clone);
  if (n_split) atomicAdd(&stat[1], n_split);
  if (n_prune) atomicAdd(&stat[2], n_prune);
  __syncthreads();
  if (tid < 3 && stat[tid]) atomicAdd((unsigned long long *)&a.counts[1 + tid], (unsigned long long)stat[tid]);
}

size_t density_workspace_bytes(int64_t n) { return (size_t)((n + kDcBlock - 1) / kDcBlock + 1) * sizeof(int64_t); }

hipError_t launch_density_control(const DensityIO &io, hipStream_t s) {
  DcArgs a{};
  a.means = io.means; a.log_scales = io.log_scales; a.quats = io.quats; a.logits = io.logits; a.coeffs = io.coeffs;
  a.acc = io.acc; a.cnt = io.cnt; a.z = io.z;
  a.n = io.n; a.k2 = 2 * io.K;
  a.eps_mu = io.eps_mu; a.eps_r = io.eps_r; a.eps_rho = io.eps_rho; a.clone_step = io.clone_step;
  a.ln_phi = io.ln_phi; a.densify = io.densify; a.prune = io.prune;
  a.o_means = io.o_means; a.o_log_scales = io.o_log_scales; a.o_quats = io.o_quats; a.o_logits = io.o_logits;
  a.o_coeffs = io.o_coeffs; a.o_acc = io.o_acc; a.o_cnt = io.o_cnt;
  a.blk = (int64_t *)io.ws;
  a.counts = io.counts;
  const int64_t nb = (io.n + kDcBlock - 1) / kDcBlock;
  if (nb > 0) {
    hipLaunchKernelGGL(k_dc_count, dim3((unsigned)nb), dim3(kDcThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_dc_scan, dim3(1), dim3(1024), 0, s, a.blk, nb, a.counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 0) return e;
  hipLaunchKernelGGL(k_dc_apply, dim3((unsigned)nb), dim3(kDcThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace gsrf
