// The steps either side of the render in a training iteration: the
// antenna-array spectrum loss and its gradient, the single-antenna losses
// (Sec. 3.4 loss function) and the per-attribute SGD update (App. Gaussian
// primitive optimization, eq. updating).
#include <math.h>

#include <mutex>

#include "gsrf_internal.h"

namespace gsrf {

// SSIM window and constants (the 3D Gaussian splatting convention: 11 x 11
// Gaussian window, sigma 1.5, zero padding, C1 = 0.01^2, C2 = 0.03^2).
constexpr int kWin = 11, kRad = 5;
constexpr float kSsimC1 = 1e-4f, kSsimC2 = 9e-4f;

// Output tile of one workgroup: TH x TW pixels.  The SSIM map at a pixel needs
// the image within kRad of it and its gradient needs the map's derivatives
// within kRad again, so a workgroup reads the tile widened by 2 kRad.
constexpr int kLossTH = 16, kLossTW = 32, kLossThreads = 256;
constexpr int kRH = kLossTH + 4 * kRad, kRW = kLossTW + 4 * kRad;   // input region (36 x 52)
constexpr int kMH = kLossTH + 2 * kRad, kMW = kLossTW + 2 * kRad;   // statistics region (26 x 42)

struct LossLds {
  float w[kWin];
  float x[kRH][kRW];             // prediction: power |S|^2 (0 outside the image)
  float y[kRH][kRW];             // target
  union {
    float h5[5][kRH][kMW];       // horizontal blur of x, y, x^2, y^2, xy
    float h3[3][kMH][kLossTW];   // horizontal blur of the derivative maps
  };
  float d[3][kMH][kMW];          // dSSIM/dmu_x, dSSIM/dE[x^2], dSSIM/dE[xy] per statistics point
  double red[3][kLossThreads / 64];
};

// One workgroup per (pair, output tile): the tile's sums of |x - y|, SSIM and
// (x - y)^2 into partials[(k * tiles + t) * 3 + {0,1,2}] (FP64), and, when
// grad is non-NULL, dL/dRe S + j dL/dIm S of its pixels; x = pscale |S|^2.
//
// L = (1 - l1 - l2) mean|x - y| + l1 (1 - mean SSIM) + l2 L_F.  With the
// unnormalised DFT, Parseval's identity makes the Fourier term
// (1/N) sum_f |F(x - y)|^2 = sum_uv (x - y)^2, so it needs no transform.
// SSIM's gradient: s(p) depends on x through mu_x = w * x, E[x^2] = w * x^2
// and E[xy] = w * (x y); with d1 = ds/dmu_x, d2 = ds/dE[x^2], d3 = ds/dE[xy]
// (mu_x's own part of the variance terms folded into d1),
// d mean(s) / dx(q) = (1/N) [(w * d1)(q) + 2 x(q) (w * d2)(q) + y(q) (w * d3)(q)]
// (w symmetric, zero outside the image).
__global__ void __launch_bounds__(kLossThreads)
k_spectrum_loss(const float2 *__restrict__ signal, const float *__restrict__ target, int n_el, int n_az,
                int tiles_az, int tiles, float pscale, float lam1, float lam2, double *__restrict__ partials,
                float2 *__restrict__ grad) {
  __shared__ LossLds L;
  const int tid = threadIdx.x;
  const int k = blockIdx.y;
  const int t = blockIdx.x;
  const int v0 = (t / tiles_az) * kLossTH, u0 = (t % tiles_az) * kLossTW;
  const size_t img = (size_t)k * n_el * n_az;
  const float inv_n = 1.0f / (float)((int64_t)n_el * n_az);

  if (tid < kWin) {
    double sum = 0.0, mine = 0.0;
    for (int i = 0; i < kWin; ++i) {
      const double r = (double)(i - kRad), e = exp(-(r * r) / 4.5);
      sum += e;
      if (i == tid) mine = e;
    }
    L.w[tid] = (float)(mine / sum);
  }
  for (int i = tid; i < kRH * kRW; i += kLossThreads) {
    const int a = i / kRW, b = i % kRW;
    const int v = v0 - 2 * kRad + a, u = u0 - 2 * kRad + b;
    float xv = 0.f, yv = 0.f;
    if (v >= 0 && v < n_el && u >= 0 && u < n_az) {
      const float2 s = signal[img + (size_t)v * n_az + u];
      xv = pscale * fmaf(s.x, s.x, s.y * s.y);
      yv = target[img + (size_t)v * n_az + u];
    }
    L.x[a][b] = xv;
    L.y[a][b] = yv;
  }
  __syncthreads();
  float w[kWin];
#pragma unroll
  for (int i = 0; i < kWin; ++i) w[i] = L.w[i];

  for (int i = tid; i < kRH * kMW; i += kLossThreads) {     // horizontal pass, five statistics
    const int a = i / kMW, c = i % kMW;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
    for (int q = 0; q < kWin; ++q) {
      const float xv = L.x[a][c + q], yv = L.y[a][c + q];
      s0 = fmaf(w[q], xv, s0);
      s1 = fmaf(w[q], yv, s1);
      s2 = fmaf(w[q], xv * xv, s2);
      s3 = fmaf(w[q], yv * yv, s3);
      s4 = fmaf(w[q], xv * yv, s4);
    }
    L.h5[0][a][c] = s0;
    L.h5[1][a][c] = s1;
    L.h5[2][a][c] = s2;
    L.h5[3][a][c] = s3;
    L.h5[4][a][c] = s4;
  }
  __syncthreads();
  double ssim_sum = 0.0;
  for (int i = tid; i < kMH * kMW; i += kLossThreads) {     // vertical pass, SSIM and its derivatives
    const int r = i / kMW, c = i % kMW;
    const int v = v0 - kRad + r, u = u0 - kRad + c;
    float d1 = 0.f, d2 = 0.f, d3 = 0.f;
    if (v >= 0 && v < n_el && u >= 0 && u < n_az) {
      float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
      for (int q = 0; q < kWin; ++q) {
        mx = fmaf(w[q], L.h5[0][r + q][c], mx);
        my = fmaf(w[q], L.h5[1][r + q][c], my);
        exx = fmaf(w[q], L.h5[2][r + q][c], exx);
        eyy = fmaf(w[q], L.h5[3][r + q][c], eyy);
        exy = fmaf(w[q], L.h5[4][r + q][c], exy);
      }
      const float n1 = 2.f * mx * my + kSsimC1, n2 = 2.f * (exy - mx * my) + kSsimC2;
      const float e1 = mx * mx + my * my + kSsimC1, e2 = (exx - mx * mx) + (eyy - my * my) + kSsimC2;
      const float s = (n1 * n2) / (e1 * e2);
      if (r >= kRad && r < kRad + kLossTH && c >= kRad && c < kRad + kLossTW) ssim_sum += (double)s;
      d1 = s * (2.f * my / n1 - 2.f * my / n2 - 2.f * mx / e1 + 2.f * mx / e2);
      d2 = -s / e2;
      d3 = 2.f * s / n2;
    }
    L.d[0][r][c] = d1;
    L.d[1][r][c] = d2;
    L.d[2][r][c] = d3;
  }
  __syncthreads();
  if (grad) {
    for (int i = tid; i < kMH * kLossTW; i += kLossThreads) {   // horizontal blur of the derivative maps
      const int r = i / kLossTW, j = i % kLossTW;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int q = 0; q < kWin; ++q) {
        s0 = fmaf(w[q], L.d[0][r][j + q], s0);
        s1 = fmaf(w[q], L.d[1][r][j + q], s1);
        s2 = fmaf(w[q], L.d[2][r][j + q], s2);
      }
      L.h3[0][r][j] = s0;
      L.h3[1][r][j] = s1;
      L.h3[2][r][j] = s2;
    }
    __syncthreads();
  }
  double l1_sum = 0.0, f_sum = 0.0;
  const float c_l1 = (1.f - lam1 - lam2) * inv_n, c_ssim = -lam1 * inv_n, c_f = 2.f * lam2;
  for (int i = tid; i < kLossTH * kLossTW; i += kLossThreads) {
    const int r = i / kLossTW, j = i % kLossTW;
    const int v = v0 + r, u = u0 + j;
    if (v >= n_el || u >= n_az) continue;
    const float xv = L.x[r + 2 * kRad][j + 2 * kRad], yv = L.y[r + 2 * kRad][j + 2 * kRad];
    const float dxy = xv - yv;
    l1_sum += (double)fabsf(dxy);
    f_sum += (double)dxy * (double)dxy;
    if (grad) {
      float b1 = 0.f, b2 = 0.f, b3 = 0.f;
#pragma unroll
      for (int q = 0; q < kWin; ++q) {
        b1 = fmaf(w[q], L.h3[0][r + q][j], b1);
        b2 = fmaf(w[q], L.h3[1][r + q][j], b2);
        b3 = fmaf(w[q], L.h3[2][r + q][j], b3);
      }
      const float sgn = dxy > 0.f ? 1.f : (dxy < 0.f ? -1.f : 0.f);
      const float dldx = c_l1 * sgn + c_ssim * (b1 + 2.f * xv * b2 + yv * b3) + c_f * dxy;
      const float2 s = signal[img + (size_t)v * n_az + u];
      const float c = 2.f * pscale * dldx;
      grad[img + (size_t)v * n_az + u] = make_float2(c * s.x, c * s.y);
    }
  }
  // fixed-order block reduction of the three sums
  const int lane = tid & 63, wave = tid >> 6;
  double vals[3] = {l1_sum, ssim_sum, f_sum};
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double x = vals[m];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    if (lane == 0) L.red[m][wave] = x;
  }
  __syncthreads();
  if (tid < 3) {
    double x = 0.0;
    for (int i = 0; i < kLossThreads / 64; ++i) x += L.red[tid][i];
    partials[((size_t)k * tiles + t) * 3 + tid] = x;
  }
}

// Per pair: the tile partials summed in tile order (one wave), then
// loss[k] = (total, L1, L_SSIM, L_Fourier).
__global__ void __launch_bounds__(64)
k_loss_final(const double *__restrict__ partials, int tiles, double n_pix, float lam1, float lam2,
             float *__restrict__ loss) {
  const int k = blockIdx.x, lane = threadIdx.x;
  double s[3] = {0.0, 0.0, 0.0};
  for (int t = lane; t < tiles; t += 64)
#pragma unroll
    for (int m = 0; m < 3; ++m) s[m] += partials[((size_t)k * tiles + t) * 3 + m];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s[m] += __shfl_xor(s[m], d, 64);
  if (lane == 0) {
    const double l1 = s[0] / n_pix, ls = 1.0 - s[1] / n_pix, lf = s[2];
    const double tot = (1.0 - (double)lam1 - (double)lam2) * l1 + (double)lam1 * ls + (double)lam2 * lf;
    loss[4 * k + 0] = (float)tot;
    loss[4 * k + 1] = (float)l1;
    loss[4 * k + 2] = (float)ls;
    loss[4 * k + 3] = (float)lf;
  }
}

// Scratch of gsrf_loss_spectrum_noalloc: the per-tile FP64 partial sums that
// gsrf_loss_spectrum keeps in its caller's workspace, here in a fixed device
// array (one copy per GPU, held until the process ends).  In host code the
// array's name is a host-side stand-in, so kernels receive the address that
// hipGetSymbolAddress reports for the current device, looked up once per
// device.  k_spectrum_loss writes every partial it covers before
// k_loss_final reads it, so nothing has to start at zero.
constexpr size_t kLossScratchBytes = (size_t)1 << 20;
static __device__ __align__(256) double scratch[kLossScratchBytes / sizeof(double)];

size_t loss_scratch_bytes() { return kLossScratchBytes; }

hipError_t loss_scratch_address(hipStream_t s, void **out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (s) {
    int sdev = -1;
    e = hipStreamGetDevice(s, &sdev);
    if (e != hipSuccess) return e;
    if (sdev != dev) return hipErrorInvalidDevice;   // the scratch looked up must be the stream's GPU's
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

size_t loss_partials_bytes(int32_t n_pairs, int32_t n_el, int32_t n_az) {
  const size_t tiles = (size_t)((n_el + kLossTH - 1) / kLossTH) * ((n_az + kLossTW - 1) / kLossTW);
  return (size_t)n_pairs * tiles * 3 * sizeof(double);
}

hipError_t launch_loss_spectrum(const float *signal, const float *target, int32_t n_pairs, int32_t n_el, int32_t n_az,
                                float pscale, float lam1, float lam2, float *loss, float *grad_signal, void *ws,
                                hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  const int tiles_az = (n_az + kLossTW - 1) / kLossTW, tiles = tiles_az * ((n_el + kLossTH - 1) / kLossTH);
  double *partials = (double *)ws;
  hipLaunchKernelGGL(k_spectrum_loss, dim3((unsigned)tiles, (unsigned)n_pairs), dim3(kLossThreads), 0, s,
                     (const float2 *)signal, target, n_el, n_az, tiles_az, tiles, pscale, lam1, lam2, partials,
                     (float2 *)grad_signal);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_final, dim3((unsigned)n_pairs), dim3(64), 0, s, (const double *)partials, tiles,
                     (double)n_el * (double)n_az, lam1, lam2, loss);
  return hipGetLastError();
}

// Single antenna (Sec. 3.4): one thread per pair.  kind GSRF_LOSS_RSSI_DB:
// |10 log10 |S|^2 - t| against an RSSI t in dBm, gradient
// sign * (20 / ln 10) * S / |S|^2 (0 where S = 0, whose loss is +inf);
// kind GSRF_LOSS_COMPLEX_L2: |S - t|^2, gradient 2 (S - t).
__global__ void k_loss_single(const float2 *__restrict__ ssum, const float *__restrict__ target, int n_pairs,
                              int kind, float *__restrict__ loss, float2 *__restrict__ grad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pairs) return;
  const double sr = ssum[k].x, si = ssum[k].y;
  double l, gr, gi;
  if (kind == GSRF_LOSS_RSSI_DB) {
    const double p = sr * sr + si * si;
    if (p > 0.0) {
      const double d = 10.0 * log10(p) - (double)target[k];
      const double c = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) * (20.0 / log(10.0)) / p;
      l = fabs(d);
      gr = c * sr;
      gi = c * si;
    } else {
      l = HUGE_VAL;
      gr = gi = 0.0;
    }
  } else {
    const double dr = sr - (double)target[2 * k], di = si - (double)target[2 * k + 1];
    l = dr * dr + di * di;
    gr = 2.0 * dr;
    gi = 2.0 * di;
  }
  loss[k] = (float)l;
  if (grad) grad[k] = make_float2((float)gr, (float)gi);
}

hipError_t launch_loss_single(const float *signal_sum, const float *target, int32_t n_pairs, int32_t kind,
                              float *loss, float *grad_sum, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_loss_single, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, s,
                     (const float2 *)signal_sum, target, n_pairs, kind, loss, (float2 *)grad_sum);
  return hipGetLastError();
}

// SGD on every attribute in one launch (App. attribute updating):
// w <- fma(-eta, g, w), one rounding.  Segment y of the grid is attribute y.
struct SgdSeg {
  float *w[5];
  const float *g[5];
  int64_t n[5];
  float eta[5];
};

__global__ void __launch_bounds__(256) k_sgd(SgdSeg seg) {
  const int a = blockIdx.y;
  float *__restrict__ w = seg.w[a];
  const float *__restrict__ g = seg.g[a];
  const int64_t n = seg.n[a];
  const float eta = seg.eta[a];
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  int64_t done = 0;
  if ((((uintptr_t)w | (uintptr_t)g) & 15) == 0) {   // 16-byte vectors where both arrays allow them
    float4 *__restrict__ w4 = (float4 *)w;
    const float4 *__restrict__ g4 = (const float4 *)g;
    const int64_t n4 = n >> 2;
    for (int64_t i = first; i < n4; i += stride) {
      float4 x = w4[i];
      const float4 d = g4[i];
      x.x = fmaf(-eta, d.x, x.x);
      x.y = fmaf(-eta, d.y, x.y);
      x.z = fmaf(-eta, d.z, x.z);
      x.w = fmaf(-eta, d.w, x.w);
      w4[i] = x;
    }
    done = n4 << 2;
  }
  for (int64_t i = done + first; i < n; i += stride) w[i] = fmaf(-eta, g[i], w[i]);
}

hipError_t launch_sgd(int64_t n_gauss, int K, float *const w[5], const float *const g[5], const float eta[5],
                      hipStream_t s) {
  if (n_gauss == 0) return hipSuccess;
  SgdSeg seg;
  const int64_t per[5] = {3, 3, 4, 1, 2 * (int64_t)K};
  int64_t most = 0;
  for (int a = 0; a < 5; ++a) {
    seg.w[a] = w[a];
    seg.g[a] = g[a];
    seg.n[a] = n_gauss * per[a];
    seg.eta[a] = eta[a];
    if (seg.n[a] > most) most = seg.n[a];
  }
  const int64_t blocks = (most / 4 + 255) / 256 + 1;
  hipLaunchKernelGGL(k_sgd, dim3((unsigned)(blocks < 8192 ? blocks : 8192), 5), dim3(256), 0, s, seg);
  return hipGetLastError();
}

}  // namespace gsrf
