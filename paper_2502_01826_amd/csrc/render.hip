// Steps a5-a8: complex front-to-back ray accumulation (Sec. 3.4 eq. rendering;
// App. A; Alg. 1 Blend), the single-antenna sum (Sec. 3.4), the adjoint
// (App. C backward kernel; App. D) and the per-Gaussian chain rule through
// Sigma^-1 = R diag(s^-2) R^T (the covariance gradient App. D.3 omits).
//
// One workgroup renders one (pair, tile): one thread per ray, the tile's
// depth-sorted Gaussian list staged through LDS in batches.  Per staged
// Gaussian the receiver-relative geometry is formed once in FP64 (distance D,
// unit direction e as an FP32 hi+lo pair, base phase frac((|mu-tx| + D)/lambda));
// per (ray, Gaussian) everything is FP32 in the Gaussian's local frame:
//   eps = v - e,  w = M v,  A = v.w,  b = eps.w,  c = eps^T M eps,
//   Q = D^2 (c - b^2/A)  (= C - B^2/A, the Mahalanobis^2 at the chord midpoint)
//   t = D (1 - b/A)      (= -B/A, the chord midpoint)
// which avoids the cancellation of C - B^2/A at D ~ 10 m and keeps the phase
// accurate: phase/(2 pi) = frac((|mu-tx| + D)/lambda) - (D/lambda) (b/A).
#include "gsrf_internal.h"

namespace gsrf {

struct RenderArgs {
  const gsrf_pair *pairs;
  const float *prep;        // [G][kPrep]
  const float *coeffs;      // [G][K][2]
  const uint32_t *val;      // sorted Gaussian ids
  const uint32_t *tstart;   // [P*T]
  const uint32_t *tend;     // [P*T]
  int32_t T, nta, n_az, n_el, tw;
  float el_lo, el_hi, r_rx, t_min, amax;
};

// Geometry record per staged Gaussian: five float4
//   g0 = (e_hi, D)  g1 = (e_lo, D/lambda)  g2 = (M00, M11, M22, M01)
//   g3 = (M02, M12, N, o)  g4 = (phase0, D^2, 0, 0)
constexpr int kGeo = 5;

constexpr int lds_batch(int L, int NT, bool bwd) {
  // floats per staged entry: geometry + coefficients (+ accumulators for bwd)
  int K = (L + 1) * (L + 1);
  int per = 4 * kGeo + 2 * K + (bwd ? (12 + 2 * K) + 1 : 0);
  int budget = 60 * 1024 / 4;
  int b = NT;
  while (b > 32 && b * per > budget) b >>= 1;
  return b;
}

// ---------------------------------------------------------------------------
// Per-ray setup: direction (FP64 -> FP32) and the FLE basis
// Y_i = e^{j m alpha} P_l^m(sin beta), i = l^2 + l + m (Sec. 3.2 eq. FLE).
// ---------------------------------------------------------------------------
template <int L>
__device__ void ray_setup(int u, int v, const RenderArgs &a, float &vx, float &vy, float &vz, float *Yr,
                          float *Yi) {
  const double pi = 3.14159265358979323846;
  const double al = 2.0 * pi * (u + 0.5) / a.n_az;
  const double be = (double)a.el_lo + ((double)a.el_hi - (double)a.el_lo) * (v + 0.5) / a.n_el;
  const double cb = cos(be), sb = sin(be);
  vx = (float)(cb * cos(al));
  vy = (float)(cb * sin(al));
  vz = (float)sb;
  // associated Legendre P_l^m(x), m >= 0, Condon-Shortley phase, textbook recurrences
  double P[L + 1][L + 1];
  const double x = sb;
  const double s = sqrt(fmax(0.0, 1.0 - x * x));
  double pmm = 1.0;
#pragma unroll
  for (int m = 0; m <= L; ++m) {
    if (m > 0) pmm = -pmm * (2 * m - 1) * s;
    P[m][m] = pmm;
    if (m + 1 <= L) P[m + 1][m] = x * (2 * m + 1) * pmm;
#pragma unroll
    for (int l = m + 2; l <= L; ++l) P[l][m] = ((2 * l - 1) * x * P[l - 1][m] - (l + m - 1) * P[l - 2][m]) / (l - m);
  }
#pragma unroll
  for (int l = 0; l <= L; ++l) {
#pragma unroll
    for (int m = 0; m <= l; ++m) {
      const double c = cos(m * al), sn = sin(m * al);
      const double pl = P[l][m];
      Yr[l * l + l + m] = (float)(pl * c);
      Yi[l * l + l + m] = (float)(pl * sn);
      if (m > 0) {
        double f = 1.0;  // (l+m)! / (l-m)!
        for (int t = l - m + 1; t <= l + m; ++t) f *= t;
        const double pn = ((m & 1) ? -pl : pl) / f;   // P_l^{-m}
        Yr[l * l + l - m] = (float)(pn * c);
        Yi[l * l + l - m] = (float)(-pn * sn);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Stage list entry `idx` of the tile into LDS slot `slot` (FP64 geometry).
// ---------------------------------------------------------------------------
template <int K>
__device__ void stage_entry(const RenderArgs &a, uint32_t g, double rx, double ry, double rz, double tx,
                            double ty, double tz, double lam, float4 *geo, float *cf) {
  const float *pg = a.prep + (size_t)kPrep * g;
  const double mx = pg[0], my = pg[1], mz = pg[2];
  const double ex = mx - rx, ey = my - ry, ez = mz - rz;
  const double D2 = (ex * ex + ey * ey) + ez * ez;
  const double D = sqrt(D2);
  const double inv = D > 0.0 ? 1.0 / D : 0.0;
  const double e0 = ex * inv, e1 = ey * inv, e2 = ez * inv;
  const float h0 = (float)e0, h1 = (float)e1, h2 = (float)e2;
  const double qx = mx - tx, qy = my - ty, qz = mz - tz;
  const double dtx = sqrt((qx * qx + qy * qy) + qz * qz);
  const double ph = (dtx + D) / lam;
  geo[0] = make_float4(h0, h1, h2, (float)D);
  geo[1] = make_float4((float)(e0 - (double)h0), (float)(e1 - (double)h1), (float)(e2 - (double)h2), (float)(D / lam));
  // prep record (64-byte aligned): (mu, N) (M00, M11, M22, M01) (M02, M12, o, -)
  const float4 *p4 = (const float4 *)pg;
  const float4 q0 = p4[0], q1 = p4[1], q2 = p4[2];
  geo[2] = q1;
  geo[3] = make_float4(q2.x, q2.y, q0.w, q2.z);
  geo[4] = make_float4((float)(ph - floor(ph)), (float)D2, 0.f, 0.f);
  const float2 *c2 = (const float2 *)(a.coeffs + (size_t)2 * K * g);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const float2 c = c2[i];
    cf[2 * i] = c.x;
    cf[2 * i + 1] = c.y;
  }
}

// sin and cos of 2 pi x (x in revolutions): reduce to |f| <= 1/8 turn, then the
// Taylor series of sin/cos to degree 9/10 (truncation < 2e-9 on |theta| <= pi/4).
__device__ __forceinline__ void sincos_rev(float x, float &sn, float &cs) {
  const float r = x - rintf(x);
  const float q = rintf(4.0f * r);
  const float f = fmaf(-0.25f, q, r);
  const float th = f * 6.28318530717958648f;
  const float t2 = th * th;
  float ps = fmaf(t2, 2.7557319223985893e-6f, -1.9841269841269841e-4f);
  ps = fmaf(t2, ps, 8.3333333333333333e-3f);
  ps = fmaf(t2, ps, -1.6666666666666667e-1f);
  ps = fmaf(t2 * th, ps, th);
  float pc = fmaf(t2, -2.7557319223985891e-7f, 2.4801587301587302e-5f);
  pc = fmaf(t2, pc, -1.3888888888888889e-3f);
  pc = fmaf(t2, pc, 4.1666666666666667e-2f);
  pc = fmaf(t2, pc, -0.5f);
  pc = fmaf(t2, pc, 1.0f);
  const int iq = ((int)q) & 3;
  sn = (iq == 0) ? ps : (iq == 1) ? pc : (iq == 2) ? -ps : -pc;
  cs = (iq == 0) ? pc : (iq == 1) ? -ps : (iq == 2) ? -pc : ps;
}

// Everything one (ray, Gaussian) pair needs; forward and backward call the
// same function so their hit decisions and transmittances agree bit for bit.
struct Terms {
  float ex, ey, ez;     // eps = v - e
  float w0, w1, w2;     // M v
  float m0, m1, m2;     // M eps
  float rA, bA, Q;
  float G, alpha, p;
  float sn, cs;         // sin/cos of the phase
  float pr, pi;         // psi
  float pzr, pzi;       // psi e^{-j phase}
  bool clamped;
};

__device__ __forceinline__ bool test_hit(float vx, float vy, float vz, const float4 *geo, float r_rx, Terms &h) {
  const float4 g0 = geo[0], g1 = geo[1], g2 = geo[2], g3 = geo[3];
  h.ex = (vx - g0.x) - g1.x;
  h.ey = (vy - g0.y) - g1.y;
  h.ez = (vz - g0.z) - g1.z;
  const float m00 = g2.x, m11 = g2.y, m22 = g2.z, m01 = g2.w, m02 = g3.x, m12 = g3.y;
  h.w0 = fmaf(m00, vx, fmaf(m01, vy, m02 * vz));
  h.w1 = fmaf(m01, vx, fmaf(m11, vy, m12 * vz));
  h.w2 = fmaf(m02, vx, fmaf(m12, vy, m22 * vz));
  const float A = fmaf(vx, h.w0, fmaf(vy, h.w1, vz * h.w2));
  const float b = fmaf(h.ex, h.w0, fmaf(h.ey, h.w1, h.ez * h.w2));
  h.m0 = fmaf(m00, h.ex, fmaf(m01, h.ey, m02 * h.ez));
  h.m1 = fmaf(m01, h.ex, fmaf(m11, h.ey, m12 * h.ez));
  h.m2 = fmaf(m02, h.ex, fmaf(m12, h.ey, m22 * h.ez));
  const float c = fmaf(h.ex, h.m0, fmaf(h.ey, h.m1, h.ez * h.m2));
  h.rA = __builtin_amdgcn_rcpf(A);
  h.bA = b * h.rA;
  h.Q = geo[4].y * fmaf(-b, h.bA, c);
  const float t = fmaf(-g0.w, h.bA, g0.w);
  return (h.Q <= kLevel) && (t >= r_rx);
}

template <int K>
__device__ __forceinline__ void hit_terms(const float4 *geo, const float *cf, const float *Yr, const float *Yi,
                                          float amax, Terms &h) {
  const float4 g1 = geo[1], g3 = geo[3], g4 = geo[4];
  h.G = __builtin_amdgcn_exp2f(-0.72134752044448170f * h.Q);   // exp(-Q/2)
  const float oG = g3.w * h.G;
  h.clamped = oG > amax;
  h.alpha = fminf(oG, amax);
  h.p = g3.z * h.G;
  sincos_rev(fmaf(-g1.w, h.bA, g4.x), h.sn, h.cs);
  float pr = 0.f, pi = 0.f;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const float cr = cf[2 * i], ci = cf[2 * i + 1];
    pr = fmaf(cr, Yr[i], fmaf(-ci, Yi[i], pr));
    pi = fmaf(cr, Yi[i], fmaf(ci, Yr[i], pi));
  }
  h.pr = pr;
  h.pi = pi;
  h.pzr = fmaf(pr, h.cs, pi * h.sn);
  h.pzi = fmaf(pi, h.cs, -(pr * h.sn));
}

// ---------------------------------------------------------------------------
// a5: forward render.  grid = P*T workgroups, NT threads (one ray each).
// ---------------------------------------------------------------------------
template <int L, int NT, bool STATS>
__global__ __launch_bounds__(NT) void k_render_fwd(RenderArgs a, float2 *__restrict__ signal,
                                                   float2 *__restrict__ tile_sum,
                                                   unsigned long long *__restrict__ stats) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int B = lds_batch(L, NT, false);
  extern __shared__ float4 smem[];
  float4 *sgeo = smem;                          // [B][kGeo]
  float *scf = (float *)(smem + kGeo * B);      // [B][2K]
  const int gt = blockIdx.x;
  const int k = gt / a.T;
  const int tile = gt - k * a.T;
  const int tv = tile / a.nta, tu = tile - tv * a.nta;
  const int th_ = NT / a.tw;
  const int u = tu * a.tw + (int)threadIdx.x % a.tw;
  const int v = tv * th_ + (int)threadIdx.x / a.tw;
  const bool valid = (u < a.n_az) && (v < a.n_el);
  const gsrf_pair pr = a.pairs[k];
  const double lam = kC0 / pr.freq_hz;
  float vx = 0.f, vy = 0.f, vz = 1.f, Yr[K], Yi[K];
  ray_setup<L>(valid ? u : 0, valid ? v : 0, a, vx, vy, vz, Yr, Yi);
  const uint32_t s0 = a.tstart[gt], s1 = a.tend[gt];
  float T = 1.f, Sr = 0.f, Si = 0.f;
  bool done = !valid || (1.0f < a.t_min);
  unsigned long long n_test = 0, n_hit = 0, n_staged = 0;
  for (uint32_t base = s0; base < s1; base += B) {
    const int nb = (int)min((uint32_t)B, s1 - base);
    __syncthreads();
    if ((int)threadIdx.x < nb)
      stage_entry<K>(a, a.val[base + threadIdx.x], pr.rx[0], pr.rx[1], pr.rx[2], pr.tx[0], pr.tx[1], pr.tx[2], lam,
                     sgeo + kGeo * threadIdx.x, scf + 2 * K * threadIdx.x);
    if (STATS && threadIdx.x == 0) n_staged += nb;
    __syncthreads();
    if (!done) {
      for (int j = 0; j < nb; ++j) {
        Terms h;
        const float4 *geo = sgeo + kGeo * j;
        if (STATS) ++n_test;
        if (test_hit(vx, vy, vz, geo, a.r_rx, h)) {
          if (STATS) ++n_hit;
          hit_terms<K>(geo, scf + 2 * K * j, Yr, Yi, a.amax, h);
          const float ctr = h.p * h.pzr, cti = h.p * h.pzi;
          Sr = fmaf(T, ctr, Sr);
          Si = fmaf(T, cti, Si);
          T = T * (1.0f - h.alpha);
          if (T < a.t_min) {
            done = true;
            break;
          }
        }
      }
    }
    if (__syncthreads_and(done ? 1 : 0)) break;
  }
  if (STATS) {
    // instrumentation: tests, processed hits, staged entries, rays
    if (n_test) atomicAdd(stats + 0, n_test);
    if (n_hit) atomicAdd(stats + 1, n_hit);
    if (n_staged) atomicAdd(stats + 2, n_staged);
    if (valid) atomicAdd(stats + 3, 1ull);
    return;
  }
  if (valid) signal[((size_t)k * a.n_el + v) * a.n_az + u] = make_float2(Sr, Si);
  // deterministic tile partial of S_hat (fixed tree order)
  __syncthreads();
  float *red = (float *)smem;
  red[threadIdx.x] = Sr;
  red[NT + threadIdx.x] = Si;
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

// a6: S_hat per pair (tiles summed in fixed order, FP64) and RSSI in dBm.
__global__ void k_rssi(const float2 *__restrict__ tile_sum, int32_t T, float *__restrict__ signal_sum,
                       float *__restrict__ rssi) {
  __shared__ double sr[256], si[256];
  const int k = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int t = threadIdx.x; t < T; t += 256) {
    const float2 v = tile_sum[(size_t)k * T + t];
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

// ---------------------------------------------------------------------------
// a7: backward.  Same traversal; per hit the lane forms its contribution to
// the per-Gaussian accumulators, waves reduce across lanes, LDS collects the
// four waves, and one burst of global atomics per (tile, Gaussian) flushes.
// Accumulator layout per Gaussian (acc_stride = 11 + 2K floats):
//   dL/dM (M00 M11 M22 M01 M02 M12), dL/dmu (3), dL/dN, dL/do, dL/dc (2K).
// LDS adds one slot for sum dL/dt, whose TX-leg share (mu - tx)/|mu - tx| is
// applied at the flush.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int L, int NT>
__global__ __launch_bounds__(NT) void k_render_bwd(RenderArgs a, const float2 *__restrict__ signal,
                                                   const float2 *__restrict__ grad_signal,
                                                   const float2 *__restrict__ grad_sum, int32_t acc_stride,
                                                   float *__restrict__ acc) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int B = lds_batch(L, NT, true);
  constexpr int NACC = 12 + 2 * K;
  extern __shared__ float4 smem[];
  float4 *sgeo = smem;                              // [B][kGeo]
  float *scf = (float *)(smem + kGeo * B);          // [B][2K]
  float *sacc = scf + 2 * K * B;                    // [B][NACC]
  int *sflag = (int *)(sacc + NACC * B);            // [B]
  const int gt = blockIdx.x;
  const int k = gt / a.T;
  const int tile = gt - k * a.T;
  const int tv = tile / a.nta, tu = tile - tv * a.nta;
  const int th_ = NT / a.tw;
  const int u = tu * a.tw + (int)threadIdx.x % a.tw;
  const int v = tv * th_ + (int)threadIdx.x / a.tw;
  const bool valid = (u < a.n_az) && (v < a.n_el);
  const int lane = threadIdx.x & 63;
  const gsrf_pair pr = a.pairs[k];
  const double lam = kC0 / pr.freq_hz;
  const float twopi_lam = (float)(2.0 * 3.14159265358979323846 / lam);
  float vx = 0.f, vy = 0.f, vz = 1.f, Yr[K], Yi[K];
  ray_setup<L>(valid ? u : 0, valid ? v : 0, a, vx, vy, vz, Yr, Yi);
  float Sfr = 0.f, Sfi = 0.f, Gr = 0.f, Gi = 0.f;
  if (valid) {
    const size_t ri = ((size_t)k * a.n_el + v) * a.n_az + u;
    const float2 sf = signal[ri], gg = grad_signal[ri];
    Sfr = sf.x; Sfi = sf.y; Gr = gg.x; Gi = gg.y;
    if (grad_sum) {
      const float2 gs = grad_sum[k];
      Gr += gs.x;
      Gi += gs.y;
    }
  }
  for (int i = threadIdx.x; i < NACC * B; i += NT) sacc[i] = 0.f;
  for (int i = threadIdx.x; i < B; i += NT) sflag[i] = 0;
  const uint32_t s0 = a.tstart[gt], s1 = a.tend[gt];
  float T = 1.f, Pr = 0.f, Pi = 0.f;
  bool done = !valid || (1.0f < a.t_min);
  for (uint32_t base = s0; base < s1; base += B) {
    const int nb = (int)min((uint32_t)B, s1 - base);
    __syncthreads();
    if ((int)threadIdx.x < nb)
      stage_entry<K>(a, a.val[base + threadIdx.x], pr.rx[0], pr.rx[1], pr.rx[2], pr.tx[0], pr.tx[1], pr.tx[2], lam,
                     sgeo + kGeo * threadIdx.x, scf + 2 * K * threadIdx.x);
    __syncthreads();
    // waves whose lanes are all finished skip the batch (wave-uniform branch)
    if (__ballot(!done) != 0) {
      for (int j = 0; j < nb; ++j) {
        Terms h;
        const float4 *geo = sgeo + kGeo * j;
        const float *cf = scf + 2 * K * j;
        bool hit = false;
        if (!done) hit = test_hit(vx, vy, vz, geo, a.r_rx, h);
        if (__ballot(hit) == 0) continue;
        float c[12];
        float dpr = 0.f, dpi = 0.f;
#pragma unroll
        for (int f = 0; f < 12; ++f) c[f] = 0.f;
        if (hit) {
          hit_terms<K>(geo, cf, Yr, Yi, a.amax, h);
          const float ctr = h.p * h.pzr, cti = h.p * h.pzi;
          Pr = fmaf(T, ctr, Pr);
          Pi = fmaf(T, cti, Pi);
          const float Rr = Sfr - Pr, Ri = Sfi - Pi;
          const float dLdp = T * fmaf(Gr, h.pzr, Gi * h.pzi);
          const float dLdphi = T * fmaf(Gr, cti, -(Gi * ctr));
          const float dLda = h.clamped ? 0.f : -fmaf(Gr, Rr, Gi * Ri) / (1.0f - h.alpha);
          const float4 g0 = geo[0], g3 = geo[3];
          const float D = g0.w;
          const float dLdG = fmaf(dLdp, g3.z, dLda * g3.w);
          const float gQ = -0.5f * h.G * dLdG;
          const float gt_ = dLdphi * twopi_lam;
          const float gtA = gt_ * h.rA;
          const float px = D * fmaf(-h.bA, vx, h.ex), py = D * fmaf(-h.bA, vy, h.ey), pz = D * fmaf(-h.bA, vz, h.ez);
          const float qx = D * fmaf(-h.bA, h.w0, h.m0), qy = D * fmaf(-h.bA, h.w1, h.m1),
                      qz = D * fmaf(-h.bA, h.w2, h.m2);
          c[0] = fmaf(gQ * px, px, -(gtA * vx * px));
          c[1] = fmaf(gQ * py, py, -(gtA * vy * py));
          c[2] = fmaf(gQ * pz, pz, -(gtA * vz * pz));
          c[3] = fmaf(gQ * px, py, -0.5f * gtA * fmaf(vx, py, px * vy));
          c[4] = fmaf(gQ * px, pz, -0.5f * gtA * fmaf(vx, pz, px * vz));
          c[5] = fmaf(gQ * py, pz, -0.5f * gtA * fmaf(vy, pz, py * vz));
          c[6] = fmaf(-2.0f * gQ, qx, gtA * h.w0);
          c[7] = fmaf(-2.0f * gQ, qy, gtA * h.w1);
          c[8] = fmaf(-2.0f * gQ, qz, gtA * h.w2);
          c[9] = dLdp * h.G;     // dL/dN
          c[10] = dLda * h.G;    // dL/do
          c[11] = gt_;           // dL/dt (TX leg applied at flush)
          const float Tp = T * h.p;
          dpr = Tp * fmaf(Gr, h.cs, -(Gi * h.sn));
          dpi = Tp * fmaf(Gi, h.cs, Gr * h.sn);
          T = T * (1.0f - h.alpha);
          if (T < a.t_min) done = true;
        }
        float *dst = sacc + NACC * j;
#pragma unroll
        for (int f = 0; f < 12; ++f) {
          const float s = wave_sum(c[f]);
          if (lane == 0) atomicAdd(dst + f, s);
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const float cr = wave_sum(fmaf(dpr, Yr[i], dpi * Yi[i]));
          const float ci = wave_sum(fmaf(dpi, Yr[i], -(dpr * Yi[i])));
          if (lane == 0) {
            atomicAdd(dst + 12 + 2 * i, cr);
            atomicAdd(dst + 13 + 2 * i, ci);
          }
        }
        if (lane == 0) sflag[j] = 1;
      }
    }
    __syncthreads();
    // flush: one thread per staged Gaussian with any hit in this tile
    if ((int)threadIdx.x < nb && sflag[threadIdx.x]) {
      const uint32_t g = a.val[base + threadIdx.x];
      float *src = sacc + NACC * threadIdx.x;
      const float *pg = a.prep + (size_t)kPrep * g;
      const double qx = (double)pg[0] - pr.tx[0], qy = (double)pg[1] - pr.tx[1], qz = (double)pg[2] - pr.tx[2];
      const double dn = sqrt((qx * qx + qy * qy) + qz * qz);
      const double inv = dn > 0.0 ? 1.0 / dn : 0.0;
      const float gtx = src[11];
      float *dst = acc + (size_t)acc_stride * g;
#pragma unroll
      for (int f = 0; f < 6; ++f) unsafeAtomicAdd(dst + f, src[f]);
      unsafeAtomicAdd(dst + 6, fmaf(gtx, (float)(qx * inv), src[6]));
      unsafeAtomicAdd(dst + 7, fmaf(gtx, (float)(qy * inv), src[7]));
      unsafeAtomicAdd(dst + 8, fmaf(gtx, (float)(qz * inv), src[8]));
      unsafeAtomicAdd(dst + 9, src[9]);
      unsafeAtomicAdd(dst + 10, src[10]);
#pragma unroll
      for (int i = 0; i < 2 * K; ++i) unsafeAtomicAdd(dst + 11 + i, src[12 + i]);
#pragma unroll
      for (int f = 0; f < NACC; ++f) src[f] = 0.f;
      sflag[threadIdx.x] = 0;
    }
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
__global__ void k_chain(const float *__restrict__ log_scales, const float *__restrict__ quats,
                        const float *__restrict__ logits, const float *__restrict__ acc, int32_t acc_stride,
                        int32_t K, int64_t G, float *__restrict__ d_means, float *__restrict__ d_ls,
                        float *__restrict__ d_q, float *__restrict__ d_a, float *__restrict__ d_c) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const float *A = acc + (size_t)acc_stride * g;
  const float Gm[3][3] = {{A[0], A[3], A[4]}, {A[3], A[1], A[5]}, {A[4], A[5], A[2]}};
  d_means[3 * g + 0] = A[6];
  d_means[3 * g + 1] = A[7];
  d_means[3 * g + 2] = A[8];
  for (int i = 0; i < 2 * K; ++i) d_c[(size_t)2 * K * g + i] = A[11 + i];
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
  const float ls[3] = {l0, l1, l2};
  (void)ls;
  for (int i = 0; i < 3; ++i) {
    const float gd = fmaf(R[0][i], GR[0][i], fmaf(R[1][i], GR[1][i], R[2][i] * GR[2][i]));
    d_ls[3 * g + i] = fmaf(-2.f * d[i], gd, -Nn * A[9]);
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
  d_a[g] = A[10] * o * (1.f - o);
}

// ---------------------------------------------------------------------------
// Instrumentation events recorded around the main render kernels.
// ---------------------------------------------------------------------------
static hipEvent_t g_ev[4] = {nullptr, nullptr, nullptr, nullptr};

void set_kernel_events(void *fwd_start, void *fwd_stop, void *bwd_start, void *bwd_stop) {
  g_ev[0] = (hipEvent_t)fwd_start;
  g_ev[1] = (hipEvent_t)fwd_stop;
  g_ev[2] = (hipEvent_t)bwd_start;
  g_ev[3] = (hipEvent_t)bwd_stop;
}

static void mark(int i, hipStream_t s) {
  if (g_ev[i]) (void)hipEventRecord(g_ev[i], s);
}

// ---------------------------------------------------------------------------
// launch helpers: dispatch on (L, threads per tile)
// ---------------------------------------------------------------------------
static RenderArgs make_args(const gsrf_problem *p, const Layout &lay, char *ws) {
  RenderArgs a;
  const int cur = lay.sort_passes & 1;
  a.pairs = p->pairs;
  a.prep = (const float *)(ws + lay.prep);
  a.coeffs = p->coeffs;
  a.val = (const uint32_t *)(ws + lay.val[cur]);
  a.tstart = (const uint32_t *)(ws + lay.tile_start);
  a.tend = (const uint32_t *)(ws + lay.tile_end);
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

template <int L, int NT>
static hipError_t fwd_launch(const RenderArgs &a, int64_t nblocks, float2 *sig, float2 *tsum,
                             unsigned long long *stats, hipStream_t s) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int B = lds_batch(L, NT, false);
  size_t lds = (size_t)B * (kGeo * 16 + 2 * K * 4);
  if (lds < (size_t)NT * 8) lds = (size_t)NT * 8;
  if (stats)
    hipLaunchKernelGGL((k_render_fwd<L, NT, true>), dim3((unsigned)nblocks), dim3(NT), lds, s, a, sig, tsum, stats);
  else
    hipLaunchKernelGGL((k_render_fwd<L, NT, false>), dim3((unsigned)nblocks), dim3(NT), lds, s, a, sig, tsum, stats);
  return hipGetLastError();
}

template <int L, int NT>
static hipError_t bwd_launch(const RenderArgs &a, int64_t nblocks, const float2 *sig, const float2 *gsig,
                             const float2 *gsum, int32_t stride, float *acc, hipStream_t s) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int B = lds_batch(L, NT, true);
  const size_t lds = (size_t)B * (kGeo * 16 + 2 * K * 4 + (12 + 2 * K) * 4 + 4);
  hipLaunchKernelGGL((k_render_bwd<L, NT>), dim3((unsigned)nblocks), dim3(NT), lds, s, a, sig, gsig, gsum, stride, acc);
  return hipGetLastError();
}

#define GSRF_DISPATCH_NT(FN, L, ...)                                       \
  switch (nt) {                                                            \
    case 64: return FN<L, 64>(__VA_ARGS__);                                \
    case 128: return FN<L, 128>(__VA_ARGS__);                              \
    default: return FN<L, 256>(__VA_ARGS__);                               \
  }

#define GSRF_DISPATCH(FN, ...)                                             \
  switch (p->grid.fle_L) {                                                 \
    case 0: GSRF_DISPATCH_NT(FN, 0, __VA_ARGS__)                           \
    case 1: GSRF_DISPATCH_NT(FN, 1, __VA_ARGS__)                           \
    case 2: GSRF_DISPATCH_NT(FN, 2, __VA_ARGS__)                           \
    case 3: GSRF_DISPATCH_NT(FN, 3, __VA_ARGS__)                           \
    case 4: GSRF_DISPATCH_NT(FN, 4, __VA_ARGS__)                           \
    case 5: GSRF_DISPATCH_NT(FN, 5, __VA_ARGS__)                           \
    default: GSRF_DISPATCH_NT(FN, 6, __VA_ARGS__)                          \
  }

hipError_t launch_render_fwd(const gsrf_problem *p, const Layout &lay, char *ws, float *signal, float *signal_sum,
                             float *rssi_dbm, hipStream_t s) {
  if (p->n_pairs == 0) return hipSuccess;
  const RenderArgs a = make_args(p, lay, ws);
  const int nt = p->grid.tile_w * p->grid.tile_h;
  const int64_t nblocks = (int64_t)p->n_pairs * lay.T;
  float2 *tsum = (float2 *)(ws + lay.tile_sum);
  mark(0, s);
  hipError_t e = [&]() -> hipError_t {
    GSRF_DISPATCH(fwd_launch, a, nblocks, (float2 *)signal, tsum, (unsigned long long *)nullptr, s)
  }();
  mark(1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rssi, dim3(p->n_pairs), dim3(256), 0, s, tsum, lay.T, signal_sum, rssi_dbm);
  return hipGetLastError();
}

hipError_t launch_render_stats(const gsrf_problem *p, const Layout &lay, char *ws, int64_t *counts, hipStream_t s) {
  hipError_t e = fill<int64_t>(counts, 0, 4, s);
  if (e != hipSuccess || p->n_pairs == 0) return e;
  const RenderArgs a = make_args(p, lay, ws);
  const int nt = p->grid.tile_w * p->grid.tile_h;
  const int64_t nblocks = (int64_t)p->n_pairs * lay.T;
  return [&]() -> hipError_t {
    GSRF_DISPATCH(fwd_launch, a, nblocks, (float2 *)nullptr, (float2 *)nullptr, (unsigned long long *)counts, s)
  }();
}

hipError_t launch_render_bwd(const gsrf_problem *p, const Layout &lay, char *ws, const float *signal,
                             const float *grad_signal, const float *grad_sum, float *d_means, float *d_log_scales,
                             float *d_quats, float *d_logits, float *d_coeffs, hipStream_t s) {
  float *acc = (float *)(ws + lay.grad_acc);
  hipError_t e = fill<float>(acc, 0.f, p->n_gauss * lay.acc_stride, s);
  if (e != hipSuccess) return e;
  if (p->n_pairs > 0) {
    const RenderArgs a = make_args(p, lay, ws);
    const int nt = p->grid.tile_w * p->grid.tile_h;
    const int64_t nblocks = (int64_t)p->n_pairs * lay.T;
    mark(2, s);
    e = [&]() -> hipError_t {
      GSRF_DISPATCH(bwd_launch, a, nblocks, (const float2 *)signal, (const float2 *)grad_signal,
                    (const float2 *)grad_sum, lay.acc_stride, acc, s)
    }();
    mark(3, s);
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
