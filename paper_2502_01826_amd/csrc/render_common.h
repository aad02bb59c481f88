// Device code shared by the forward and adjoint renderers (Sec. 3.4 eq.
// rendering; App. A; App. D.3).  Both kernels call the same inline functions
// for the hit test, the per-hit terms and the transmittance scan, so their
// hit decisions, transmittances and termination points agree bit for bit.
//
// Per staged Gaussian the receiver-relative geometry is formed once in FP64
// (distance D, unit direction e as an FP32 hi+lo pair, base phase
// frac((|mu-tx| + D)/lambda)); per (ray, Gaussian) everything is FP32 in the
// Gaussian's local frame:
//   eps = v - e,  w = M v,  A = v.w,  b = eps.w,  c = eps^T M eps,
//   Q = D^2 (c - b^2/A)  (= C - B^2/A, the Mahalanobis^2 at the chord midpoint)
//   t = D (1 - b/A)      (= -B/A, the chord midpoint)
// which avoids the cancellation of C - B^2/A at D ~ 10 m and keeps the phase
// accurate: phase/(2 pi) = frac((|mu-tx| + D)/lambda) - (D/lambda) (b/A).
//
// A ray may be served by G lanes (G = 1, 2, 4): the G lanes of a ray test G
// consecutive entries of the depth-ordered list at once, and an exclusive
// product scan over the group gives each hit its incoming transmittance
// T_j = T * prod_{i<j}(1 - alpha_i), so "process hit j iff T_j >= t_min" is
// decided per hit exactly as in the sequential definition.
#pragma once

#include "gsrf_internal.h"

namespace gsrf {

struct RenderArgs {
  const gsrf_pair *pairs;
  const float *prep;        // [G][kPrep]
  const float *coeffs;      // [G][K][2]
  const uint32_t *val;      // sorted Gaussian ids
  const uint32_t *tstart;   // [P*T]
  const uint32_t *tend;     // [P*T]
  uint32_t *hitmask;        // [splats][R / 32]: per list entry, its hits over the tile's rays (two-phase
                            // traversal: written by the forward, read by the adjoint)
  uint32_t *mask_end;       // [P*T][area / 32]: per 32-ray block of a tile, the end of the list prefix whose
                            // masks the forward wrote (it stops once all its rays have terminated)
  const float *rays;        // [n_el * n_az][ray_stride(K)] ray table made by gsrf_project
  const float *logits;      // [G] opacity logits (the chord transmittance's attenuation coefficient)
  int32_t T, nta, n_az, n_el, tw;
  float el_lo, el_hi, r_rx, t_min, amax;
  int32_t fle_g;            // 1: radiance at the Gaussian's direction (variant kernels only)
  int32_t chord;            // 1: chord transmittance exp(-alpha dt) (variant kernels only)
};

// Geometry record per staged Gaussian: five float4
//   g0 = (e_hi, D)  g1 = (e_lo, D/lambda)  g2 = (M00, M11, M22, M01)
//   g3 = (M02, M12, N, o)  g4 = (phase0, D^2, carrier-step phase terms)
constexpr int kGeo = 5;

// Number of accumulator slots the adjoint reduces per (ray, hit):
// dL/dM (6), dL/dmu through delta (3), dL/dN, dL/do, dL/dt, dL/dc (2K).
constexpr int n_acc(int L) { return 12 + 2 * (L + 1) * (L + 1); }
constexpr int pow2_at_least(int n) { return n <= 32 ? 32 : (n <= 64 ? 64 : 128); }

constexpr int lds_batch(int L, int NT, bool bwd, int cap = 256) {
  // floats per staged entry: geometry + coefficients (+ TX leg, accumulators and flag for bwd)
  int K = (L + 1) * (L + 1);
  int per = 4 * kGeo + 2 * K + (bwd ? 4 + n_acc(L) + 1 : 0);
  int budget = 60 * 1024 / 4;
  int b = NT < cap ? NT : cap;
  while (b > 32 && b * per > budget) b >>= 1;
  return b;
}

// ---------------------------------------------------------------------------
// Per-ray data from the ray table: the FP32 direction and FLE basis
// Y_i = e^{j m alpha} P_l^m(sin beta), i = l^2 + l + m (Sec. 3.2 eq. FLE),
// evaluated in FP64 once per problem by gsrf_project.
// ---------------------------------------------------------------------------
__device__ __forceinline__ const float4 *ray_row(int u, int v, const RenderArgs &a, int K) {
  return (const float4 *)(a.rays + (size_t)(v * a.n_az + u) * ray_stride(K));
}

__device__ __forceinline__ void ray_load_dir(int u, int v, const RenderArgs &a, int K, float &vx, float &vy,
                                             float &vz) {
  const float4 d = ray_row(u, v, a, K)[0];
  vx = d.x;
  vy = d.y;
  vz = d.z;
}

template <int L>
__device__ __forceinline__ void ray_load(int u, int v, const RenderArgs &a, float &vx, float &vy, float &vz, float *Yr,
                                         float *Yi) {
  constexpr int K = (L + 1) * (L + 1);
  constexpr int NQ = (2 * K + 3) / 4;
  const float4 *r4 = ray_row(u, v, a, K);
  const float4 d = r4[0];
  vx = d.x;
  vy = d.y;
  vz = d.z;
  float y[4 * NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const float4 c = r4[1 + q];
    y[4 * q] = c.x;
    y[4 * q + 1] = c.y;
    y[4 * q + 2] = c.z;
    y[4 * q + 3] = c.w;
  }
#pragma unroll
  for (int i = 0; i < K; ++i) {
    Yr[i] = y[2 * i];
    Yi[i] = y[2 * i + 1];
  }
}

// ---------------------------------------------------------------------------
// Stage Gaussian g into an LDS slot (FP64 geometry relative to RX and TX).
// ---------------------------------------------------------------------------
// txg (adjoint only, else null) receives the TX leg of dL/dt, the unit vector
// (mu - tx)/|mu - tx|, and g's bits in w.  STEP (the multi-carrier forward):
// g4.zw = ((|mu - tx| + D), D) * step_rev with step_rev = (carrier step)/c, so
// that a hit at t adds (|mu - tx| + t) * step / c turns per carrier step.
// VAR (the paper-literal variant kernels): with a.fle_g the entry's radiance
// psi_k = sum_i c_i Y_i(e) at the direction e of mu from the receiver is
// formed here, once per entry, and stored as cf[0..1] in place of the
// coefficients; with a.chord g3.w holds the attenuation coefficient
// exp(logit) in place of the opacity.
template <int L>
__device__ __forceinline__ void psi_at_direction(double ex, double ey, double ez, const float *c, double &pr,
                                                 double &pi) {
  // Y_lm = w^m Q_l^m(x), w = ex + j ey, x = ez, Q_l^m = P_l^m / (1 - x^2)^(m/2);
  // Y_{l,-m} = (-1)^m (l-m)!/(l+m)! conj(w)^m Q_l^m (Sec. 3.2 eq. FLE)
  double wr = 1.0, wi = 0.0;      // w^m
  double qmm = 1.0;               // Q_m^m = (-1)^m (2m-1)!!
  pr = 0.0;
  pi = 0.0;
#pragma unroll
  for (int m = 0; m <= L; ++m) {
    if (m > 0) {
      const double nr = wr * ex - wi * ey, ni = wr * ey + wi * ex;
      wr = nr;
      wi = ni;
      qmm = -qmm * (2 * m - 1);
    }
    double q2 = 0.0, q1 = qmm;
#pragma unroll
    for (int l = m; l <= L; ++l) {
      double q;
      if (l == m) {
        q = qmm;
      } else if (l == m + 1) {
        q = ez * (2 * m + 1) * qmm;
        q2 = q1;
        q1 = q;
      } else {
        q = ((2 * l - 1) * ez * q1 - (l + m - 1) * q2) / (l - m);
        q2 = q1;
        q1 = q;
      }
      const double yr = wr * q, yi = wi * q;
      const int ip = l * l + l + m;
      const double cr = c[2 * ip], ci = c[2 * ip + 1];
      pr += cr * yr - ci * yi;
      pi += cr * yi + ci * yr;
      if (m > 0) {
        double f = 1.0;   // (l+m)! / (l-m)!
        for (int t = l - m + 1; t <= l + m; ++t) f *= t;
        const double s = ((m & 1) ? -1.0 : 1.0) / f;
        const int in = l * l + l - m;
        const double nr = s * yr, ni = -s * yi;       // (-1)^m (l-m)!/(l+m)! conj(w^m) Q
        const double dr = c[2 * in], di = c[2 * in + 1];
        pr += dr * nr - di * ni;
        pi += dr * ni + di * nr;
      }
    }
  }
}

template <int K, bool STEP = false, bool VAR = false>
__device__ void stage_entry(const RenderArgs &a, uint32_t g, double rx, double ry, double rz, double tx,
                            double ty, double tz, double inv_lam, float4 *geo, float *cf, float4 *txg = nullptr,
                            double step_rev = 0.0) {
  const float *pg = a.prep + (size_t)kPrep * g;
  // prep record (64-byte aligned): (mu, N) (M00, M11, M22, M01) (M02, M12, o, -)
  const float4 *p4 = (const float4 *)pg;
  const float4 q0 = p4[0], q1 = p4[1], q2 = p4[2];
  const double mx = q0.x, my = q0.y, mz = q0.z;
  const double ex = mx - rx, ey = my - ry, ez = mz - rz;
  const double D2 = (ex * ex + ey * ey) + ez * ez;
  const double D = sqrt(D2);
  const double inv = D > 0.0 ? 1.0 / D : 0.0;
  const double e0 = ex * inv, e1 = ey * inv, e2 = ez * inv;
  const float h0 = (float)e0, h1 = (float)e1, h2 = (float)e2;
  const double qx = mx - tx, qy = my - ty, qz = mz - tz;
  const double dtx = sqrt((qx * qx + qy * qy) + qz * qz);
  const double ph = (dtx + D) * inv_lam;
  geo[0] = make_float4(h0, h1, h2, (float)D);
  geo[1] = make_float4((float)(e0 - (double)h0), (float)(e1 - (double)h1), (float)(e2 - (double)h2),
                       (float)(D * inv_lam));
  geo[2] = q1;
  geo[3] = make_float4(q2.x, q2.y, q0.w, q2.z);
  if constexpr (STEP)
    geo[4] = make_float4((float)(ph - floor(ph)), (float)D2, (float)((dtx + D) * step_rev), (float)(D * step_rev));
  else
    geo[4] = make_float4((float)(ph - floor(ph)), (float)D2, 0.f, 0.f);
  if (txg) {
    const double it = dtx > 0.0 ? 1.0 / dtx : 0.0;
    *txg = make_float4((float)(qx * it), (float)(qy * it), (float)(qz * it), __uint_as_float(g));
  }
  if constexpr (VAR) {
    geo[4].w = (float)(D - (double)(float)D);   // D's low part: the midpoint order's key
    if (a.chord) geo[3].w = expf(a.logits[g]);
    if (a.fle_g) {
      constexpr int LL = K == 1 ? 0 : K == 4 ? 1 : K == 9 ? 2 : K == 16 ? 3 : K == 25 ? 4 : K == 36 ? 5 : 6;
      double pr, pi;
      psi_at_direction<LL>(e0, e1, e2, a.coeffs + (size_t)2 * K * g, pr, pi);
      cf[0] = (float)pr;
      cf[1] = (float)pi;
      return;
    }
  }
  const float4 *c4 = (const float4 *)(a.coeffs + (size_t)2 * K * g);
  if ((K & 1) == 0) {   // 2K floats per Gaussian: 16-byte aligned rows when K is even
#pragma unroll
    for (int i = 0; i < K / 2; ++i) ((float4 *)cf)[i] = c4[i];
  } else {
    const float2 *c2 = (const float2 *)(a.coeffs + (size_t)2 * K * g);
#pragma unroll
    for (int i = 0; i < K; ++i) ((float2 *)cf)[i] = c2[i];
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
  // quarter turns: swap sin/cos on odd quadrants, then flip signs (branch free)
  const int iq = ((int)q) & 3;
  const bool swap = (iq & 1) != 0;
  const float s0 = swap ? pc : ps, c0 = swap ? ps : pc;
  sn = __int_as_float(__float_as_int(s0) ^ ((iq & 2) << 30));
  cs = __int_as_float(__float_as_int(c0) ^ (((iq + 1) & 2) << 30));
}

struct Terms {
  float ex, ey, ez;     // eps = v - e
  float w0, w1, w2;     // M v
  float m0, m1, m2;     // M eps
  float rA, bA, Q;
  float G, alpha, p;
  float sn, cs;         // sin/cos of the phase
  float pr, pi;         // psi
  float pzr, pzi;       // psi e^{-j phase}
  float keep;           // transmittance factor of the hit (1 - alpha, or exp(-alpha_k dt))
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

template <int K, bool VAR = false>
__device__ __forceinline__ void hit_terms(const float4 *geo, const float *cf, const float *Yr, const float *Yi,
                                          float amax, Terms &h, int fle_g = 0, int chord = 0) {
  const float4 g1 = geo[1], g3 = geo[3], g4 = geo[4];
  h.G = __builtin_amdgcn_exp2f(-0.72134752044448170f * h.Q);   // exp(-Q/2)
  if (VAR && chord) {
    // App. A.2: rho = exp(-alpha_k dt), dt = t_out - t_in = 2 sqrt((9 - Q) / A)
    const float dt = 2.0f * sqrtf(fmaxf(kLevel - h.Q, 0.f) * h.rA);
    h.keep = __builtin_amdgcn_exp2f(-1.44269504088896341f * g3.w * dt);
    h.alpha = 1.0f - h.keep;
    h.clamped = false;
  } else {
    const float oG = g3.w * h.G;
    h.clamped = oG > amax;
    h.alpha = fminf(oG, amax);
    h.keep = 1.0f - h.alpha;
  }
  h.p = g3.z * h.G;
  sincos_rev(fmaf(-g1.w, h.bA, g4.x), h.sn, h.cs);
  float pr = 0.f, pi = 0.f;
  if (VAR && fle_g) {
    pr = cf[0];
    pi = cf[1];
  } else {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const float cr = cf[2 * i], ci = cf[2 * i + 1];
      pr = fmaf(cr, Yr[i], fmaf(-ci, Yi[i], pr));
      pi = fmaf(cr, Yi[i], fmaf(ci, Yr[i], pi));
    }
  }
  h.pr = pr;
  h.pi = pi;
  h.pzr = fmaf(pr, h.cs, pi * h.sn);
  h.pzi = fmaf(pi, h.cs, -(pr * h.sn));
}

// ---------------------------------------------------------------------------
// Cross-lane primitives without LDS traffic.  The G lanes of a ray are
// adjacent and G <= 8, so a ray's group stays inside a DPP quad (G <= 4) or
// a half row (G = 8); the reduce-scatter over the rays of a wave pairs lanes
// at distance 32 and 16 with the gfx950 permlane swaps and at 8, 4, 2, 1
// with row rotation, swizzle and quad permutations.
// ---------------------------------------------------------------------------
constexpr int quad_perm(int l0, int l1, int l2, int l3) { return l0 | (l1 << 2) | (l2 << 4) | (l3 << 6); }
constexpr int kDppRowRor8 = 0x128;        // lane i of a 16-lane row reads lane (i + 8) mod 16 = i ^ 8
constexpr int kDppRowShr1 = 0x111;        // lane i of a row reads lane i - 1 (row_shr:1)
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kSwizzleXor4 = 0x101F;      // bit-mask swizzle: and 0x1f, or 0, xor 4
constexpr int kSwizzleLast8 = 0x00F8;     // bit-mask swizzle: and 0x18, or 7 (last lane of the 8-lane group)

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// value of lane (lane ^ D)
template <int D>
__device__ __forceinline__ float xor_lane(float x, int lane) {
  if constexpr (D == 32 || D == 16) {
    const auto r = (D == 32) ? __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false)
                             : __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float((lane & D) ? r[0] : r[1]);
  } else if constexpr (D == 8) {
    return dpp<kDppRowRor8>(x);
  } else if constexpr (D == 4) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), kSwizzleXor4));
  } else if constexpr (D == 2) {
    return dpp<quad_perm(2, 3, 0, 1)>(x);
  } else {
    return dpp<quad_perm(1, 0, 3, 2)>(x);
  }
}

// One reduce-scatter exchange at lane distance D of the slot pair (a, b):
// on return a holds a summed over the lane pair in the lane without bit D
// and b summed in the lane with bit D.
template <int D>
__device__ __forceinline__ void pair_sum(float &a, float b, int lane) {
  if constexpr (D == 32 || D == 16) {
    // swap: a' = (a of the low lane, b of the low lane), b' = (a of the high
    // lane, b of the high lane) per pair, so a' + b' is the pair sum of a in
    // the low lane and of b in the high lane
    const auto r = (D == 32) ? __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false)
                             : __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  } else {
    const float as = a + xor_lane<D>(a, lane);
    const float bs = b + xor_lane<D>(b, lane);
    a = (lane & D) ? bs : as;
  }
}

// Exclusive product and total of f over the G lanes of a ray (lanes q = 0..G-1
// adjacent in the wave).  Every lane of the wave must call it.
template <int G>
__device__ __forceinline__ void group_prod(float f, int q, float &excl, float &total) {
  if constexpr (G == 1) {
    excl = 1.f;
    total = f;
  } else if constexpr (G == 2) {
    const float lo = dpp<quad_perm(0, 0, 2, 2)>(f);
    const float incl = (q >= 1) ? f * lo : f;
    excl = (q == 0) ? 1.f : lo;
    total = dpp<quad_perm(1, 1, 3, 3)>(incl);
  } else if constexpr (G == 4) {
    const float s1 = dpp<quad_perm(0, 0, 1, 2)>(f);
    const float x = (q >= 1) ? f * s1 : f;
    const float s2 = dpp<quad_perm(0, 1, 0, 1)>(x);
    const float incl = (q >= 2) ? x * s2 : x;
    const float e = dpp<quad_perm(0, 0, 1, 2)>(incl);
    excl = (q == 0) ? 1.f : e;
    total = dpp<quad_perm(3, 3, 3, 3)>(incl);
  } else {
    static_assert(G == 8, "lanes per ray: 1, 2, 4 or 8");
    const float s1 = dpp<kDppRowShr1>(f);
    const float x = (q >= 1) ? f * s1 : f;
    const float s2 = dpp<kDppRowShr2>(x);
    const float y = (q >= 2) ? x * s2 : x;
    const float s4 = dpp<kDppRowShr4>(y);
    const float incl = (q >= 4) ? y * s4 : y;
    const float e = dpp<kDppRowShr1>(incl);
    excl = (q == 0) ? 1.f : e;
    total = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(incl), kSwizzleLast8));
  }
}

// Inclusive sum and total of x over the G lanes of a ray.
template <int G>
__device__ __forceinline__ void group_sum(float x, int q, float &incl, float &total) {
  if constexpr (G == 1) {
    incl = x;
    total = x;
  } else if constexpr (G == 2) {
    const float lo = dpp<quad_perm(0, 0, 2, 2)>(x);
    incl = (q >= 1) ? x + lo : x;
    total = dpp<quad_perm(1, 1, 3, 3)>(incl);
  } else if constexpr (G == 4) {
    const float s1 = dpp<quad_perm(0, 0, 1, 2)>(x);
    const float y = (q >= 1) ? x + s1 : x;
    const float s2 = dpp<quad_perm(0, 1, 0, 1)>(y);
    incl = (q >= 2) ? y + s2 : y;
    total = dpp<quad_perm(3, 3, 3, 3)>(incl);
  } else {
    static_assert(G == 8, "lanes per ray: 1, 2, 4 or 8");
    const float s1 = dpp<kDppRowShr1>(x);
    const float y = (q >= 1) ? x + s1 : x;
    const float s2 = dpp<kDppRowShr2>(y);
    const float z = (q >= 2) ? y + s2 : y;
    const float s4 = dpp<kDppRowShr4>(z);
    incl = (q >= 4) ? z + s4 : z;
    total = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(incl), kSwizzleLast8));
  }
}

// FP64 forms of the above for the running complex sums of a ray: a 64-bit
// value moves as its two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double swizzle_last8_64(double v) {
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), kSwizzleLast8);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), kSwizzleLast8);
  return __hiloint2double(hi, lo);
}

// Inclusive prefix and total of x over the G lanes of a ray, in FP64.
template <int G>
__device__ __forceinline__ void group_sum64(double x, int q, double &incl, double &total) {
  if constexpr (G == 1) {
    incl = x;
    total = x;
  } else if constexpr (G == 2) {
    const double lo = dpp64<quad_perm(0, 0, 2, 2)>(x);
    incl = (q >= 1) ? x + lo : x;
    total = dpp64<quad_perm(1, 1, 3, 3)>(incl);
  } else if constexpr (G == 4) {
    const double s1 = dpp64<quad_perm(0, 0, 1, 2)>(x);
    const double y = (q >= 1) ? x + s1 : x;
    const double s2 = dpp64<quad_perm(0, 1, 0, 1)>(y);
    incl = (q >= 2) ? y + s2 : y;
    total = dpp64<quad_perm(3, 3, 3, 3)>(incl);
  } else {
    static_assert(G == 8, "lanes per ray: 1, 2, 4 or 8");
    const double s1 = dpp64<kDppRowShr1>(x);
    const double y = (q >= 1) ? x + s1 : x;
    const double s2 = dpp64<kDppRowShr2>(y);
    const double z = (q >= 2) ? y + s2 : y;
    const double s4 = dpp64<kDppRowShr4>(z);
    incl = (q >= 4) ? z + s4 : z;
    total = swizzle_last8_64(incl);
  }
}

// Reduce-scatter across the lanes of a wave that share q = lane % G (the rays
// of the wave), by recursive halving: at lane distance D the lane keeps half of
// its live slots and adds the partner's copy of them.  On return the lane holds
// slots [first, first + NV*G/64) of its group's entry, summed over all 64/G
// rays.  When NV*G < 64 the last halvings have a single live slot left: the
// pair of lanes then both hold it and only the one without bit D writes it.
// Every index is a compile-time constant, so v stays in registers.
template <int NV, int G, int D>
__device__ __forceinline__ void rs_step(float (&v)[NV], int lane, int &first, bool &writer) {
  if constexpr (D >= G) {
    constexpr int LIVE = (NV * D / 32 >= 1) ? NV * D / 32 : 1;
    if constexpr (LIVE > 1) {
      constexpr int H = LIVE / 2;
#pragma unroll
      for (int i = 0; i < H; ++i) pair_sum<D>(v[i], v[i + H], lane);
      if (lane & D) first += H;
    } else {
      v[0] += xor_lane<D>(v[0], lane);
      if (lane & D) writer = false;
    }
    rs_step<NV, G, D / 2>(v, lane, first, writer);
  }
}

template <int NV, int G>
__device__ __forceinline__ void reduce_scatter(float (&v)[NV], int lane, int *first, bool *writer) {
  int f = 0;
  bool w = true;
  rs_step<NV, G, 32>(v, lane, f, w);
  *first = f;
  *writer = w;
}

// Accumulator slots of the adjoint (SoA in global memory, acc[f * n_gauss + g]):
//   0-5 dL/dM (M00 M11 M22 M01 M02 M12), 6-8 dL/dmu, 9 dL/dN, 10 dL/do,
//   11.. dL/dc (2K); the LDS copy adds slot 11 + 2K = sum of dL/dt, whose TX leg
//   (mu - tx)/|mu - tx| is folded into dL/dmu at the flush.
// Contributions of one processed hit j to the Gaussian's accumulator slots.
// Rr, Ri: remainder sum_{i>j} T_i c~_i; (Gr, Gi): dL/dS of the ray.
template <int K, int NV>
__device__ __forceinline__ void hit_adjoint(const Terms &h, const float4 *geo, float Tj, float ctr, float cti,
                                            float Rr, float Ri, float Gr, float Gi, float vx, float vy, float vz,
                                            const float *Yr, const float *Yi, float twopi_lam, float (&c)[NV]) {
  constexpr int SLOT_T = 11 + 2 * K;
  const float dLdp = Tj * fmaf(Gr, h.pzr, Gi * h.pzi);
  const float dLdphi = Tj * fmaf(Gr, cti, -(Gi * ctr));
  const float dLda = h.clamped ? 0.f : -fmaf(Gr, Rr, Gi * Ri) / (1.0f - h.alpha);
  const float4 g0 = geo[0], g3 = geo[3];
  const float D = g0.w;
  const float dLdG = fmaf(dLdp, g3.z, dLda * g3.w);
  const float gQ = -0.5f * h.G * dLdG;
  const float gt_ = dLdphi * twopi_lam;
  const float gtA = gt_ * h.rA;
  // x_mid - mu = D (eps - (b/A) v), M (x_mid - mu) = D (M eps - (b/A) M v)
  const float px = D * fmaf(-h.bA, vx, h.ex), py = D * fmaf(-h.bA, vy, h.ey), pz = D * fmaf(-h.bA, vz, h.ez);
  const float qx = D * fmaf(-h.bA, h.w0, h.m0), qy = D * fmaf(-h.bA, h.w1, h.m1), qz = D * fmaf(-h.bA, h.w2, h.m2);
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
  const float Tp = Tj * h.p;
  const float dpr = Tp * fmaf(Gr, h.cs, -(Gi * h.sn));
  const float dpi = Tp * fmaf(Gi, h.cs, Gr * h.sn);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    c[11 + 2 * i] = fmaf(dpr, Yr[i], dpi * Yi[i]);
    c[12 + 2 * i] = fmaf(dpi, Yr[i], -(dpr * Yi[i]));
  }
  c[SLOT_T] = gt_;       // dL/dt; TX leg applied at the flush
}

// The same contributions in parts of 16 slots, for a caller that reduces each
// part before forming the next (fewer values live at once): adj_hit forms the
// per-hit scalars, adj_slot<K>(s) slot s from them (s a compile-time index
// after unrolling).  A zero AdjHit gives zero in every slot.
struct AdjHit {
  float gQ, gtA, gt, px, py, pz, qx, qy, qz, w0, w1, w2, dN, dO, dpr, dpi;
};

__device__ __forceinline__ AdjHit adj_hit(const Terms &h, const float4 *geo, float Tj, float ctr, float cti, float Rr,
                                          float Ri, float Gr, float Gi, float vx, float vy, float vz,
                                          float twopi_lam) {
  AdjHit a;
  const float dLdp = Tj * fmaf(Gr, h.pzr, Gi * h.pzi);
  const float dLdphi = Tj * fmaf(Gr, cti, -(Gi * ctr));
  const float dLda = h.clamped ? 0.f : -fmaf(Gr, Rr, Gi * Ri) / (1.0f - h.alpha);
  const float4 g0 = geo[0], g3 = geo[3];
  const float D = g0.w;
  const float dLdG = fmaf(dLdp, g3.z, dLda * g3.w);
  a.gQ = -0.5f * h.G * dLdG;
  a.gt = dLdphi * twopi_lam;
  a.gtA = a.gt * h.rA;
  a.px = D * fmaf(-h.bA, vx, h.ex);
  a.py = D * fmaf(-h.bA, vy, h.ey);
  a.pz = D * fmaf(-h.bA, vz, h.ez);
  a.qx = D * fmaf(-h.bA, h.w0, h.m0);
  a.qy = D * fmaf(-h.bA, h.w1, h.m1);
  a.qz = D * fmaf(-h.bA, h.w2, h.m2);
  a.w0 = h.w0;
  a.w1 = h.w1;
  a.w2 = h.w2;
  a.dN = dLdp * h.G;
  a.dO = dLda * h.G;
  const float Tp = Tj * h.p;
  a.dpr = Tp * fmaf(Gr, h.cs, -(Gi * h.sn));
  a.dpi = Tp * fmaf(Gi, h.cs, Gr * h.sn);
  return a;
}

// The per-hit scalars for several carriers f_c = f_b + c df (c = 0 .. C-1) at
// once.  Carrier c's term is p psi e^{-j phi_c} with phi_c = phi_b + c delta, so
// every sum over carriers of conj(G_c) times a carrier-c term is conj(Ge)
// times the base-carrier term, with Ge = sum_c G_c e^{j c delta}; the path
// length enters carrier c's phase as 2 pi f_c / c0, which adds
// Ge2 = sum_c c G_c e^{j c delta} at 2 pi df / c0.  num is
// sum_c Re(conj(G_c) R_c), the carriers' remainders after the hit.
__device__ __forceinline__ AdjHit adj_hit_multi(const Terms &h, const float4 *geo, float Tj, float ctr, float cti,
                                                float num, float Ger, float Gei, float Ge2r, float Ge2i, float vx,
                                                float vy, float vz, float twopi_lam, float twopi_dlam) {
  AdjHit a;
  const float dLdp = Tj * fmaf(Ger, h.pzr, Gei * h.pzi);
  const float dLdphi = Tj * fmaf(Ger, cti, -(Gei * ctr));
  const float dLdphi2 = Tj * fmaf(Ge2r, cti, -(Ge2i * ctr));
  const float dLda = h.clamped ? 0.f : -num / (1.0f - h.alpha);
  const float4 g0 = geo[0], g3 = geo[3];
  const float D = g0.w;
  const float dLdG = fmaf(dLdp, g3.z, dLda * g3.w);
  a.gQ = -0.5f * h.G * dLdG;
  a.gt = fmaf(dLdphi, twopi_lam, dLdphi2 * twopi_dlam);
  a.gtA = a.gt * h.rA;
  a.px = D * fmaf(-h.bA, vx, h.ex);
  a.py = D * fmaf(-h.bA, vy, h.ey);
  a.pz = D * fmaf(-h.bA, vz, h.ez);
  a.qx = D * fmaf(-h.bA, h.w0, h.m0);
  a.qy = D * fmaf(-h.bA, h.w1, h.m1);
  a.qz = D * fmaf(-h.bA, h.w2, h.m2);
  a.w0 = h.w0;
  a.w1 = h.w1;
  a.w2 = h.w2;
  a.dN = dLdp * h.G;
  a.dO = dLda * h.G;
  const float Tp = Tj * h.p;
  a.dpr = Tp * fmaf(Ger, h.cs, -(Gei * h.sn));
  a.dpi = Tp * fmaf(Gei, h.cs, Ger * h.sn);
  return a;
}

// Ge = sum_c G_c e^{j c delta} and Ge2 = sum_c c G_c e^{j c delta} over the
// chunk's carriers (g: its kGcChunk values of dL/dS of the ray), with
// (sd, cd) = (sin delta, cos delta): the phase step between carriers.
template <int NC>
__device__ __forceinline__ void carrier_sums_n(const float2 *g, float sd, float cd, float &Ger, float &Gei, float &Ge2r,
                                               float &Ge2i) {
  float zr = 1.f, zi = 0.f;
  Ger = Gei = Ge2r = Ge2i = 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const float2 gc = g[c];
    const float tr = fmaf(gc.x, zr, -(gc.y * zi)), ti = fmaf(gc.x, zi, gc.y * zr);
    Ger += tr;
    Gei += ti;
    Ge2r = fmaf((float)c, tr, Ge2r);
    Ge2i = fmaf((float)c, ti, Ge2i);
    const float nr = fmaf(zr, cd, -(zi * sd)), ni = fmaf(zi, cd, zr * sd);
    zr = nr;
    zi = ni;
  }
}

template <int K>
__device__ __forceinline__ float adj_slot(int s, const AdjHit &a, float vx, float vy, float vz, const float *Yr,
                                          const float *Yi) {
  constexpr int SLOT_T = 11 + 2 * K;
  switch (s) {
    case 0: return fmaf(a.gQ * a.px, a.px, -(a.gtA * vx * a.px));
    case 1: return fmaf(a.gQ * a.py, a.py, -(a.gtA * vy * a.py));
    case 2: return fmaf(a.gQ * a.pz, a.pz, -(a.gtA * vz * a.pz));
    case 3: return fmaf(a.gQ * a.px, a.py, -0.5f * a.gtA * fmaf(vx, a.py, a.px * vy));
    case 4: return fmaf(a.gQ * a.px, a.pz, -0.5f * a.gtA * fmaf(vx, a.pz, a.px * vz));
    case 5: return fmaf(a.gQ * a.py, a.pz, -0.5f * a.gtA * fmaf(vy, a.pz, a.py * vz));
    case 6: return fmaf(-2.0f * a.gQ, a.qx, a.gtA * a.w0);
    case 7: return fmaf(-2.0f * a.gQ, a.qy, a.gtA * a.w1);
    case 8: return fmaf(-2.0f * a.gQ, a.qz, a.gtA * a.w2);
    case 9: return a.dN;
    case 10: return a.dO;
    default:
      if (s == SLOT_T) return a.gt;
      if (s > SLOT_T) return 0.f;
      {
        const int i = (s - 11) >> 1;
        return ((s - 11) & 1) ? fmaf(a.dpi, Yr[i], -(a.dpr * Yi[i])) : fmaf(a.dpr, Yr[i], a.dpi * Yi[i]);
      }
  }
}

// Flush of a staged batch's LDS accumulators to the global accumulators
// acc[n_gauss][S] (row stride S >= 11 + 2K floats, 64-byte aligned rows), one
// lane per (entry, slot) so that the atomics of one wave instruction land on
// one or two Gaussians' rows instead of one row per lane.  dL/dt's TX leg
// (mu - tx)/|mu - tx| (txg, staged with the entry together with its Gaussian
// id) is folded into dL/dmu on the way.  Entries whose flag is clear had no
// processed hit.  Every thread of the workgroup calls it, after a barrier
// that ends the batch's accumulation; it leaves every slot but dL/dt zeroed,
// and the caller clears the flags and the dL/dt slots before the next batch.
template <int K, int NT>
__device__ __forceinline__ void flush_batch(int nb, float *sacc, const uint32_t *sflag, const float4 *txg,
                                            float *__restrict__ acc, int S) {
  constexpr int SLOT_T = 11 + 2 * K;
  constexpr int NACC = 12 + 2 * K;
  constexpr int FW = pow2_at_least(NACC);
  for (int i = threadIdx.x; i < nb * FW; i += NT) {
    const int e = i / FW, f = i % FW;
    if (f < SLOT_T) {
      float *src = sacc + NACC * e + f;
      if (sflag[e]) {
        const float4 tg = txg[e];
        float v = *src;
        if (f >= 6 && f <= 8) v = fmaf(sacc[NACC * e + SLOT_T], f == 6 ? tg.x : (f == 7 ? tg.y : tg.z), v);
        unsafeAtomicAdd(acc + (size_t)__float_as_uint(tg.w) * S + f, v);
      }
      *src = 0.f;
    }
  }
}

}  // namespace gsrf
