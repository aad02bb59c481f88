// Steps a1-a2: per-Gaussian activation and orthographic splatting of every
// (pair, Gaussian) record, ending with the per-tile splat counts and ranges.
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
// The same launch also clears the per-(tile, sub-bucket) counters (grid
// stride) and, in workgroup 0, makes the record base of every pair:
// rec_base[k] = sum_{k'<k} |scene(k')|, rec_base[P] = R.
__device__ void rec_base_scan(const gsrf_pair *__restrict__ pairs, const int64_t *__restrict__ scene_off, int32_t P,
                              int64_t *__restrict__ rec_base) {
  __shared__ int64_t sh[256];
  const int tid = threadIdx.x;
  const int per = (P + 255) / 256;
  const int lo = tid * per, hi = min(P, lo + per);
  int64_t local = 0;
  for (int k = lo; k < hi; ++k) {
    const int s = pairs[k].scene;
    local += scene_off[s + 1] - scene_off[s];
  }
  sh[tid] = local;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t v = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += v;
    __syncthreads();
  }
  int64_t run = sh[tid] - local;
  for (int k = lo; k < hi; ++k) {
    rec_base[k] = run;
    const int s = pairs[k].scene;
    run += scene_off[s + 1] - scene_off[s];
  }
  if (tid == 255) rec_base[P] = sh[255];
}

// Ray (u, v) of the receiver grid: azimuth alpha_u = 2 pi (u + 1/2) / n_az,
// elevation beta_v = el_lo + (el_hi - el_lo) (v + 1/2) / n_el; its direction
// rounded to FP32 and the FLE basis Y_i = e^{j m alpha} P_l^m(sin beta),
// i = l^2 + l + m (Sec. 3.2 eq. FLE), evaluated in FP64 and rounded to FP32,
// stored as one ray-table row: (vx, vy, vz, 0, Yr_0, Yi_0, Yr_1, Yi_1, ...).
template <int L>
__device__ void ray_table_row(int u, int v, int n_az, int n_el, float el_lo, float el_hi, float *row) {
  const double pi = 3.14159265358979323846;
  const double al = 2.0 * pi * (u + 0.5) / n_az;
  const double be = (double)el_lo + ((double)el_hi - (double)el_lo) * (v + 0.5) / n_el;
  const double cb = cos(be), sb = sin(be), ca = cos(al), sa = sin(al);
  row[0] = (float)(cb * ca);
  row[1] = (float)(cb * sa);
  row[2] = (float)sb;
  row[3] = 0.f;
  float *Y = row + 4;
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
  // cos(m alpha), sin(m alpha) by the angle-addition recurrence
  double cm[L + 1], sm[L + 1];
  cm[0] = 1.0;
  sm[0] = 0.0;
#pragma unroll
  for (int m = 1; m <= L; ++m) {
    cm[m] = cm[m - 1] * ca - sm[m - 1] * sa;
    sm[m] = sm[m - 1] * ca + cm[m - 1] * sa;
  }
#pragma unroll
  for (int l = 0; l <= L; ++l) {
#pragma unroll
    for (int m = 0; m <= l; ++m) {
      const double c = cm[m], sn = sm[m];
      const double pl = P[l][m];
      Y[2 * (l * l + l + m)] = (float)(pl * c);
      Y[2 * (l * l + l + m) + 1] = (float)(pl * sn);
      if (m > 0) {
        double f = 1.0;  // (l+m)! / (l-m)!
        for (int t = l - m + 1; t <= l + m; ++t) f *= t;
        const double pn = ((m & 1) ? -pl : pl) / f;   // P_l^{-m}
        Y[2 * (l * l + l - m)] = (float)(pn * c);
        Y[2 * (l * l + l - m) + 1] = (float)(-pn * sn);
      }
    }
  }
  for (int i = 4 + 2 * (L + 1) * (L + 1); i < ray_stride((L + 1) * (L + 1)); ++i) row[i] = 0.f;
}

// Workgroups [0, ceil(G / 256)) activate Gaussians; the next ceil(n_rays / 256)
// make the ray table, which depends on the grid only.
template <int L>
__global__ __launch_bounds__(256) void k_activate(const float *__restrict__ means, const float *__restrict__ log_scales,
                                                  const float *__restrict__ quats, const float *__restrict__ logits,
                                                  int64_t G, float *__restrict__ prep, uint32_t *__restrict__ tile_cnt,
                                                  int64_t n_cnt, const gsrf_pair *__restrict__ pairs,
                                                  const int64_t *__restrict__ scene_off, int32_t P,
                                                  int64_t *__restrict__ rec_base, int n_az, int n_el, float el_lo,
                                                  float el_hi, float *__restrict__ rays, uint32_t *__restrict__ long_q) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_cnt; i += stride) tile_cnt[i] = 0u;
  if (long_q && blockIdx.x == 0 && threadIdx.x < kLongQueueHeader) long_q[threadIdx.x] = 0u;
  if (blockIdx.x == 0 && P > 0) rec_base_scan(pairs, scene_off, P, rec_base);
  const int64_t nb_g = (G + 255) / 256;
  if ((int64_t)blockIdx.x >= nb_g) {
    const int64_t ray = ((int64_t)blockIdx.x - nb_g) * 256 + threadIdx.x;
    if (ray < (int64_t)n_az * n_el) {
      const int v = (int)(ray / n_az), u = (int)(ray - (int64_t)v * n_az);
      ray_table_row<L>(u, v, n_az, n_el, el_lo, el_hi, rays + ray * ray_stride((L + 1) * (L + 1)));
    }
    return;
  }
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
  float4 *o = (float4 *)(prep + kPrep * g);
  o[0] = make_float4(means[3 * g + 0], means[3 * g + 1], means[3 * g + 2], inv_2pi_15 * expf(-(l0 + l1 + l2)));
  o[1] = make_float4(M[0][0], M[1][1], M[2][2], 0.5f * (M[0][1] + M[1][0]));
  o[2] = make_float4(0.5f * (M[0][2] + M[2][0]), 0.5f * (M[1][2] + M[2][1]), 1.f / (1.f + expf(-logits[g])), 0.f);
  // binning: bounding-sphere radius 3 max(s) (FP32, as the cap evaluation uses it) and max log-scale
  const float lmax = fmaxf(fmaxf(l0, l1), l2);
  o[3] = make_float4(3.0f * expf(lmax), lmax, 0.f, 0.f);
}

// ---------------------------------------------------------------------------
// a2: per (pair, Gaussian) depth key and conservative tile rectangle, FP64.
//   e = mu - r, D^2 = (ex ex + ey ey) + ez ez (no FMA), key = bits(fp32(D^2)).
//   Culled if D + Rb < r_rx (1 - 1e-6) with Rb = 3 max(s).  If D <= Rb (1+1e-6)
//   every row and column is covered.  Otherwise theta = asin(Rb/D) + slack,
//   rows with centre elevation in [beta_c - theta, beta_c + theta], and columns
//   with centre azimuth within asin(sin theta / cos beta_c) of alpha_c unless
//   the band reaches a pole.  Columns wrap at the azimuth seam.
// The workgroup (RB records of one pair) counts its splats per tile in LDS
// and adds the counts to tile_cnt with one atomic per touched tile.
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
// Ray index ranges -> tile rectangle (integer tail shared by both evaluations).
// Tile sides are powers of two (the area is 32, 64, 128 or 256) and every
// dividend below is non-negative (rows are clipped to the grid, and one turn
// added to a negative first column makes it non-negative because the columns
// span less than one and a half turns), so the tile indices are shifts.
__device__ __forceinline__ ushort4 tile_rect(int v_lo, int v_hi, int u_lo, int u_hi, bool full, int n_az, int tw,
                                             int th, int32_t nta) {
  if (full) { u_lo = 0; u_hi = n_az - 1; }
  if (!((v_lo <= v_hi) && (full || u_hi >= u_lo))) return make_ushort4(0, 0, 0, 0);
  if (u_lo < 0) { u_lo += n_az; u_hi += n_az; }
  const int sw = __builtin_ctz((unsigned)tw), sh = __builtin_ctz((unsigned)th);
  int tu0 = u_lo >> sw;
  int ntu = (u_hi < n_az) ? ((u_hi >> sw) - tu0 + 1) : ((nta - tu0) + ((u_hi - n_az) >> sw) + 1);
  if (ntu >= nta) { tu0 = 0; ntu = nta; }
  const int tv0 = v_lo >> sh;
  const int ntv = (v_hi >> sh) - tv0 + 1;
  return make_ushort4((unsigned short)tu0, (unsigned short)ntu, (unsigned short)tv0, (unsigned short)ntv);
}

// The same rectangle evaluated in FP32, accepted only when every discrete
// decision (cull, inside, pole, and the four ceil/floor of ray indices) lies
// farther from its threshold than kFastAngTol (in angle, or that angle in index
// units) plus 2e-6 of the index's magnitude.  Under the guards used here
// (Rb/D <= 0.9, cos beta_c >= 0.2, sin theta / cos beta_c <= 0.9) the FP32
// values of the four fractional ray indices differ from the FP64 ones by at
// most 1e-6 rad (measured over 1.6 M records of rooms like the benchmark's,
// 20 times below the tolerance), so an accepted result equals the FP64 one;
// otherwise the caller evaluates the FP64 definition (about 1 % of records).
constexpr float kFastAngTol = 2e-5f;
constexpr double kCosSlack = 0.99999999995;           // cos(kCapSlack)
constexpr double kSinSlack = 9.9999999998333333e-06;  // sin(kCapSlack)
static_assert(kCapSlack == 1e-5, "kCosSlack and kSinSlack are cos and sin of kCapSlack");
constexpr float kFastRelTol = 2e-6f;

__device__ __forceinline__ bool near_int(float x, float tol) { return fabsf(x - rintf(x)) <= tol; }

__device__ __forceinline__ bool cap_rect_fp32(float ex, float ey, float ez, float D, float Rb, const gsrf_grid &grid,
                                              int32_t nta, ushort4 *out) {
  const float DR = D + Rb;
  if (fabsf(DR - grid.r_rx) <= 1e-5f * (DR + grid.r_rx)) return false;
  if (DR < grid.r_rx) {
    *out = make_ushort4(0, 0, 0, 0);
    return true;
  }
  if (fabsf(D - Rb) <= 1e-5f * DR) return false;
  if (D <= Rb) {
    *out = tile_rect(0, grid.n_el - 1, 0, grid.n_az - 1, true, grid.n_az, grid.tile_w, grid.tile_h, nta);
    return true;
  }
  const float sr = Rb / D;
  if (sr > 0.9f) return false;
  const float theta = asinf(sr) + (float)kCapSlack;
  const float rho = sqrtf(ex * ex + ey * ey);
  const float bc = atan2f(ez, rho);
  const float lo = bc - theta, hi = bc + theta;
  const float halfpi = 1.57079632679489662f;
  if (fabsf(hi - halfpi) <= kFastAngTol || fabsf(lo + halfpi) <= kFastAngTol) return false;
  const float dbeta = (grid.el_hi - grid.el_lo) / (float)grid.n_el;
  const float xl = (lo - grid.el_lo) / dbeta - 0.5f, xh = (hi - grid.el_lo) / dbeta - 0.5f;
  const float tolv = kFastAngTol / dbeta;
  if (near_int(xl, tolv + kFastRelTol * (fabsf(xl) + 1.f)) || near_int(xh, tolv + kFastRelTol * (fabsf(xh) + 1.f)))
    return false;
  int v_lo = (int)ceilf(xl), v_hi = (int)floorf(xh);
  if (v_lo < 0) v_lo = 0;
  if (v_hi > grid.n_el - 1) v_hi = grid.n_el - 1;
  bool full = (hi >= halfpi) || (lo <= -halfpi);
  int u_lo = 0, u_hi = grid.n_az - 1;
  if (!full) {
    const float cb = rho / D;                                    // cos(beta_c)
    if (cb < 0.2f) return false;
    // sin(theta) = sin(asin(sr) + slack) = sr cos(slack) + cos(asin(sr)) sin(slack), cos(slack) = 1 in FP32
    const float r = fmaf(sqrtf(fmaxf(0.f, 1.f - sr * sr)), (float)kCapSlack, sr) / cb;
    if (r > 0.9f) return false;
    const float da = asinf(r);
    const float ac = atan2f(ey, ex);
    const float dalpha = 6.28318530717958648f / (float)grid.n_az;
    const float ul = (ac - da) / dalpha - 0.5f, uh = (ac + da) / dalpha - 0.5f;
    const float tolu = kFastAngTol / dalpha;
    if (near_int(ul, tolu + kFastRelTol * (fabsf(ul) + 1.f)) || near_int(uh, tolu + kFastRelTol * (fabsf(uh) + 1.f)))
      return false;
    u_lo = (int)ceilf(ul);
    u_hi = (int)floorf(uh);
    if (u_hi - u_lo + 1 >= grid.n_az) full = true;
  }
  *out = tile_rect(v_lo, v_hi, u_lo, u_hi, full, grid.n_az, grid.tile_w, grid.tile_h, nta);
  return true;
}

// FP64 evaluation of the rectangle, in the operation order documented above,
// except that sin(theta) and cos(beta_c) come from identities instead of two
// more transcendental calls: sin(asin(x) + s) = x cos s + sqrt(1 - x^2) sin s and
// cos(atan2(e_z, rho)) = rho / D (FP64 differences ~1e-16, far inside the 1e-9
// band within which a decision counts as marginal).  Scalar arguments: not
// inlined, and nothing of the caller's needs memory.
__device__ __noinline__ ushort4 cap_rect_fp64(float mx, float my, float mz, float rx, float ry, float rz, float lmaxf,
                                              int n_az, int n_el, float el_lo_f, float el_hi_f, float r_rx, int tw,
                                              int th, int32_t nta) {
  const double ex = (double)mx - (double)rx;
  const double ey = (double)my - (double)ry;
  const double ez = (double)mz - (double)rz;
  const double D2 = (ex * ex + ey * ey) + ez * ez;
  const double D = sqrt(D2);
  const double Rb = 3.0 * exp((double)lmaxf);
  const double el_lo = (double)el_lo_f, el_hi = (double)el_hi_f;
  const double pi = 3.14159265358979323846;
  if (D + Rb < (double)r_rx * (1.0 - 1e-6)) return make_ushort4(0, 0, 0, 0);
  const bool inside = D <= Rb * (1.0 + 1e-6);
  long v_lo, v_hi, u_lo = 0, u_hi = n_az - 1;
  bool full;
  if (inside) {
    v_lo = 0; v_hi = n_el - 1; full = true;
  } else {
    const double sr = fmin(Rb / D, 1.0);
    const double theta = asin(sr) + kCapSlack;
    const double rho = sqrt(ex * ex + ey * ey);
    const double bc = atan2(ez, rho);
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
      const double sin_theta = sr * kCosSlack + sqrt(1.0 - sr * sr) * kSinSlack;
      const double da = asin(fmin(sin_theta / (rho / D), 1.0));
      u_lo = (long)ceil((ac - da) / dalpha - 0.5);
      u_hi = (long)floor((ac + da) / dalpha - 0.5);
      if (u_hi - u_lo + 1 >= n_az) full = true;
    }
  }
  return tile_rect((int)v_lo, (int)v_hi, (int)u_lo, (int)u_hi, full, n_az, tw, th, nta);
}

// The paper's footprint (Sec. 3.3, splatting), FP64, as a binning variant:
// projected centre (u_k, v_k) = floor of the direction's ray-index
// coordinates; Sigma2D = J Sigma J^T with J the Jacobian of
// x -> (alpha / d_alpha, (beta - el_lo) / d_beta) at mu and
// Sigma = R diag(s^2) R^T; r_k = 3 sqrt(lambda_max(Sigma2D)); the circle's
// bounding square u_k +- m, v_k +- m with m = floor(r_k), rows clipped,
// columns modulo n_az.  Not conservative: J linearises the map.  The cap's
// exact guards stay (cull when D + Rb < r_rx, everything when the receiver
// lies within Rb); on the receiver's vertical, or when 2m + 1 >= n_az, every
// column is covered.
__device__ __noinline__ ushort4 footprint_rect_fp64(float mx, float my, float mz, float rx, float ry, float rz,
                                                    const float *q_f, const float *ls_f, int n_az, int n_el,
                                                    float el_lo_f, float el_hi_f, float r_rx, int tw, int th,
                                                    int32_t nta) {
  const double ex = (double)mx - (double)rx;
  const double ey = (double)my - (double)ry;
  const double ez = (double)mz - (double)rz;
  const double rho2 = ex * ex + ey * ey;
  const double D2 = rho2 + ez * ez;
  const double D = sqrt(D2);
  const double l0 = ls_f[0], l1 = ls_f[1], l2 = ls_f[2];
  const double Rb = 3.0 * exp(fmax(fmax(l0, l1), l2));
  if (D + Rb < (double)r_rx * (1.0 - 1e-6)) return make_ushort4(0, 0, 0, 0);
  if (D <= Rb * (1.0 + 1e-6)) return tile_rect(0, n_el - 1, 0, n_az - 1, true, n_az, tw, th, nta);
  const double pi = 3.14159265358979323846;
  const double dalpha = 2.0 * pi / n_az;
  const double dbeta = ((double)el_hi_f - (double)el_lo_f) / n_el;
  const double rho = sqrt(rho2);
  double alpha = atan2(ey, ex);
  if (alpha < 0) alpha += 2.0 * pi;
  long u_k = (long)floor(alpha / dalpha);
  if (u_k > n_az - 1) u_k = n_az - 1;
  const long v_k = (long)floor((atan2(ez, rho) - (double)el_lo_f) / dbeta);
  long m;
  bool full;
  if (rho == 0.0) {
    m = n_el;
    full = true;
  } else {
    double w = q_f[0], x = q_f[1], y = q_f[2], z = q_f[3];
    const double qn = sqrt(w * w + x * x + y * y + z * z);
    w /= qn; x /= qn; y /= qn; z /= qn;
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    const double s2[3] = {exp(2.0 * l0), exp(2.0 * l1), exp(2.0 * l2)};
    // rows of J: d alpha / dx and d beta / dx in index units
    const double ja[3] = {-ey / rho2 / dalpha, ex / rho2 / dalpha, 0.0};
    const double jb[3] = {-ez * ex / (D2 * rho) / dbeta, -ez * ey / (D2 * rho) / dbeta, rho / D2 / dbeta};
    // J Sigma J^T = sum_i s_i^2 (J r_i)(J r_i)^T over the columns r_i of R
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = 0; i < 3; ++i) {
      const double pa = ja[0] * R[0][i] + ja[1] * R[1][i] + ja[2] * R[2][i];
      const double pb = jb[0] * R[0][i] + jb[1] * R[1][i] + jb[2] * R[2][i];
      a += s2[i] * pa * pa;
      b += s2[i] * pa * pb;
      c += s2[i] * pb * pb;
    }
    const double lam = 0.5 * (a + c) + sqrt(0.25 * (a - c) * (a - c) + b * b);
    const double r_k = 3.0 * sqrt(lam);
    m = (long)floor(fmin(r_k, 1e9));
    full = 2 * m + 1 >= n_az;
  }
  const long v_lo = v_k - m < 0 ? 0 : v_k - m;
  const long v_hi = v_k + m > n_el - 1 ? n_el - 1 : v_k + m;
  if (full) return tile_rect((int)v_lo, (int)v_hi, 0, n_az - 1, true, n_az, tw, th, nta);
  return tile_rect((int)v_lo, (int)v_hi, (int)(u_k - m), (int)(u_k + m), false, n_az, tw, th, nta);
}

// One record: depth key (always FP64: bits of fp32(D^2), D^2 without FMA)
// and an attempt at the rectangle in FP32; false when the FP64 evaluation
// is needed.
__device__ __forceinline__ bool project_record_fast(const gsrf_pair &pr, float4 mu, float Rb, const gsrf_grid &grid,
                                                    int32_t nta, uint32_t *key_out, ushort4 *rect) {
  const double ex = (double)mu.x - (double)pr.rx[0];
  const double ey = (double)mu.y - (double)pr.rx[1];
  const double ez = (double)mu.z - (double)pr.rx[2];
  const double D2 = (ex * ex + ey * ey) + ez * ez;
  *key_out = __float_as_uint((float)D2);
  return cap_rect_fp32((float)ex, (float)ey, (float)ez, sqrtf((float)D2), Rb, grid, nta, rect);
}

// Workgroup = C chunks of RB consecutive records of one pair (C = 1, or 4 for
// large batches, where emit's workgroup takes 4 x 256 records and so shares
// one sub-bucket with all four): each chunk's keys and rectangles in FP32, then
// one FP64 pass, packed onto the first lanes, for every record of the C chunks
// that the FP32 evaluation could not decide (about 1 %: nearly every 256-record
// chunk has one, so evaluating them chunk by chunk cost a whole wave pass per
// chunk); then per chunk a balanced expansion of the rectangles into the
// per-tile counts in LDS, and one atomic per touched tile on the workgroup's
// sub-bucket counter.  The sub-bucket of a record is (record index / emit's
// workgroup size) % kSub, so this kernel counts into the sub-bucket from which
// emit's workgroup of the same records later reserves: sub_shift =
// log2(emit workgroup / (C RB)).
// FOOT: bin by the paper's footprint (grid.footprint = 1) instead of the cap.
template <int RB, bool FOOT, int C = 1>
__global__ __launch_bounds__(RB) void k_project(const gsrf_pair *__restrict__ pairs,
                                                 const int64_t *__restrict__ scene_off,
                                                 const int64_t *__restrict__ rec_base, const float *__restrict__ prep,
                                                 const float *__restrict__ quats, const float *__restrict__ log_scales,
                                                 gsrf_grid grid, int32_t nta,
                                                 int32_t T, int64_t PT, int sub_shift, uint32_t *__restrict__ rec_key,
                                                 ushort4 *__restrict__ rec_rect, uint32_t *__restrict__ tile_cnt) {
  extern __shared__ uint32_t hist[];   // [T]
  __shared__ RectScan<RB> rs;
  __shared__ ushort4 rects[C * RB];
  __shared__ int fallback[C * RB];
  __shared__ int n_fallback;
  const int k = blockIdx.y;
  const gsrf_pair pr = pairs[k];
  const int64_t g0 = scene_off[pr.scene];
  const int64_t n = scene_off[pr.scene + 1] - g0;
  const int64_t j0 = (int64_t)blockIdx.x * (C * RB);   // the workgroup's first record
  if (C > 1 && j0 >= n) return;                        // (uniform)
  for (int t = threadIdx.x; t < T; t += blockDim.x) hist[t] = 0;
  if (threadIdx.x == 0) n_fallback = 0;
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    const int64_t j = j0 + c * RB + threadIdx.x;
    ushort4 rc = make_ushort4(0, 0, 0, 0);
    if (j < n) {
      uint32_t key;
      const float4 *pg = (const float4 *)(prep + (size_t)kPrep * (g0 + j));   // (mu, N) ... (3 max s, max log s)
      if (!project_record_fast(pr, pg[0], pg[3].x, grid, nta, &key, &rc) || FOOT)
        fallback[atomicAdd(&n_fallback, 1)] = c * RB + threadIdx.x;
      rec_key[rec_base[k] + j] = key;
    }
    rects[c * RB + threadIdx.x] = rc;
  }
  __syncthreads();
  // records the FP32 evaluation could not decide, packed onto the first lanes
  for (int i = threadIdx.x; i < n_fallback; i += RB) {
    const int slot = fallback[i];
    const float *pg = prep + (size_t)kPrep * (g0 + j0 + slot);
    const int64_t g = g0 + j0 + slot;
    if constexpr (FOOT) {
      rects[slot] = footprint_rect_fp64(pg[0], pg[1], pg[2], pr.rx[0], pr.rx[1], pr.rx[2], quats + 4 * g,
                                        log_scales + 3 * g, grid.n_az, grid.n_el, grid.el_lo, grid.el_hi,
                                        grid.r_rx, grid.tile_w, grid.tile_h, nta);
      continue;
    }
    rects[slot] = cap_rect_fp64(pg[0], pg[1], pg[2], pr.rx[0], pr.rx[1], pr.rx[2], pg[13], grid.n_az, grid.n_el,
                                grid.el_lo, grid.el_hi, grid.r_rx, grid.tile_w, grid.tile_h, nta);
  }
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    const int64_t j = j0 + c * RB + threadIdx.x;
    const ushort4 rc = rects[c * RB + threadIdx.x];
    if (j < n) rec_rect[rec_base[k] + j] = rc;
    rect_scan(rs, rc);
    const uint32_t total = rs.off[RB];
    rect_for_each(rs, total, nta, [&](uint32_t, int, int t) { atomicAdd(&hist[t], 1u); });
    __syncthreads();   // (the next chunk's scan rewrites rs)
  }
  uint32_t *dst = tile_cnt + (size_t)((((int64_t)blockIdx.x * C) >> sub_shift) % kSub) * PT + (size_t)k * T;
  for (int t = threadIdx.x; t < T; t += blockDim.x)
    if (hist[t]) atomicAdd(dst + t, hist[t]);
}
#pragma clang fp contract(on)

// Exclusive scan of the per-(tile, sub-bucket) counts of all pairs, in three
// launches over blocks of kScanTiles tiles: block totals, a scan of the block
// totals (which also stores the splat total and the overflow flag), and the
// per-block scan that writes the tile ranges and the sub-bucket starts
// (emission cursors).  When the total exceeds the capacity every range is
// left empty, so nothing downstream reads past it.
__device__ __forceinline__ int64_t block_sum_256(int64_t x, int64_t *sh) {
  const int tid = threadIdx.x;
  sh[tid] = x;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) sh[tid] += sh[tid + off];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *__restrict__ tile_cnt, int64_t PT,
                                                     int64_t *__restrict__ blk) {
  __shared__ int64_t sh[256];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTiles;
  int64_t local = 0;
#pragma unroll
  for (int i = 0; i < kScanTiles / 256; ++i) {
    const int64_t t = t0 + i * 256 + threadIdx.x;
    if (t < PT)
      for (int b = 0; b < kSub; ++b) local += tile_cnt[(size_t)b * PT + t];
  }
  const int64_t tot = block_sum_256(local, sh);
  if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_blocks(int64_t *__restrict__ blk, int64_t nblk, int64_t cap,
                                                      int64_t *__restrict__ counters) {
  __shared__ int64_t sh[1024];
  const int tid = threadIdx.x;
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nblk; c0 += 1024) {
    const int64_t i = c0 + tid;
    const int64_t x = i < nblk ? blk[i] : 0;
    sh[tid] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int64_t y = tid >= off ? sh[tid - off] : 0;
      __syncthreads();
      sh[tid] += y;
      __syncthreads();
    }
    if (i < nblk) blk[i] = carry + sh[tid] - x;
    carry += sh[1023];
    __syncthreads();
  }
  if (tid == 0) {
    counters[0] = carry;
    counters[1] = carry > cap ? carry : 0;
  }
}

// blk == null: the only block (P * T <= kScanTiles) also makes the total and
// the overflow flag, so the first two passes are skipped.
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *__restrict__ tile_cnt, int64_t PT,
                                                    const int64_t *__restrict__ blk, int64_t cap,
                                                    int64_t *__restrict__ counters,
                                                    uint32_t *__restrict__ tstart, uint32_t *__restrict__ tend,
                                                    uint32_t *__restrict__ tcur, uint32_t *__restrict__ long_q,
                                                    LongClasses lc) {
  __shared__ int64_t sh[256];
  __shared__ uint32_t s_cls[kLongClasses], s_base[kLongClasses];
  constexpr int PER = kScanTiles / 256;
  const int tid = threadIdx.x;
  if (tid < kLongClasses) s_cls[tid] = 0u;
  const int64_t t0 = (int64_t)blockIdx.x * kScanTiles + (int64_t)tid * PER;
  uint32_t cnt[PER][kSub];
  int64_t local = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i)
#pragma unroll
    for (int b = 0; b < kSub; ++b) {
      cnt[i][b] = (t0 + i < PT) ? tile_cnt[(size_t)b * PT + t0 + i] : 0u;
      local += cnt[i][b];
    }
  sh[tid] = local;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t y = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += y;
    __syncthreads();
  }
  bool over;
  int64_t run;
  if (blk) {
    over = counters[1] != 0;
    run = blk[blockIdx.x] + sh[tid] - local;
  } else {
    const int64_t total = sh[255];
    over = total > cap;
    run = sh[tid] - local;
    if (tid == 0) {
      counters[0] = total;
      counters[1] = over ? total : 0;
    }
  }
  const int64_t run0 = run;
  int cls[PER];
  uint32_t lpos[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) cls[i] = -1;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int64_t t = t0 + i;
    if (t >= PT) break;
    tstart[t] = over ? 0u : (uint32_t)run;
    const int64_t r0 = run;
#pragma unroll
    for (int b = 0; b < kSub; ++b) {
      tcur[(size_t)b * PT + t] = over ? 0u : (uint32_t)run;   // emission cursor of the sub-bucket
      run += cnt[i][b];
    }
    tend[t] = over ? 0u : (uint32_t)run;
    const int64_t n = over ? 0 : run - r0;
    if (long_q && n > lc.lo) {   // a long bucket: its length class, and its place in this block's share
      int c = 0;
#pragma unroll
      for (int k = 1; k < kLongClasses; ++k) c += (k < lc.n && n <= lc.thr[k]) ? 1 : 0;
      cls[i] = c;
      lpos[i] = atomicAdd(&s_cls[c], 1u);
    }
  }
  if (!long_q) return;
  __syncthreads();
  if (tid < lc.n && s_cls[tid] != 0u) s_base[tid] = atomicAdd(&long_q[tid], s_cls[tid]);
  __syncthreads();
  uint2 *lists = (uint2 *)(long_q + kLongQueueHeader);
  int64_t r = run0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    uint32_t n = 0;
#pragma unroll
    for (int b = 0; b < kSub; ++b) n += cnt[i][b];
    if (cls[i] >= 0) lists[(size_t)cls[i] * PT + s_base[cls[i]] + lpos[i]] = make_uint2((uint32_t)r, n);
    r += n;
  }
}

hipError_t launch_project(const gsrf_problem *p, const Layout &lay, char *ws, hipStream_t s) {
  float *prep = (float *)(ws + lay.prep);
  int64_t *rec_base = (int64_t *)(ws + lay.rec_base);
  const int64_t PT = (int64_t)p->n_pairs * lay.T;
  uint32_t *tile_cnt = (uint32_t *)(ws + lay.tile_cnt);
  // the long-bucket queue of a tiered sort: header cleared by k_activate,
  // lists filled by k_scan_apply
  uint32_t *long_q = PT > kSortFewTiles ? (uint32_t *)(ws + lay.long_q) : nullptr;
  const LongClasses lc = long_q ? long_classes() : LongClasses{};
  {
    const gsrf_grid &g = p->grid;
    int64_t nb = (p->n_gauss + 255) / 256 + ((int64_t)g.n_az * g.n_el + 255) / 256;
    const int64_t nb_cnt = (PT * kSub + 255) / 256;   // the counters are cleared grid-stride
    if (nb_cnt > nb) nb = nb_cnt < 4096 ? nb_cnt : 4096;
    if (nb < 1) nb = 1;
    float *rays = (float *)(ws + lay.rays);
#define GSRF_ACTIVATE(LL)                                                                                           \
  hipLaunchKernelGGL(k_activate<LL>, dim3((unsigned)nb), dim3(256), 0, s, p->means, p->log_scales, p->quats,         \
                     p->opacity_logits, p->n_gauss, prep, tile_cnt, PT * kSub, p->pairs, p->scene_offsets_dev,       \
                     p->n_pairs, rec_base, g.n_az, g.n_el, g.el_lo, g.el_hi, rays, long_q)
    switch (g.fle_L) {
      case 0: GSRF_ACTIVATE(0); break;
      case 1: GSRF_ACTIVATE(1); break;
      case 2: GSRF_ACTIVATE(2); break;
      case 3: GSRF_ACTIVATE(3); break;
      case 4: GSRF_ACTIVATE(4); break;
      case 5: GSRF_ACTIVATE(5); break;
      default: GSRF_ACTIVATE(6); break;
    }
#undef GSRF_ACTIVATE
  }
  if (lay.n_records > 0) {
    const int sub_shift = lay.rec_block == 1024 ? 2 : 0;   // emit's workgroup = 256 << sub_shift records
    dim3 grid((unsigned)((lay.max_scene + 255) / 256), (unsigned)p->n_pairs);
    if (p->grid.footprint)
      hipLaunchKernelGGL((k_project<256, true>), grid, dim3(256), (size_t)lay.T * 4, s, p->pairs, p->scene_offsets_dev,
                         rec_base, (const float *)prep, p->quats, p->log_scales, p->grid, lay.nta, lay.T, PT, sub_shift,
                         (uint32_t *)(ws + lay.rec_key), (ushort4 *)(ws + lay.rec_rect), tile_cnt);
    else if (lay.rec_block == 1024)   // four 256-record chunks per workgroup: emit's 1024 records
      hipLaunchKernelGGL((k_project<256, false, 4>), dim3((unsigned)((lay.max_scene + 1023) / 1024), (unsigned)p->n_pairs),
                         dim3(256), (size_t)lay.T * 4, s, p->pairs, p->scene_offsets_dev, rec_base, (const float *)prep,
                         p->quats, p->log_scales, p->grid, lay.nta, lay.T, PT, sub_shift,
                         (uint32_t *)(ws + lay.rec_key), (ushort4 *)(ws + lay.rec_rect), tile_cnt);
    else
      hipLaunchKernelGGL((k_project<256, false>), grid, dim3(256), (size_t)lay.T * 4, s, p->pairs, p->scene_offsets_dev,
                         rec_base, (const float *)prep, p->quats, p->log_scales, p->grid, lay.nta, lay.T, PT, sub_shift,
                         (uint32_t *)(ws + lay.rec_key), (ushort4 *)(ws + lay.rec_rect), tile_cnt);
  }
  int64_t *blk = (int64_t *)(ws + lay.scan_blk);
  int64_t *counters = (int64_t *)(ws + lay.counters);
  const int64_t nblk = (PT + kScanTiles - 1) / kScanTiles;
  if (nblk <= 1) {
    // one block: counts, total and ranges in a single launch (also P * T = 0)
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(256), 0, s, tile_cnt, PT, (const int64_t *)nullptr, lay.cap,
                       counters, (uint32_t *)(ws + lay.tile_start), (uint32_t *)(ws + lay.tile_end),
                       (uint32_t *)(ws + lay.tile_cur), long_q, lc);
  } else {
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nblk), dim3(256), 0, s, tile_cnt, PT, blk);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, blk, nblk, lay.cap, counters);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nblk), dim3(256), 0, s, tile_cnt, PT, (const int64_t *)blk,
                       lay.cap, counters, (uint32_t *)(ws + lay.tile_start), (uint32_t *)(ws + lay.tile_end),
                       (uint32_t *)(ws + lay.tile_cur), long_q, lc);
  }
  return hipGetLastError();
}

}  // namespace gsrf
