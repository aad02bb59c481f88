// Two-phase traversal of a tile's depth-ordered list (256 threads per
// (pair, tile), R = 32, 64, 128 or 256 rays), used by both the forward renderer
// (Sec. 3.4 eq. rendering; App. A) and its adjoint (App. C; App. D).
//
// Only about one in six (ray, list entry) tests is a processed hit, so doing
// the per-hit work where the test is made leaves most lanes idle.  Per staged
// batch:
//   phase 1  dense hit tests: thread t takes ray t % R against entries
//            e, e + EP, ... (e = t / R, EP = 256 / R) and ORs the hits into
//            per-ray bit rows in LDS, and into the union row of the phase-2
//            wave that serves the ray.  The forward also stores each list
//            entry's hits as an R-bit mask in the workspace; the adjoint
//            rebuilds its rows from those masks instead of testing again
//            (the same decisions, for the rays still active);
//   phase 2  each wave serves 64 / G rays with G = 256 / R adjacent lanes per
//            ray and walks the union of its rays' hit bits in depth order, G
//            entries per step (a wave-uniform scalar cursor).  A lane does the
//            per-hit work only where its ray hits its entry; the G-lane
//            product scan gives each hit its incoming transmittance
//            T_j = T * prod(1 - alpha) over the earlier hits, so "process hit
//            j iff T_j >= t_min" is decided per hit as in the sequential
//            definition.  Because the lanes sharing q meet the same entry,
//            the adjoint sums a step's contributions over the wave's rays by
//            a register reduce-scatter instead of LDS atomics (walking each
//            ray's own bits would put neighbouring rays on one Gaussian in
//            the same step).
#pragma once

#include "render_common.h"

namespace gsrf {

// kTpFwdMulti / kTpFwdMultiWide: the forward for 16 / 32 carriers
// f_c = f_0 + c * step at once (OFDM subcarriers; Sec. 4 5G CSI synthesis):
// hit decisions, alpha, p and psi do not depend on the carrier, only the
// propagation phase does, so one traversal accumulates every carrier (the
// phase factor of carrier c + 1 is that of carrier c times the step's).  The
// wide form holds twice the accumulators at half the occupancy; it pays when
// more than 16 carriers remain.
// kTpCount / kTpCollect: the two passes of the per-ray midpoint order
// (App. A.3): phase-1 tests over the whole list without termination, writing
// the entry masks and counting each ray's hits; then, from those masks, one
// record per hit (t_mid, transmittance factor, T-free contribution) at the
// ray's offset, for a per-ray sort and composite.
// Midpoint-order sort key: t_mid in units of 2^-24 m (t clamped to
// [0, 2^16) m) above a 24-bit rank of the hit in list order.
constexpr int kTmidRankBits = 24;
constexpr uint64_t kTmidRankMask = ((uint64_t)1 << kTmidRankBits) - 1;
constexpr double kTmidKeyScale = 16777216.0;                 // 2^24 per metre
constexpr double kTmidMaxT = 65536.0 - 1.0 / 16777216.0;
enum TpMode { kTpFwd = 0, kTpFwdStats = 1, kTpBwd = 2, kTpFwdMulti = 3, kTpFwdMultiWide = 4, kTpCount = 5,
              kTpCollect = 6, kTpMultiTotal = 7, kTpBwdMulti = 8 };
constexpr int kMultiChunk = 16, kMultiChunkWide = 32;
// kTpMultiTotal / kTpBwdMulti: the adjoint for kGcChunk carriers at once
// (OFDM subcarriers, Sec. 4) over the forward's hit masks.  The total pass
// walks each ray's processed hits and sums w_i = T_i Re(conj(Ge_i) c~_i) in
// FP64 -- sum_c Re(conj(G_c) S_c) of the ray, Ge_i = sum_c G_c e^{j c delta_i}
// (adj_hit_multi) -- which the adjoint pass then uses for the remainders
// sum_{i>j} w_i = total - prefix_j, as the one-carrier adjoint uses S.  The
// carriers' dL/dS of the tile's rays are held in LDS.
constexpr int kGcChunk = 16;
constexpr int multi_chunk(int mode) {
  return mode == kTpFwdMulti ? kMultiChunk : mode == kTpFwdMultiWide ? kMultiChunkWide : 1;
}

template <int R>
struct TwoPhase {
  static constexpr int NT = 256;
  static constexpr int EP = NT / R;        // entry phases (phase 1): thread t takes ray t % R, entries t / R + k EP
  static constexpr int G = NT / R;         // lanes per ray (phase 2)
  static constexpr int RPW = 64 / G;       // rays per wave (phase 2)
};

struct TpIO {
  float2 *signal;                 // forward output S [P, n_el, n_az]
  double2 *sig64;                 // S in FP64 (forward writes, adjoint reads): the remainders
                                  // S - prefix stay accurate to the size of the remainder
  float2 *tile_sum;               // forward: per-(pair, tile) partial of S_hat
  unsigned long long *stats;      // forward with counters: tests, hits, staged, rays, tile tests, walk slots
  float2 *multi;                  // multi-carrier: S [P, n_freq, n_el, n_az]
  int n_freq, f_first;            // multi-carrier: carriers in all, first carrier of this launch
  double f_step;                  // multi-carrier: carrier step (Hz)
  const float2 *grad_signal;      // adjoint: dL/dS
  const float2 *grad_sum;         // adjoint: dL/dS_hat per pair, or null
  float *acc;                     // adjoint accumulators [n_gauss][acc_stride]
  int acc_stride;
  uint32_t *ray_cnt;              // midpoint order: hits per ray [P, n_el, n_az]
  const uint64_t *ray_off;        // midpoint order: first record of each ray
  uint64_t *hit_key;              // midpoint order: (t_mid key << 24 | hit rank) per record
  float4 *hit_val;                // midpoint order: (keep, Re, Im of p psi e^{-j phi}, -) per record
  const int64_t *counters;        // [3] = records over capacity (collect writes nothing then)
  // several-carrier adjoint (io.n_freq carriers, io.f_first the chunk's first)
  const float2 *grad_multi;       // dL/dS [P, n_freq, n_el, n_az]
  const float2 *grad_sum_multi;   // dL/dS_hat [P, n_freq], or null
  double *wtot;                   // per ray: sum_c Re(conj(G_c) S_c) of the chunk (total pass writes)
};

// LDS words of a masked pass's batch fill: entry count, first position left
// over, per-wave counts (up to 4 waves), active-ray words (up to 8).
constexpr int kFillWords = 16;

// BCAP: largest staged batch (128).  Smaller batches waste fewer tests past
// the rays' termination (the last batch is tested whole), larger ones need
// fewer barriers.
template <int L, int R, int MODE, int BCAP>
struct TpShape {
  static constexpr bool BWD = MODE == kTpBwd || MODE == kTpBwdMulti;     // adjoint (accumulators)
  static constexpr bool GC = MODE == kTpBwdMulti || MODE == kTpMultiTotal;   // carriers' dL/dS in LDS
  // hit decisions taken from the forward's masks (adjoint, total pass, midpoint collect)
  static constexpr bool MASKED = BWD || MODE == kTpCollect || MODE == kTpMultiTotal;
  static constexpr int K = (L + 1) * (L + 1);
  static constexpr int B = lds_batch(L, 256, BWD, BCAP);
  static constexpr int NACC = n_acc(L);
  static constexpr int MW = (B + 31) / 32;       // mask words per row
  static constexpr int MWS = MW + 1;             // odd row stride: conflict-free column reads
  static constexpr int MWR = R / 32;             // hit-mask words per entry (one bit per ray)
  // LDS: geometry, [TX legs], coefficients, [accumulators, flags], ray rows, union rows, done flags
  static constexpr size_t kLds = (size_t)B * (kGeo * 16 + 2 * K * 4) + (BWD ? (size_t)B * (16 + NACC * 4 + 4) : 0) +
                                 (size_t)R * MWS * 4 + (size_t)4 * MW * 4 + (size_t)R * 4 +
                                 (GC ? (size_t)R * kGcChunk * 8 : 0) +
                                 (MASKED ? (size_t)(B * (MWR + 1) + kFillWords) * 4 : 0);
  static constexpr size_t lds() { return kLds < 256 * 8 ? 256 * 8 : kLds; }
};

// Phase-1 hit test of ray v against a staged Gaussian: the decision of
// test_hit (Q <= 9 and t >= r_rx) with A = v^T M v taken from the ray's
// quadratic monomials and b = v . (M eps), which needs no M v (34 VALU
// operations instead of 40).  The per-hit terms are recomputed by test_hit
// in phase 2; only the decision is taken here, in both the forward and the
// adjoint, so the two passes agree on every hit.
struct RayMono {
  float x, y, z, xx, yy, zz, xy2, xz2, yz2;
};

__device__ __forceinline__ RayMono ray_mono(float x, float y, float z) {
  return RayMono{x, y, z, x * x, y * y, z * z, 2.f * x * y, 2.f * x * z, 2.f * y * z};
}

__device__ __forceinline__ bool hit_decision(const RayMono &v, const float4 *geo, float r_rx) {
  const float4 g0 = geo[0], g1 = geo[1], g2 = geo[2], g3 = geo[3];
  const float ex = (v.x - g0.x) - g1.x, ey = (v.y - g0.y) - g1.y, ez = (v.z - g0.z) - g1.z;
  const float m00 = g2.x, m11 = g2.y, m22 = g2.z, m01 = g2.w, m02 = g3.x, m12 = g3.y;
  const float n0 = fmaf(m00, ex, fmaf(m01, ey, m02 * ez));
  const float n1 = fmaf(m01, ex, fmaf(m11, ey, m12 * ez));
  const float n2 = fmaf(m02, ex, fmaf(m12, ey, m22 * ez));
  const float A = fmaf(m00, v.xx, fmaf(m11, v.yy, fmaf(m22, v.zz, fmaf(m01, v.xy2, fmaf(m02, v.xz2, m12 * v.yz2)))));
  const float b = fmaf(v.x, n0, fmaf(v.y, n1, v.z * n2));
  const float c = fmaf(ex, n0, fmaf(ey, n1, ez * n2));
  const float bA = b * __builtin_amdgcn_rcpf(A);
  const float Q = geo[4].y * fmaf(-b, bA, c);
  const float t = fmaf(-g0.w, bA, g0.w);
  return (Q <= kLevel) && (t >= r_rx);
}

// 32 x 32 bit transpose across the 32 lanes of a half-wave: on return lane l
// holds, as bit i, bit l of lane i's input.  Five exchanges at lane distances
// 16, 8, 4, 2, 1, each swapping the off-diagonal blocks of that size.
template <int J>
__device__ __forceinline__ uint32_t transpose_step(uint32_t x, int lane, uint32_t m) {
  const uint32_t y = __float_as_uint(xor_lane<J>(__uint_as_float(x), lane));
  return (lane & J) ? ((x & ~m) | ((y >> J) & m)) : ((x & m) | ((y << J) & ~m));
}

__device__ __forceinline__ uint32_t transpose32(uint32_t x, int lane) {
  x = transpose_step<16>(x, lane, 0x0000FFFFu);
  x = transpose_step<8>(x, lane, 0x00FF00FFu);
  x = transpose_step<4>(x, lane, 0x0F0F0F0Fu);
  x = transpose_step<2>(x, lane, 0x33333333u);
  x = transpose_step<1>(x, lane, 0x55555555u);
  return x;
}

// Phase 1: hit bits of ray v against entries e, e + EP, ... < nb, one 32-entry
// word at a time (32 / EP tests unrolled per word).
template <int EP, int MW>
__device__ __forceinline__ unsigned phase1_tests(const RayMono &v, const float4 *sgeo, int nb, int e, float r_rx,
                                                 uint32_t *mask_row, uint32_t *uni_row) {
  unsigned n_test = 0;
#pragma unroll 1
  for (int w = 0; w < MW; ++w) {
    const int j0 = w * 32;
    if (j0 >= nb) break;
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < 32 / EP; ++i) {
      const int jj = j0 + e + i * EP;
      if (jj < nb) {
        ++n_test;
        if (hit_decision(v, sgeo + kGeo * jj, r_rx)) bits |= 1u << (jj & 31);
      }
    }
    if (bits) {
      atomicOr(mask_row + w, bits);
      atomicOr(uni_row + w, bits);
    }
  }
  return n_test;
}

// The next batch of a pass that takes its hit decisions from the forward's
// masks.  About a third of the list entries the forward stages hit any of the
// tile's rays (the binning rectangles are conservative boxes around caps, and
// the rays are a sparse grid), so such a pass stages only the entries whose
// forward mask has a bit on a ray still active:
// the workgroup scans the list from `pos`, KS entries per thread per step, keeps
// those entries in list order (their mask words in smw, Gaussian ids in sval) up
// to B of them, and leaves `pos` at the first entry not taken.  The hits of every
// ray are the same, in the same order, as over the whole list.  Masks past the
// forward's end for a ray block (mend, at most s1) count as empty: the forward
// stops once all its rays have terminated and writes no masks beyond.  Returns
// the batch's entry count (0: the list holds no further hit on an active ray).
template <int R, int B, int MWR, int SPLIT>
__device__ __forceinline__ int fill_masked(const RenderArgs &a, uint32_t &pos, uint32_t s1, const uint32_t *mend,
                                           int half, const int *sdone, uint32_t *smw, uint32_t *sval,
                                           uint32_t *sfill) {
  constexpr int NT = 256, KS = 4, W = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t *swc = sfill + 2, *sact = sfill + 2 + W;
  {
    const bool act = tid < R && !sdone[tid < R ? tid : 0];
    const uint64_t bm = __ballot(act);
    if (lane == 0 && 2 * wave < MWR) {
      sact[2 * wave] = (uint32_t)bm;
      if (2 * wave + 1 < MWR) sact[2 * wave + 1] = (uint32_t)(bm >> 32);
    }
  }
  __syncthreads();
  uint32_t act[MWR];
#pragma unroll
  for (int rb = 0; rb < MWR; ++rb) act[rb] = sact[rb];
  int nb = 0;
  while (nb < B && pos < s1) {   // (nb and pos stay uniform)
    const uint32_t p0 = pos + (uint32_t)tid * KS;
    uint32_t mw[KS][MWR], gv[KS], take = 0;
#pragma unroll
    for (int e = 0; e < KS; ++e) {
      const uint32_t p = p0 + e;
      gv[e] = 0u;
      uint32_t any = 0u;
#pragma unroll
      for (int rb = 0; rb < MWR; ++rb) {
        mw[e][rb] = p < mend[rb] ? a.hitmask[(size_t)p * (MWR * SPLIT) + half * MWR + rb] : 0u;
        any |= mw[e][rb] & act[rb];
      }
      if (p < s1) gv[e] = a.val[p];
      if (any) take |= 1u << e;
    }
    const int c = __builtin_popcount(take);
    int incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) swc[wave] = (uint32_t)incl;
    __syncthreads();
    int woff = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int x = (int)swc[w];
      woff += w < wave ? x : 0;
      tot += x;
    }
    int slot = nb + woff + incl - c;
#pragma unroll
    for (int e = 0; e < KS; ++e)
      if ((take >> e) & 1u) {
        if (slot < B) {
#pragma unroll
          for (int rb = 0; rb < MWR; ++rb) smw[slot * MWR + rb] = mw[e][rb];
          sval[slot] = gv[e];
        } else if (slot == B) {
          sfill[1] = p0 + e;   // the first entry left for the next batch
        }
        ++slot;
      }
    __syncthreads();
    if (nb + tot > B) {
      pos = sfill[1];
      nb = B;
    } else {
      pos += (uint32_t)(KS * NT);
      nb += tot;
    }
  }
  return nb;
}

// SPLIT = 2: the bin tile (2R rays) is rendered by two workgroups, each taking
// R rays (the upper or lower half of the tile's rows) over the whole list;
// forward launches with few tiles use it to double the waves in flight.  The
// hit masks have the same layout either way (ray r of the tile is bit r % 32
// of word r / 32), so the adjoint need not split as the forward did.
template <int L, int R, int MODE, int BCAP, int SPLIT, bool VAR = false>
__global__ __launch_bounds__(256) void k_render_tp(RenderArgs a, TpIO io) {
  using TP = TwoPhase<R>;
  using SH = TpShape<L, R, MODE, BCAP>;
  constexpr int FC = multi_chunk(MODE);
  constexpr bool BWD = SH::BWD, STATS = MODE == kTpFwdStats, MULTI = FC > 1;
  constexpr bool COUNT = MODE == kTpCount, COLLECT = MODE == kTpCollect;
  constexpr bool GC = SH::GC, MTOT = MODE == kTpMultiTotal, BMULTI = MODE == kTpBwdMulti;
  constexpr bool MASKED = SH::MASKED;   // hit decisions from the forward's masks
  if constexpr (COLLECT)
    if (io.counters[3] != 0) return;           // records over capacity: the whole launch writes nothing
  constexpr int NT = TP::NT, G = TP::G, EP = TP::EP, RPW = TP::RPW;
  constexpr int K = SH::K, B = SH::B, NACC = SH::NACC, MW = SH::MW, MWS = SH::MWS;
  constexpr int NV = pow2_at_least(NACC);
  extern __shared__ float4 smem[];
  float4 *sgeo = smem;                                      // [B][kGeo]
  float4 *stx = smem + kGeo * B;                            // [B]         (adjoint: TX leg, Gaussian id)
  float *scf = (float *)(stx + (BWD ? B : 0));              // [B][2K]
  float *sacc = scf + 2 * K * B;                            // [B][NACC]   (adjoint)
  uint32_t *sflag = (uint32_t *)(sacc + (BWD ? NACC * B : 0));  // [B]    (adjoint)
  uint32_t *smask = (uint32_t *)(sflag + (BWD ? B : 0));    // [R][MWS]
  uint32_t *suni = smask + R * MWS;                         // [4][MW]
  int *sdone = (int *)(suni + 4 * MW);                      // [R]
  float2 *sgc = (float2 *)(sdone + R);                      // [R][kGcChunk] (several-carrier adjoint)
  uint32_t *smw = (uint32_t *)(sgc + (GC ? R * kGcChunk : 0));   // [B][MWR] batch's mask words (masked passes)
  uint32_t *sval = smw + B * SH::MWR;                             // [B] batch's Gaussian ids (masked passes)
  uint32_t *sfill = sval + B;                                     // [kFillWords] batch fill state (masked passes)
  constexpr int MWR = SH::MWR;
  const int gt = blockIdx.x;                 // (pair, tile, half)
  const int gtile = gt / SPLIT, half = gt - gtile * SPLIT;
  const int k = gtile / a.T;
  const int tile = gtile - k * a.T;
  const int tv = tile / a.nta, tu = tile - tv * a.nta;
  const int th_ = R / a.tw;                  // rows of this workgroup
  const int v0 = (tv * SPLIT + half) * th_;  // its first row
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // phase-2 identity: ray r, lane q of its group
  const int r = tid / G, q = tid % G;
  const int u = tu * a.tw + r % a.tw, v = v0 + r / a.tw;
  const bool valid = (u < a.n_az) && (v < a.n_el);
  // phase-1 identity: ray r1, entry phase e
  const int r1 = tid % R, e = tid / R;
  const int u1 = tu * a.tw + r1 % a.tw, v1 = v0 + r1 / a.tw;
  const bool valid1 = (u1 < a.n_az) && (v1 < a.n_el);
  const gsrf_pair pr = a.pairs[k];
  // (multi-carrier: the launch's first carrier)
  const double freq = (MULTI || GC) ? pr.freq_hz + io.f_first * io.f_step : pr.freq_hz;
  const double lam = kC0 / freq, inv_lam = freq / kC0;
  const double step_rev = (MULTI || GC) ? io.f_step / kC0 : 0.0;
  float mr[FC], mi[FC];   // multi-carrier accumulators
#pragma unroll
  for (int c = 0; c < FC; ++c) mr[c] = mi[c] = 0.f;
  float vx = 0.f, vy = 0.f, vz = 1.f, Yr[K], Yi[K];
  ray_load<L>(valid ? u : 0, valid ? v : 0, a, vx, vy, vz, Yr, Yi);
  RayMono w1;
  {
    float wx, wy, wz;
    ray_load_dir(valid1 ? u1 : 0, valid1 ? v1 : 0, a, K, wx, wy, wz);
    w1 = ray_mono(wx, wy, wz);
  }
  float twopi_lam = 0.f, twopi_dlam = 0.f, Gr = 0.f, Gi = 0.f;
  double Sfr = 0.0, Sfi = 0.0;
  if constexpr (GC) {
    // the chunk's carriers' dL/dS (+ dL/dS_hat) of the tile's rays; zero past the last carrier
    const int nc = min(kGcChunk, io.n_freq - io.f_first);
    for (int i = tid; i < R * kGcChunk; i += NT) {
      const int rr = i / kGcChunk, c = i - rr * kGcChunk;
      const int uu = tu * a.tw + rr % a.tw, vv = v0 + rr / a.tw;
      float2 gv = make_float2(0.f, 0.f);
      if (c < nc && uu < a.n_az && vv < a.n_el) {
        const size_t kc = (size_t)k * io.n_freq + io.f_first + c;
        gv = io.grad_multi[(kc * a.n_el + vv) * a.n_az + uu];
        if (io.grad_sum_multi) {
          const float2 gs = io.grad_sum_multi[kc];
          gv.x += gs.x;
          gv.y += gs.y;
        }
      }
      sgc[i] = gv;
    }
    twopi_dlam = (float)(2.0 * 3.14159265358979323846 * io.f_step / kC0);
  }
  if constexpr (BMULTI) {
    twopi_lam = (float)(2.0 * 3.14159265358979323846 / lam);
    if (valid) Sfr = io.wtot[((size_t)k * a.n_el + v) * a.n_az + u];
    for (int i = tid; i < NACC * B; i += NT) sacc[i] = 0.f;
    for (int i = tid; i < B; i += NT) sflag[i] = 0u;
  } else if constexpr (BWD) {
    twopi_lam = (float)(2.0 * 3.14159265358979323846 / lam);
    if (valid) {
      const size_t ri = ((size_t)k * a.n_el + v) * a.n_az + u;
      const double2 sf = io.sig64[ri];
      const float2 gg = io.grad_signal[ri];
      Sfr = sf.x; Sfi = sf.y; Gr = gg.x; Gi = gg.y;
      if (io.grad_sum) {
        const float2 gs = io.grad_sum[k];
        Gr += gs.x;
        Gi += gs.y;
      }
    }
    for (int i = tid; i < NACC * B; i += NT) sacc[i] = 0.f;
    for (int i = tid; i < B; i += NT) sflag[i] = 0u;
  }
  const uint32_t s0 = a.tstart[gtile], s1 = v0 < a.n_el ? a.tend[gtile] : s0;   // a half below the grid: no rays
  // S (forward) and the prefix sum_{j<=i} T_j c~_j (adjoint) in FP64: each
  // term T_j c~_j is an exact FP64 product of two FP32 values, formed
  // identically by both passes, so R_i = S - prefix_i is accurate to ~1e-16 |S|
  // and vanishes with the remainder (the last hit of a ray)
  float T = 1.f;
  double Sr = 0.0, Si = 0.0, Pr = 0.0, Pi = 0.0;
  bool done = !valid || (1.0f < a.t_min);
  if (q == 0) sdone[r] = done ? 1 : 0;
  unsigned long long n_test = 0, n_hit = 0, n_staged = 0, n_tile_tests = 0, n_steps = 0;
  uint32_t n_ray_hits = 0;   // midpoint order: the ray's hits so far (count: phase-1 thread e = 0; collect: its G lanes)
  uint64_t ray_base = 0;
  if constexpr (COLLECT)
    if (valid) ray_base = io.ray_off[((size_t)k * a.n_el + v) * a.n_az + u];
  int n_valid_rays = 0;
  if constexpr (STATS) {
    const int tu_w = min(a.tw, a.n_az - tu * a.tw), tv_h = max(0, min(th_, a.n_el - v0));
    n_valid_rays = tu_w * tv_h;
  }
  // each staging thread's list entry for the next batch is loaded one batch
  // ahead, so staging waits for one global round trip (the entry's records), not two
  uint32_t g_next = (!MASKED && tid < B && s0 + tid < s1) ? a.val[s0 + tid] : 0u;
  uint32_t base = s0;   // the batch's first list entry (masked passes: the next entry to scan)
  uint32_t mend[MASKED ? MWR : 1];   // masked passes: the forward's end per ray block, at most s1
  uint32_t s1m = s0;
  if constexpr (MASKED) {
#pragma unroll
    for (int rb = 0; rb < MWR; ++rb) {
      mend[rb] = min(s1, a.mask_end[(size_t)gtile * (MWR * SPLIT) + half * MWR + rb]);
      s1m = max(s1m, mend[rb]);
    }
  }
  while (true) {
    int nb;
    if constexpr (MASKED) {
      __syncthreads();
      nb = fill_masked<R, B, MWR, SPLIT>(a, base, s1m, mend, half, sdone, smw, sval, sfill);
      if (nb == 0) break;
    } else {
      if (base >= s1) break;
      nb = (int)min((uint32_t)B, s1 - base);
    }
    __syncthreads();
    const uint32_t g_cur = MASKED ? (tid < nb ? sval[tid] : 0u) : g_next;
    if (tid < nb)
      stage_entry<K, MULTI || GC, VAR>(a, g_cur, pr.rx[0], pr.rx[1], pr.rx[2], pr.tx[0], pr.tx[1], pr.tx[2], inv_lam,
                                 sgeo + kGeo * tid, scf + 2 * K * tid, BWD ? stx + tid : nullptr, step_rev);
    if (!MASKED && tid < B && base + B + tid < s1) g_next = a.val[base + B + tid];
    if constexpr (BWD)
      for (int i = tid; i < nb; i += NT) {   // what the previous batch's flush left
        sflag[i] = 0u;
        sacc[NACC * i + NACC - 1] = 0.f;
      }
    if constexpr (!MASKED)
      for (int i = tid; i < R * MWS + 4 * MW; i += NT) smask[i] = 0u;   // ray rows and union rows

    if (STATS && tid == 0) {
      n_staged += nb;
      n_tile_tests += (unsigned long long)nb * n_valid_rays;
    }
    __syncthreads();
    // ---- phase 1: the forward tests; the adjoint takes the forward's hit masks ----
    if constexpr (!MASKED) {
      if (valid1 && !sdone[r1]) {
        const unsigned nt = phase1_tests<EP, MW>(w1, sgeo, nb, e, a.r_rx, smask + r1 * MWS, suni + (r1 / RPW) * MW);
        if (STATS) n_test += nt;
      }
      __syncthreads();
      if constexpr (COUNT) {
        if (e == 0 && valid1)
          for (int w = 0; w < MW; ++w) n_ray_hits += __builtin_popcount(smask[r1 * MWS + w]);
      }
      if constexpr (MODE == kTpFwd || COUNT) {
        // entry masks = transpose of the ray rows, one 32 x 32 bit block per
        // half-wave: block (ray block rb, entry word w); lane l of the half
        // reads ray 32 rb + l's row word and ends with entry 32 w + l's bits
        constexpr int NBLK = (R / 32) * MW;
        const int hl = lane & 31;
        for (int blk = (tid >> 5); blk < NBLK; blk += NT / 32) {
          const int rb = blk / MW, w = blk - rb * MW;
          const uint32_t m = transpose32(smask[(rb * 32 + hl) * MWS + w], hl);
          const int j = w * 32 + hl;
          if (j < nb) a.hitmask[(size_t)(base + j) * (MWR * SPLIT) + half * MWR + rb] = m;
        }
      }
    } else {
      // (the adjoint, and the midpoint order's collect pass) the forward's
      // entry masks, transposed back into the rows of the rays still active;
      // then the union rows of the phase-2 waves
      constexpr int NBLK = (R / 32) * MW;
      const int hl = lane & 31;
      for (int blk = (tid >> 5); blk < NBLK; blk += NT / 32) {
        const int rb = blk / MW, w = blk - rb * MW;
        const int j = w * 32 + hl;
        const uint32_t m = j < nb ? smw[j * MWR + rb] : 0u;
        const uint32_t row = transpose32(m, hl);
        const int rr = rb * 32 + hl;
        smask[rr * MWS + w] = sdone[rr] ? 0u : row;
      }
      __syncthreads();
      for (int i = tid; i < 4 * MW; i += NT) {
        const int wv = i / MW, w = i - wv * MW;
        uint32_t u = 0;
        for (int rr = wv * RPW; rr < (wv + 1) * RPW; ++rr) u |= smask[rr * MWS + w];
        suni[wv * MW + w] = u;
      }
      __syncthreads();
    }
    // ---- midpoint order, collect: one record per hit of the ray, in list order ----
    if constexpr (COLLECT) {
      if (valid) {
        const uint32_t *mine = smask + r * MWS;
        for (int w = 0; w < MW; ++w) {
          uint32_t bits = mine[w];
          while (bits) {
            const int j = w * 32 + __builtin_ctz(bits);
            bits &= bits - 1;
            if ((int)(n_ray_hits & (G - 1)) == q) {
              const float4 *geo = sgeo + kGeo * j;
              Terms h;
              test_hit(vx, vy, vz, geo, a.r_rx, h);            // the terms of the phase-1 hit
              hit_terms<K, true>(geo, scf + 2 * K * j, Yr, Yi, a.amax, h, a.fle_g, a.chord);
              // t_mid = D (1 - b/A) with D = hi + lo, in FP64 from the FP32 terms (error
              // ~1e-7 m), as a fixed-point key of 2^-24 m over [0, 2^16) m above the rank
              const double dh = geo[0].w;
              const double tm = fmin(fmax(dh - dh * (double)h.bA + (double)geo[4].w, 0.0), kTmidMaxT);
              io.hit_key[ray_base + n_ray_hits] =
                  ((uint64_t)(tm * kTmidKeyScale) << kTmidRankBits) | (n_ray_hits & kTmidRankMask);
              io.hit_val[ray_base + n_ray_hits] = make_float4(h.keep, h.p * h.pzr, h.p * h.pzi, 0.f);
            }
            ++n_ray_hits;
          }
        }
      }
    }
    // ---- phase 2: walk the wave's union, G entries per step ----
    if (!COUNT && !COLLECT && __ballot(!done) != 0) {        // wave-uniform
      const uint32_t *uw = suni + wave * MW;
      const uint32_t *mine = smask + r * MWS;
      int wi = 0;
      uint32_t rb = __builtin_amdgcn_readfirstlane(uw[0]);
      while (true) {
        int j = -1, first = -1;
#pragma unroll
        for (int i = 0; i < G; ++i) {                        // scalar: the cursor is wave-uniform
          while (rb == 0 && wi + 1 < MW) rb = __builtin_amdgcn_readfirstlane(uw[++wi]);
          int jj = -1;
          if (rb != 0) {
            jj = wi * 32 + __builtin_ctz(rb);
            rb &= rb - 1;
          }
          if (i == 0) first = jj;
          if (q == i) j = jj;
        }
        if (first < 0) break;
        if (STATS) ++n_steps;
        const bool hit = !done && j >= 0 && ((mine[j >> 5] >> (j & 31)) & 1u);
        const float4 *geo = sgeo + kGeo * (j >= 0 ? j : 0);
        Terms h;
        float f = 1.f, ctr = 0.f, cti = 0.f;
        if (hit) {
          test_hit(vx, vy, vz, geo, a.r_rx, h);               // the terms of the phase-1 hit
          hit_terms<K, VAR>(geo, scf + 2 * K * j, Yr, Yi, a.amax, h, a.fle_g, a.chord);
          f = h.keep;
          ctr = h.p * h.pzr;
          cti = h.p * h.pzi;
        }
        float excl, total;
        group_prod<G>(f, q, excl, total);
        const float Tj = T * excl;
        const bool proc = hit && (Tj >= a.t_min);
        if constexpr (MTOT) {
          // the ray's sum over hits of T_j Re(conj(Ge_j) c~_j), FP64
          if (proc) {
            float sd, cd, Ger, Gei, Ge2r, Ge2i;
            const float4 g4 = geo[4];
            sincos_rev(fmaf(-h.bA, g4.w, g4.z), sd, cd);
            carrier_sums_n<kGcChunk>(sgc + r * kGcChunk, sd, cd, Ger, Gei, Ge2r, Ge2i);
            Sr = fma((double)Tj, (double)fmaf(Ger, ctr, Gei * cti), Sr);
          }
          T = T * total;
          done = done || (T < a.t_min);
        } else if constexpr (!BWD) {
          if (proc) {
            Sr = fma((double)Tj, (double)ctr, Sr);
            Si = fma((double)Tj, (double)cti, Si);
            if (STATS) ++n_hit;
            if constexpr (MULTI) {
              // carrier c: p psi e^{-j phi_c}, phi_{c+1} = phi_c + 2 pi (|mu - tx| + t) step / c0
              float sns, css;
              const float4 g4 = geo[4];
              sincos_rev(fmaf(-h.bA, g4.w, g4.z), sns, css);
              const float w = Tj * h.p;
              float zr = h.pzr, zi = h.pzi;
#pragma unroll
              for (int c = 0; c < FC; ++c) {
                mr[c] = fmaf(w, zr, mr[c]);
                mi[c] = fmaf(w, zi, mi[c]);
                const float nr = fmaf(zr, css, zi * sns), ni = fmaf(zi, css, -(zr * sns));
                zr = nr;
                zi = ni;
              }
            }
          }
          T = T * total;
          done = done || (T < a.t_min);
        } else {
          // FP64 prefix of the hits' terms: T_j c~_j (one carrier), or the scalar
          // T_j Re(conj(Ge_j) c~_j) (several), whose total the total pass left in Sfr
          double wr = 0.0, wi_ = 0.0;
          float Ger = 0.f, Gei = 0.f, Ge2r = 0.f, Ge2i = 0.f;
          if constexpr (BMULTI) {
            if (proc) {
              float sd, cd;
              const float4 g4 = geo[4];
              sincos_rev(fmaf(-h.bA, g4.w, g4.z), sd, cd);
              carrier_sums_n<kGcChunk>(sgc + r * kGcChunk, sd, cd, Ger, Gei, Ge2r, Ge2i);
              wr = (double)Tj * (double)fmaf(Ger, ctr, Gei * cti);
            }
          } else if (proc) {
            wr = (double)Tj * (double)ctr;
            wi_ = (double)Tj * (double)cti;
          }
          double wr_in, wi_in = 0.0, wr_tot, wi_tot = 0.0;
          group_sum64<G>(wr, q, wr_in, wr_tot);
          if constexpr (!BMULTI) group_sum64<G>(wi_, q, wi_in, wi_tot);
          T = T * total;
          done = done || (T < a.t_min);
          if (__ballot(proc) != 0) {
            AdjHit ah{};
            if (proc) {
              if constexpr (BMULTI) {
                const float num = (float)(Sfr - (Pr + wr_in));
                ah = adj_hit_multi(h, geo, Tj, ctr, cti, num, Ger, Gei, Ge2r, Ge2i, vx, vy, vz, twopi_lam,
                                   twopi_dlam);
              } else {
                const float Rr = (float)(Sfr - (Pr + wr_in)), Ri = (float)(Sfi - (Pi + wi_in));
                ah = adj_hit(h, geo, Tj, ctr, cti, Rr, Ri, Gr, Gi, vx, vy, vz, twopi_lam);
              }
              sflag[j] = 1u;
            }
            // the slots in parts of 16, each reduced over the wave's rays before the next is formed
            constexpr int NF = (16 * G >= 64) ? 16 * G / 64 : 1;
            float *dst = sacc + NACC * (j >= 0 ? j : 0);
#pragma unroll
            for (int part = 0; part < NV / 16; ++part) {
              float c[16];
#pragma unroll
              for (int i = 0; i < 16; ++i) c[i] = adj_slot<K>(part * 16 + i, ah, vx, vy, vz, Yr, Yi);
              int first_slot;
              bool writer;
              reduce_scatter<16, G>(c, lane, &first_slot, &writer);
              if (writer && j >= 0) {
#pragma unroll
                for (int i = 0; i < NF; ++i)
                  if (part * 16 + first_slot + i < NACC) atomicAdd(dst + part * 16 + first_slot + i, c[i]);
              }
            }
          }
          Pr += wr_tot;
          Pi += wi_tot;
        }
        if (__ballot(!done) == 0) break;
      }
      if (q == 0 && done) sdone[r] = 1;
    }
    if constexpr (BWD) {
      __syncthreads();
      flush_batch<K, NT>(nb, sacc, sflag, stx, io.acc, io.acc_stride);
    }
    if (__syncthreads_and(done ? 1 : 0)) {
      if constexpr (!MASKED) base += (uint32_t)nb;
      break;
    }
    if constexpr (!MASKED) base += B;
  }
  if constexpr (MODE == kTpFwd || COUNT) {   // the end of the masks written, per ray block
    if (tid < MWR) a.mask_end[(size_t)gtile * (MWR * SPLIT) + half * MWR + tid] = min(base, s1);
  }
  if constexpr (COUNT) {
    if (e == 0 && valid1) io.ray_cnt[((size_t)k * a.n_el + v1) * a.n_az + u1] = n_ray_hits;
    return;
  }
  if constexpr (COLLECT) return;
  if constexpr (MTOT) {
    double xr = Sr;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) xr += __shfl_xor(xr, d, G);
    if (valid && q == 0) io.wtot[((size_t)k * a.n_el + v) * a.n_az + u] = xr;
    return;
  }
  if constexpr (!BWD) {
    if constexpr (G > 1) {   // the ray's total over its G lanes
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        Sr += __shfl_xor(Sr, d, G);
        Si += __shfl_xor(Si, d, G);
      }
    }
    if constexpr (STATS) {
      if (n_test) atomicAdd(io.stats + 0, n_test);
      if (n_hit) atomicAdd(io.stats + 1, n_hit);
      if (n_staged) atomicAdd(io.stats + 2, n_staged);
      if (valid && q == 0) atomicAdd(io.stats + 3, 1ull);
      if (n_tile_tests) atomicAdd(io.stats + 4, n_tile_tests);
      if (lane == 0 && n_steps) atomicAdd(io.stats + 5, 64ull * n_steps);
      return;
    }
    if constexpr (MULTI) {   // the ray's carriers, summed over its G lanes
      const int nc = min(FC, io.n_freq - io.f_first);
#pragma unroll
      for (int c = 0; c < FC; ++c) {
        float xr = mr[c], xi = mi[c];
        if constexpr (G > 1) {
#pragma unroll
          for (int d = 1; d < G; d <<= 1) {
            xr += __shfl_xor(xr, d, G);
            xi += __shfl_xor(xi, d, G);
          }
        }
        if (valid && q == 0 && c < nc)
          io.multi[(((size_t)k * io.n_freq + io.f_first + c) * a.n_el + v) * a.n_az + u] = make_float2(xr, xi);
      }
      return;
    }
    if (valid && q == 0) {
      const size_t ri = ((size_t)k * a.n_el + v) * a.n_az + u;
      io.signal[ri] = make_float2((float)Sr, (float)Si);
      if (io.sig64) io.sig64[ri] = make_double2(Sr, Si);
    }
    // tile partial of S_hat in a fixed order: each wave's rays by a butterfly,
    // then the four wave totals in wave order
    float xr = (q == 0) ? (float)Sr : 0.f, xi = (q == 0) ? (float)Si : 0.f;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      xr += __shfl_xor(xr, d, 64);
      xi += __shfl_xor(xi, d, 64);
    }
    __syncthreads();
    float *red = (float *)smem;
    if (lane == 0) {
      red[wave] = xr;
      red[4 + wave] = xi;
    }
    __syncthreads();
    if (tid == 0) io.tile_sum[gt] = make_float2((red[0] + red[1]) + (red[2] + red[3]), (red[4] + red[5]) + (red[6] + red[7]));
  }
}

// Launches of at most this many (pair, tile) units hold their adjoint
// workgroups to two per CU (by their LDS request).  Otherwise all of them fit
// at once (three waves per SIMD), three to some CUs and two to the rest, and
// the CUs with three finish last; with two per CU the remaining workgroups
// start wherever a CU frees first (the benchmark's 540 tiles: 104 -> 98 us).
constexpr int64_t kAdjPairedBlocks = 2048;
constexpr size_t kLdsPerCu = 160 * 1024;

template <int L, int R, int MODE, int BCAP, int SPLIT, bool VAR = false>
hipError_t tp_launch(const RenderArgs &a, const TpIO &io, int64_t nblocks, hipStream_t s) {
  constexpr size_t lds0 = TpShape<L, R, MODE, BCAP>::lds();
  const size_t lds = (TpShape<L, R, MODE, BCAP>::BWD && nblocks <= kAdjPairedBlocks && lds0 <= kLdsPerCu / 3)
                         ? kLdsPerCu / 3 + 256 : lds0;
  if (lds > 65536) {   // high FLE degrees: opt in to more than 64 KB of LDS
    const hipError_t e = hipFuncSetAttribute((const void *)k_render_tp<L, R, MODE, BCAP, SPLIT, VAR>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_render_tp<L, R, MODE, BCAP, SPLIT, VAR>), dim3((unsigned)(nblocks * SPLIT)), dim3(256), lds,
                     s, a, io);
  return hipGetLastError();
}

// Workgroups below which a launch counts as latency-bound: the forward then
// splits tiles of 64 rays or more in two (the adjoint, with more registers per
// thread, would not fit the extra workgroups on the chip at once).
constexpr int64_t kFewBlocks = 2048;

// Workgroups per tile of the two-phase forward (1 or 2) for a launch over
// `tiles` (pair, tile) units: the split halves the tile's rows, so a tile of
// one row is never split.
inline int tp_split(int area, int64_t tiles, int tile_h) {
  return (area >= 64 && tile_h >= 2 && tiles <= kFewBlocks) ? 2 : 1;
}

template <int L, int MODE>
hipError_t tp_dispatch(int area, const RenderArgs &a, const TpIO &io, int64_t nblocks, hipStream_t s) {
  if constexpr (MODE == kTpFwd || multi_chunk(MODE) > 1) {   // (the counters follow whole tiles, as the adjoint does)
    if (tp_split(area, nblocks, area / a.tw) == 2) {
      // the split forward stages 256 entries per batch: fewer barriers at three
      // workgroups per CU (LDS) beat more waves here (200k step: 59.7 -> 58.0 us),
      // whereas launches with many tiles keep 128 (the 500k batch: 9.6 against 11.1 ms)
      constexpr int BC = MODE == kTpFwd ? 256 : 128;
      switch (area) {
        case 64: return tp_launch<L, 32, MODE, BC, 2>(a, io, nblocks, s);
        case 128: return tp_launch<L, 64, MODE, BC, 2>(a, io, nblocks, s);
        default: return tp_launch<L, 128, MODE, BC, 2>(a, io, nblocks, s);
      }
    }
  }
  switch (area) {
    case 32: return tp_launch<L, 32, MODE, 128, 1>(a, io, nblocks, s);
    case 64: return tp_launch<L, 64, MODE, 128, 1>(a, io, nblocks, s);
    case 128: return tp_launch<L, 128, MODE, 128, 1>(a, io, nblocks, s);
    default: return tp_launch<L, 256, MODE, 128, 1>(a, io, nblocks, s);
  }
}

// The paper-literal variant kernels (per-Gaussian FLE, chord transmittance,
// and the two passes of the per-ray midpoint order): whole tiles, runtime
// switches read from RenderArgs.
template <int L, int MODE>
hipError_t tp_dispatch_var(int area, const RenderArgs &a, const TpIO &io, int64_t nblocks, hipStream_t s) {
  switch (area) {
    case 32: return tp_launch<L, 32, MODE, 128, 1, true>(a, io, nblocks, s);
    case 64: return tp_launch<L, 64, MODE, 128, 1, true>(a, io, nblocks, s);
    case 128: return tp_launch<L, 128, MODE, 128, 1, true>(a, io, nblocks, s);
    default: return tp_launch<L, 256, MODE, 128, 1, true>(a, io, nblocks, s);
  }
}

}  // namespace gsrf
