// Internal declarations shared by the libgsrf translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gsrf.h"

namespace gsrf {

// Speed of light fixed by the two-path example of Sec. 2 (3 m <-> 10 ns).
constexpr double kC0 = 3.0e8;
// Widening of the bounding cap used for binning (rad); covers the FP32
// rounding of ray directions with a wide margin.
constexpr double kCapSlack = 1e-5;
// 3-sigma ellipsoid level (App. D.3.1).
constexpr float kLevel = 9.0f;
// Per-Gaussian prepared record: mu(3), N, M00 M11 M22 M01 M02 M12, o, pad, 3 max(s), max log s, pad(2).
constexpr int kPrep = 16;

// Binning: splats are emitted into per-tile buckets (key, Gaussian) and each
// tile's bucket is sorted by one workgroup of kTileSortThreads threads, through
// LDS for buckets of at most `sort_chunk` entries, else through global scratch.
constexpr int kTileSortThreads = 1024;
constexpr int kMaxTiles = 8192;           // per pair; LDS histograms in project/emit
constexpr int kMaxCarriers = 4096;        // carriers of one multi-carrier forward
// Records per workgroup in emit: 256, or 1024 for large batches (fewer
// workgroups per tile means fewer global cursor atomics per record); project
// always uses 256 and counts into the sub-bucket of emit's workgroup.
constexpr int64_t kBigBatchRecords = (int64_t)1 << 22;
// Each tile's bucket is split into kSub contiguous sub-buckets; emit's
// workgroup b (and project's workgroups of the same records) counts into and
// reserves from sub-bucket (b % kSub), which
// divides the atomic traffic per counter by kSub.  Counters and cursors are
// stored sub-major: [kSub][P * T].
constexpr int kSub = 8;
// Tiles per block of the three-pass tile-count scan (256 threads x 4).
constexpr int kScanTiles = 1024;
// Launches with more (pair, tile) units than this sort the buckets in tiers by
// length (one workgroup per tile below that).
constexpr int64_t kSortFewTiles = 2048;
// Queue of the long buckets of a tiered sort.  The tile-range scan appends
// each tile whose bucket holds more than thr[n] entries to the list of its
// length class c (thr[c + 1] < entries <= thr[c], thr descending); the two
// long-bucket sort kernels take classes [0, split) and [split, n), longest
// class first, one bucket per atomic pop, so that no workgroup is left with
// the heaviest buckets at the end.  Queue memory: kLongQueueHeader words
// (class counts, then the pop counters of the two kernels), then
// kLongClasses lists of P * T (bucket start, entries) pairs.
constexpr int kLongClasses = 7;
constexpr int kLongQueueHeader = 16;
struct LongClasses {
  int32_t n, split;
  int32_t thr[kLongClasses + 1];
  int32_t lo;   // thr[n]: the longest bucket left to the shorter tiers
};
// The classes for the device's sort chunks (sort.hip).
LongClasses long_classes();
// Ray table row (floats, 16-byte aligned): direction (3), pad, then the FLE
// basis interleaved Yr_0, Yi_0, Yr_1, Yi_1, ... (2K).
constexpr int ray_stride(int K) { return (4 + 2 * K + 3) / 4 * 4; }

// Balanced expansion of the tile rectangles of a workgroup's RB records
// (RB = 256 or 1024, one per thread): the rectangles' splat counts are scanned;
// then either every thread takes splats s = tid, tid + RB, ..., locating the
// owning record by binary search (rect_splat), or each thread takes an equal run
// of consecutive splats (rect_for_each).
template <int RB>
struct RectScan {
  ushort4 rect[RB];
  float inv_ntu[RB];       // 1 / (tile columns) of each rectangle
  uint32_t off[RB + 1];
  uint32_t wsum[RB / 64];
};

template <int RB>
__device__ __forceinline__ void rect_scan(RectScan<RB> &rs, ushort4 rc) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t c = (uint32_t)rc.y * rc.w;
  rs.rect[tid] = rc;
  rs.inv_ntu[tid] = 1.0f / (float)(rc.y > 0 ? rc.y : 1);
  uint32_t inc = c;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  if (lane == 63) rs.wsum[wave] = inc;
  __syncthreads();
  uint32_t base = 0;
#pragma unroll
  for (int w = 0; w < RB / 64 - 1; ++w) base += (w < wave) ? rs.wsum[w] : 0u;
  rs.off[tid + 1] = base + inc;
  if (tid == 0) rs.off[0] = 0;
  __syncthreads();
}

// splat s of the workgroup: owning record (thread slot; the last record whose
// offset is <= s) and its tile id
template <int RB>
__device__ __forceinline__ int rect_splat(const RectScan<RB> &rs, uint32_t s, int nta, int *tile) {
  int pos = 0;
#pragma unroll
  for (int step = RB / 2; step >= 1; step >>= 1)
    if (rs.off[pos + step] <= s) pos += step;
  const ushort4 rc = rs.rect[pos];
  const uint32_t local = s - rs.off[pos];
  // row = floor((local + 1/2) / ntu): the quotient is at most ntv + 1 and at
  // least 1/(2 ntu) from an integer, and ntu * ntv <= kMaxTiles keeps its FP32
  // error two orders of magnitude below that distance
  const uint32_t q = (uint32_t)(((float)local + 0.5f) * rs.inv_ntu[pos]);
  const int tv = rc.z + (int)q;
  int tu = rc.x + (int)(local - q * rc.y);
  if (tu >= nta) tu -= nta;
  *tile = tv * nta + tu;
  return pos;
}

// Every splat of the workgroup, f(s, record slot, tile id): thread tid takes the
// contiguous splats [tid E, tid E + E), E = ceil(total / RB), finds the record
// of its first splat by binary search (the last record whose offset is <= s)
// and walks forward from there, stepping through the rectangle's columns and
// rows and on to the next record with splats.
template <int RB, typename F>
__device__ __forceinline__ void rect_for_each(const RectScan<RB> &rs, uint32_t total, int nta, F f) {
  const uint32_t E = (total + RB - 1) / RB;
  uint32_t s = (uint32_t)threadIdx.x * E;
  const uint32_t send = min(total, s + E);
  if (s >= send) return;
  int pos = 0;
#pragma unroll
  for (int step = RB / 2; step >= 1; step >>= 1)
    if (rs.off[pos + step] <= s) pos += step;
  uint32_t nxt = rs.off[pos + 1];
  ushort4 rc = rs.rect[pos];
  const uint32_t local = s - rs.off[pos];
  const uint32_t q = (uint32_t)(((float)local + 0.5f) * rs.inv_ntu[pos]);   // (as in rect_splat)
  int tv = rc.z + (int)q;
  int cu = (int)(local - q * rc.y);
  for (;;) {
    int tu = rc.x + cu;
    if (tu >= nta) tu -= nta;
    f(s, pos, tv * nta + tu);
    if (++s >= send) break;
    if (s < nxt) {
      if (++cu == (int)rc.y) { cu = 0; ++tv; }
    } else {   // off[RB] = total > s ends the walk
      do { ++pos; nxt = rs.off[pos + 1]; } while (nxt <= s);
      rc = rs.rect[pos];
      tv = rc.z;
      cu = 0;
    }
  }
}

// Byte offsets of every workspace array plus derived sizes.
struct Layout {
  size_t prep, rec_base, rec_key, rec_rect, counters;
  size_t tile_cnt, tile_start, tile_end, tile_cur;
  size_t scan_blk;        // per-block totals of the tile-count scan
  size_t ekv;             // emitted buckets (unsorted): (depth key, Gaussian id) pairs
  size_t klo, val;        // sorted tile lists: depth key, Gaussian id
  size_t tkv;             // sort scratch for buckets longer than the LDS chunk: (key, id) pairs
  size_t long_q;          // long-bucket queue of the tiered sort (P * T > kSortFewTiles only)
  size_t tile_sum, grad_acc;
  size_t hitmask;         // two-phase traversal: per splat, tile-area / 32 words of forward hit bits
  size_t mask_end;        // two-phase traversal: per (pair, tile, 32-ray block), the end of the masks written
  size_t sig64;           // [P][n_el * n_az] double2: the forward's S in FP64, read by the adjoint
  size_t wtot;            // [P][n_el * n_az] double: the several-carrier adjoint's per-ray totals
  size_t rays;            // [n_el * n_az][ray_stride(K)] ray directions and FLE basis (FP32)
  // per-ray midpoint order (depth_order = 1): hits per ray, first record per
  // ray, block sums of their scan, and the records (sort key, terms)
  size_t ray_cnt, ray_off, tmid_blk, hit_key, hit_val;
  int64_t hit_cap;
  size_t total;
  int64_t n_records;
  int32_t rec_block;      // records per workgroup in emit (256 or 1024)
  int64_t max_scene;
  int64_t cap;
  int32_t T, nta, nte;
  int32_t K, acc_stride;
};

inline int fle_K(int L) { return (L + 1) * (L + 1); }

// Instrumentation events (set by gsrf_set_kernel_events): 0/1 around the
// forward render kernel (the multi-carrier traversals), 2/3 around the
// adjoint kernel.
void mark_kernel_event(int i, hipStream_t s);


struct RenderArgs;
RenderArgs make_render_args(const gsrf_problem *p, const Layout &lay, char *ws);

// A paper-literal variant of the render is selected (per-ray midpoint order,
// per-Gaussian FLE or chord transmittance).
inline bool has_variant(const gsrf_grid &g) { return g.depth_order != 0 || g.fle_eval != 0 || g.transmittance != 0; }
// Rays per midpoint-order scan block.
constexpr int kTmidScan = 1024;

// Launch helpers implemented in the .hip files; each returns hipSuccess or the
// launch error.
hipError_t launch_project(const gsrf_problem *p, const Layout &lay, char *ws, hipStream_t s);
hipError_t launch_bin_sort(const gsrf_problem *p, const Layout &lay, char *ws, hipStream_t s);
hipError_t launch_render_fwd(const gsrf_problem *p, const Layout &lay, char *ws, float *signal,
                             float *signal_sum, float *rssi_dbm, hipStream_t s);
hipError_t launch_render_stats(const gsrf_problem *p, const Layout &lay, char *ws, int64_t *counts, hipStream_t s);
hipError_t launch_render_fwd_variant(const gsrf_problem *p, const Layout &lay, char *ws, float *signal,
                                     float *signal_sum, float *rssi_dbm, hipStream_t s);
hipError_t launch_render_fwd_multi(const gsrf_problem *p, const Layout &lay, char *ws, int32_t n_freq, double f_step,
                                   float *signal, float *signal_sum, hipStream_t s);
hipError_t launch_render_bwd_multi(const gsrf_problem *p, const Layout &lay, char *ws, int32_t n_freq, double f_step,
                                   const float *grad_signal, const float *grad_sum, float *d_means,
                                   float *d_log_scales, float *d_quats, float *d_logits, float *d_coeffs,
                                   hipStream_t s);
hipError_t launch_render_bwd(const gsrf_problem *p, const Layout &lay, char *ws, const float *signal,
                             const float *grad_signal, const float *grad_sum, float *d_means,
                             float *d_log_scales, float *d_quats, float *d_logits, float *d_coeffs,
                             hipStream_t s);

// Training steps (train.hip).
size_t loss_partials_bytes(int32_t n_pairs, int32_t n_el, int32_t n_az);
// Bytes of the fixed device scratch behind gsrf_loss_spectrum_noalloc, and
// its address on the current device (hipErrorInvalidDevice when a non-null
// stream belongs to another device).
size_t loss_scratch_bytes();
hipError_t loss_scratch_address(hipStream_t s, void **out);
hipError_t launch_loss_spectrum(const float *signal, const float *target, int32_t n_pairs, int32_t n_el, int32_t n_az,
                                float pscale, float lam1, float lam2, float *loss, float *grad_signal, void *ws,
                                hipStream_t s);
hipError_t launch_loss_single(const float *signal_sum, const float *target, int32_t n_pairs, int32_t kind,
                              float *loss, float *grad_sum, hipStream_t s);
hipError_t launch_sgd(int64_t n_gauss, int K, float *const w[5], const float *const g[5], const float eta[5],
                      hipStream_t s);

// Adaptive density control (density.hip).
struct DensityIO {
  const float *means, *log_scales, *quats, *logits, *coeffs, *acc, *z;
  const int32_t *cnt;
  int64_t n;
  int K;
  double eps_mu, eps_r, eps_rho, clone_step;
  float ln_phi;
  int densify, prune;
  float *o_means, *o_log_scales, *o_quats, *o_logits, *o_coeffs, *o_acc;
  int32_t *o_cnt;
  int64_t *counts;
  void *ws;
};
size_t density_workspace_bytes(int64_t n);
hipError_t launch_grad_accum(int64_t n, const float *d_means, float *acc, int32_t *cnt, hipStream_t s);
hipError_t launch_density_control(const DensityIO &io, hipStream_t s);

// Dynamic LDS available to one workgroup on the current device (bytes).
size_t max_lds_per_block();

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <typename T>
inline hipError_t fill(T *p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace gsrf
