// Host side of the C ABI: argument validation, workspace layout and launch
// sequencing.  Nothing here allocates device memory or synchronises, except
// gsrf_splat_count, whose contract is to synchronise.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "gsrf_internal.h"

namespace gsrf {

static thread_local char g_err[512];

static gsrf_status fail(gsrf_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static gsrf_status fail(gsrf_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

static gsrf_status dev(hipError_t e, const char *where) {
  if (e == hipSuccess) return GSRF_OK;
  return fail(GSRF_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

static hipEvent_t g_kernel_events[4] = {nullptr, nullptr, nullptr, nullptr};

void mark_kernel_event(int i, hipStream_t s) {
  if (g_kernel_events[i]) (void)hipEventRecord(g_kernel_events[i], s);
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Validates the host-readable parts of a problem and computes its layout.
static gsrf_status plan(const gsrf_problem *p, Layout *lay, bool need_device) {
  if (!p || !lay) return fail(GSRF_EINVAL, "null problem or output");
  const gsrf_grid &g = p->grid;
  if (g.n_az <= 0 || g.n_el <= 0 || g.n_az > 65535 || g.n_el > 65535)
    return fail(GSRF_EINVAL, "grid size %d x %d out of range [1, 65535]", g.n_az, g.n_el);
  if (g.fle_L < 0 || g.fle_L > 6) return fail(GSRF_EINVAL, "fle_L = %d outside [0, 6]", g.fle_L);
  const int nt = g.tile_w * g.tile_h;
  if (g.tile_w <= 0 || g.tile_h <= 0 || (nt != 32 && nt != 64 && nt != 128 && nt != 256))
    return fail(GSRF_EINVAL, "tile %d x %d: tile_w * tile_h must be 32, 64, 128 or 256", g.tile_w, g.tile_h);
  if (g.lanes_per_ray != 0 && g.lanes_per_ray != 1 && g.lanes_per_ray != 2 && g.lanes_per_ray != 4)
    return fail(GSRF_EINVAL, "lanes_per_ray = %d: must be 0, 1, 2 or 4", g.lanes_per_ray);
  if (g.footprint != 0 && g.footprint != 1)
    return fail(GSRF_EINVAL, "footprint = %d: must be 0 (exact cap) or 1 (paper footprint)", g.footprint);
  if (nt == 32 && g.lanes_per_ray != 0)
    return fail(GSRF_EINVAL, "32-ray tiles need the two-phase traversal (lanes_per_ray = 0)");
  if ((g.depth_order != 0 && g.depth_order != 1) || (g.fle_eval != 0 && g.fle_eval != 1) ||
      (g.transmittance != 0 && g.transmittance != 1))
    return fail(GSRF_EINVAL, "depth_order = %d, fle_eval = %d, transmittance = %d: each must be 0 or 1",
                g.depth_order, g.fle_eval, g.transmittance);
  if (has_variant(g) && g.lanes_per_ray != 0)
    return fail(GSRF_EINVAL, "the paper-literal variants need the two-phase traversal (lanes_per_ray = 0)");
  if (g.depth_order && (p->hit_capacity < 0 || p->hit_capacity >= ((int64_t)1 << 40)))
    return fail(GSRF_EINVAL, "hit_capacity = %lld outside [0, 2^40)", (long long)p->hit_capacity);
  if (!(g.el_lo < g.el_hi) || g.el_lo < -1.5707964f || g.el_hi > 1.5707964f)
    return fail(GSRF_EINVAL, "elevation span [%g, %g] invalid", (double)g.el_lo, (double)g.el_hi);
  if (!(g.r_rx >= 0.f) || !(g.t_min >= 0.f) || !(g.alpha_max > 0.f && g.alpha_max < 1.f))
    return fail(GSRF_EINVAL, "need r_rx >= 0, t_min >= 0, 0 < alpha_max < 1");
  if (p->n_gauss < 0 || p->n_gauss >= ((int64_t)1 << 31)) return fail(GSRF_EINVAL, "n_gauss = %lld", (long long)p->n_gauss);
  if (p->n_pairs < 0 || p->n_pairs > 65535) return fail(GSRF_EINVAL, "n_pairs = %d outside [0, 65535]", p->n_pairs);
  if (p->n_scenes < 1) return fail(GSRF_EINVAL, "n_scenes must be >= 1");
  if (!p->scene_offsets) return fail(GSRF_EINVAL, "scene_offsets (host) is NULL");
  if (p->scene_offsets[0] != 0 || p->scene_offsets[p->n_scenes] != p->n_gauss)
    return fail(GSRF_EINVAL, "scene_offsets must start at 0 and end at n_gauss");
  int64_t max_scene = 0;
  for (int s = 0; s < p->n_scenes; ++s) {
    const int64_t n = p->scene_offsets[s + 1] - p->scene_offsets[s];
    if (n < 0) return fail(GSRF_EINVAL, "scene_offsets not non-decreasing at %d", s);
    if (n > max_scene) max_scene = n;
  }
  if (p->n_pairs > 0 && !p->pair_scene) return fail(GSRF_EINVAL, "pair_scene (host) is NULL");
  int64_t R = 0, max_used = 0;
  for (int k = 0; k < p->n_pairs; ++k) {
    const int s = p->pair_scene[k];
    if (s < 0 || s >= p->n_scenes) return fail(GSRF_EINVAL, "pair %d: scene %d out of range", k, s);
    const int64_t n = p->scene_offsets[s + 1] - p->scene_offsets[s];
    R += n;
    if (n > max_used) max_used = n;
  }
  if (p->splat_capacity < 0 || p->splat_capacity >= ((int64_t)1 << 32) - 1)
    return fail(GSRF_EINVAL, "splat_capacity = %lld outside [0, 2^32 - 1)", (long long)p->splat_capacity);
  const int nta = (g.n_az + g.tile_w - 1) / g.tile_w;
  const int nte = (g.n_el + g.tile_h - 1) / g.tile_h;
  const int64_t T = (int64_t)nta * nte;
  if ((int64_t)p->n_pairs * T >= ((int64_t)1 << 31)) return fail(GSRF_EINVAL, "n_pairs * tiles too large");
  if (need_device) {
    if (p->n_gauss > 0 && (!p->means || !p->log_scales || !p->quats || !p->opacity_logits || !p->coeffs))
      return fail(GSRF_EINVAL, "a Gaussian parameter pointer is NULL");
    if (!p->scene_offsets_dev) return fail(GSRF_EINVAL, "scene_offsets_dev is NULL");
    if (p->n_pairs > 0 && !p->pairs) return fail(GSRF_EINVAL, "pairs is NULL");
    if (!p->workspace) return fail(GSRF_EINVAL, "workspace is NULL");
    if ((uintptr_t)p->workspace & 255) return fail(GSRF_EINVAL, "workspace must be 256-byte aligned");
  }
  if (T > kMaxTiles) return fail(GSRF_EINVAL, "%lld tiles per pair exceed %d", (long long)T, kMaxTiles);
  Layout L{};
  L.n_records = R;
  L.rec_block = R >= kBigBatchRecords ? 1024 : 256;
  L.max_scene = max_used;
  L.cap = p->splat_capacity;
  L.T = (int32_t)T;
  L.nta = nta;
  L.nte = nte;
  L.K = fle_K(g.fle_L);
  L.acc_stride = (11 + 2 * L.K + 15) / 16 * 16;   // 64-byte rows of the adjoint accumulators
  const int64_t PT = (int64_t)p->n_pairs * T;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const int64_t G = p->n_gauss;
  L.prep = take((size_t)G * kPrep * 4);
  L.rec_base = take((size_t)(p->n_pairs + 1) * 8);
  L.rec_key = take((size_t)R * 4);
  L.rec_rect = take((size_t)R * 8);
  L.counters = take(4 * 8);
  L.tile_cnt = take((size_t)PT * kSub * 4);
  L.tile_start = take((size_t)PT * 4);
  L.tile_end = take((size_t)PT * 4);
  L.tile_cur = take((size_t)PT * kSub * 4);
  L.scan_blk = take((size_t)((PT + kScanTiles - 1) / kScanTiles + 1) * 8);
  L.ekv = take((size_t)L.cap * 8);
  L.klo = take((size_t)L.cap * 4);
  L.val = take((size_t)L.cap * 4);
  L.tkv = take((size_t)L.cap * 8);
  L.long_q = take(PT > kSortFewTiles ? (size_t)kLongQueueHeader * 4 + (size_t)kLongClasses * PT * 8 : 0);
  L.tile_sum = take((size_t)PT * 2 * 8);   // per render workgroup: up to two per tile
  L.grad_acc = take((size_t)G * L.acc_stride * 4);
  L.hitmask = take(g.lanes_per_ray == 0 ? (size_t)L.cap * (size_t)(g.tile_w * g.tile_h / 32) * 4 : 0);
  L.mask_end = take(g.lanes_per_ray == 0 ? (size_t)PT * (size_t)(g.tile_w * g.tile_h / 32) * 4 : 0);
  L.sig64 = take((size_t)p->n_pairs * g.n_az * g.n_el * 16);
  L.wtot = take(g.lanes_per_ray == 0 ? (size_t)p->n_pairs * g.n_az * g.n_el * 8 : 0);
  L.rays = take((size_t)g.n_az * g.n_el * ray_stride(L.K) * 4);
  {
    const int64_t n_all = g.depth_order ? (int64_t)p->n_pairs * g.n_az * g.n_el : 0;
    L.hit_cap = g.depth_order ? p->hit_capacity : 0;
    L.ray_cnt = take((size_t)n_all * 4);
    L.ray_off = take((size_t)n_all * 8);
    L.tmid_blk = take((size_t)((n_all + kTmidScan - 1) / kTmidScan + 1) * 8);
    L.hit_key = take((size_t)L.hit_cap * 8);
    L.hit_val = take((size_t)L.hit_cap * 16);
  }
  L.total = o;
  if (need_device && p->workspace_bytes < L.total)
    return fail(GSRF_EINVAL, "workspace_bytes %zu < required %zu", p->workspace_bytes, L.total);
  *lay = L;
  return GSRF_OK;
}

}  // namespace gsrf

using namespace gsrf;

extern "C" {

const char *gsrf_status_str(gsrf_status s) {
  switch (s) {
    case GSRF_OK: return "GSRF_OK";
    case GSRF_EINVAL: return "GSRF_EINVAL";
    case GSRF_ECAPACITY: return "GSRF_ECAPACITY";
    case GSRF_EDEVICE: return "GSRF_EDEVICE";
    case GSRF_ENOTSUP: return "GSRF_ENOTSUP";
  }
  return "GSRF_UNKNOWN";
}

const char *gsrf_last_error(void) { return g_err; }

gsrf_status gsrf_workspace_size(const gsrf_problem *p, size_t *bytes) {
  if (!bytes) return fail(GSRF_EINVAL, "bytes is NULL");
  Layout L;
  gsrf_status st = plan(p, &L, false);
  if (st != GSRF_OK) return st;
  *bytes = L.total;
  return GSRF_OK;
}

gsrf_status gsrf_layout_of(const gsrf_problem *p, gsrf_layout *out) {
  if (!out) return fail(GSRF_EINVAL, "out is NULL");
  Layout L;
  gsrf_status st = plan(p, &L, false);
  if (st != GSRF_OK) return st;
  out->rec_key = L.rec_key;
  out->rec_rect = L.rec_rect;
  out->rec_base = L.rec_base;
  out->counters = L.counters;
  out->sorted_klo = L.klo;
  out->sorted_val = L.val;
  out->tile_start = L.tile_start;
  out->tile_end = L.tile_end;
  out->n_records = L.n_records;
  out->n_tiles = L.T;
  out->n_tiles_az = L.nta;
  return GSRF_OK;
}

gsrf_status gsrf_project(const gsrf_problem *p, void *stream) {
  Layout L;
  gsrf_status st = plan(p, &L, true);
  if (st != GSRF_OK) return st;
  return dev(launch_project(p, L, (char *)p->workspace, (hipStream_t)stream), "gsrf_project");
}

gsrf_status gsrf_splat_count(const gsrf_problem *p, int64_t *n_splats, void *stream) {
  if (!n_splats) return fail(GSRF_EINVAL, "n_splats is NULL");
  Layout L;
  gsrf_status st = plan(p, &L, true);
  if (st != GSRF_OK) return st;
  int64_t c[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(c, (char *)p->workspace + L.counters, sizeof(c), hipMemcpyDeviceToHost,
                                (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return dev(e, "gsrf_splat_count");
  *n_splats = c[0];
  if (c[0] > L.cap) return fail(GSRF_ECAPACITY, "%lld splats exceed capacity %lld", (long long)c[0], (long long)L.cap);
  return GSRF_OK;
}

gsrf_status gsrf_ray_hit_count(const gsrf_problem *p, int64_t *n_hits, void *stream) {
  if (!n_hits) return fail(GSRF_EINVAL, "n_hits is NULL");
  Layout L;
  gsrf_status st = plan(p, &L, true);
  if (st != GSRF_OK) return st;
  if (!p->grid.depth_order) return fail(GSRF_EINVAL, "gsrf_ray_hit_count needs depth_order = 1");
  int64_t c[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(c, (char *)p->workspace + L.counters, sizeof(c), hipMemcpyDeviceToHost,
                                (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return dev(e, "gsrf_ray_hit_count");
  *n_hits = c[2];
  if (c[2] > L.hit_cap)
    return fail(GSRF_ECAPACITY, "%lld hit records exceed capacity %lld", (long long)c[2], (long long)L.hit_cap);
  return GSRF_OK;
}

gsrf_status gsrf_bin_sort(const gsrf_problem *p, void *stream) {
  Layout L;
  gsrf_status st = plan(p, &L, true);
  if (st != GSRF_OK) return st;
  return dev(launch_bin_sort(p, L, (char *)p->workspace, (hipStream_t)stream), "gsrf_bin_sort");
}

gsrf_status gsrf_render_fwd(const gsrf_problem *p, float *signal, float *signal_sum, float *rssi_dbm, void *stream) {
  Layout L;
  gsrf_status st = plan(p, &L, true);
  if (st != GSRF_OK) return st;
  if (p->n_pairs > 0 && (!signal || !signal_sum)) return fail(GSRF_EINVAL, "signal or signal_sum is NULL");
  return dev(launch_render_fwd(p, L, (char *)p->workspace, signal, signal_sum, rssi_dbm, (hipStream_t)stream),
             "gsrf_render_fwd");
}

gsrf_status gsrf_render_fwd_multi(const gsrf_problem *p, int32_t n_freq, double freq_step_hz, float *signal,
                                  float *signal_sum, void *stream) {
  if (!p) return fail(GSRF_EINVAL, "problem is NULL");
  if (n_freq < 1 || n_freq > kMaxCarriers) return fail(GSRF_EINVAL, "n_freq = %d outside [1, %d]", n_freq, kMaxCarriers);
  if (!(freq_step_hz >= 0.0) || !(freq_step_hz < 1e12)) return fail(GSRF_EINVAL, "freq_step_hz = %g", freq_step_hz);
  if (p->grid.lanes_per_ray != 0)
    return fail(GSRF_ENOTSUP, "the multi-carrier forward uses the two-phase traversal (lanes_per_ray = 0)");
  if (has_variant(p->grid)) return fail(GSRF_ENOTSUP, "the multi-carrier forward has no paper-literal variants");
  Layout L;
  gsrf_status st = plan(p, &L, true);
  if (st != GSRF_OK) return st;
  if (p->n_pairs > 0 && (!signal || !signal_sum)) return fail(GSRF_EINVAL, "signal or signal_sum is NULL");
  return dev(launch_render_fwd_multi(p, L, (char *)p->workspace, n_freq, freq_step_hz, signal, signal_sum,
                                     (hipStream_t)stream),
             "gsrf_render_fwd_multi");
}

gsrf_status gsrf_render_bwd(const gsrf_problem *p, const float *signal, const float *grad_signal,
                            const float *grad_sum, float *d_means, float *d_log_scales, float *d_quats,
                            float *d_logits, float *d_coeffs, void *stream) {
  Layout L;
  gsrf_status st = plan(p, &L, true);
  if (st != GSRF_OK) return st;
  if (p->n_pairs > 0 && (!signal || !grad_signal)) return fail(GSRF_EINVAL, "signal or grad_signal is NULL");
  if (p->n_gauss > 0 && (!d_means || !d_log_scales || !d_quats || !d_logits || !d_coeffs))
    return fail(GSRF_EINVAL, "a gradient output pointer is NULL");
  if (has_variant(p->grid)) return fail(GSRF_ENOTSUP, "no adjoint for the paper-literal render variants");
  return dev(launch_render_bwd(p, L, (char *)p->workspace, signal, grad_signal, grad_sum, d_means, d_log_scales,
                               d_quats, d_logits, d_coeffs, (hipStream_t)stream),
             "gsrf_render_bwd");
}

gsrf_status gsrf_render_bwd_multi(const gsrf_problem *p, int32_t n_freq, double freq_step_hz,
                                  const float *grad_signal, const float *grad_sum, float *d_means,
                                  float *d_log_scales, float *d_quats, float *d_logits, float *d_coeffs,
                                  void *stream) {
  if (!p) return fail(GSRF_EINVAL, "problem is NULL");
  if (n_freq < 1 || n_freq > kMaxCarriers) return fail(GSRF_EINVAL, "n_freq = %d outside [1, %d]", n_freq, kMaxCarriers);
  if (!(freq_step_hz >= 0.0) || !(freq_step_hz < 1e12)) return fail(GSRF_EINVAL, "freq_step_hz = %g", freq_step_hz);
  if (p->grid.lanes_per_ray != 0)
    return fail(GSRF_ENOTSUP, "the multi-carrier adjoint uses the two-phase traversal (lanes_per_ray = 0)");
  if (has_variant(p->grid)) return fail(GSRF_ENOTSUP, "no adjoint for the paper-literal render variants");
  Layout L;
  gsrf_status st = plan(p, &L, true);
  if (st != GSRF_OK) return st;
  if (p->n_pairs > 0 && !grad_signal) return fail(GSRF_EINVAL, "grad_signal is NULL");
  if (p->n_gauss > 0 && (!d_means || !d_log_scales || !d_quats || !d_logits || !d_coeffs))
    return fail(GSRF_EINVAL, "a gradient output pointer is NULL");
  return dev(launch_render_bwd_multi(p, L, (char *)p->workspace, n_freq, freq_step_hz, grad_signal, grad_sum, d_means,
                                     d_log_scales, d_quats, d_logits, d_coeffs, (hipStream_t)stream),
             "gsrf_render_bwd_multi");
}

gsrf_status gsrf_render_stats(const gsrf_problem *p, int64_t *counts, void *stream) {
  Layout L;
  gsrf_status st = plan(p, &L, true);
  if (st != GSRF_OK) return st;
  if (!counts) return fail(GSRF_EINVAL, "counts is NULL");
  if (has_variant(p->grid)) return fail(GSRF_ENOTSUP, "no traversal counters for the paper-literal render variants");
  return dev(launch_render_stats(p, L, (char *)p->workspace, counts, (hipStream_t)stream), "gsrf_render_stats");
}

static gsrf_status check_spectrum(int32_t n_pairs, int32_t n_el, int32_t n_az) {
  if (n_pairs < 0 || n_pairs > 65535) return fail(GSRF_EINVAL, "n_pairs = %d outside [0, 65535]", n_pairs);
  if (n_el < 1 || n_az < 1 || n_el > 65535 || n_az > 65535)
    return fail(GSRF_EINVAL, "spectrum %d x %d out of range [1, 65535]", n_el, n_az);
  return GSRF_OK;
}

gsrf_status gsrf_loss_workspace_size(int32_t n_pairs, int32_t n_el, int32_t n_az, size_t *bytes) {
  if (!bytes) return fail(GSRF_EINVAL, "bytes is NULL");
  const gsrf_status st = check_spectrum(n_pairs, n_el, n_az);
  if (st != GSRF_OK) return st;
  *bytes = loss_partials_bytes(n_pairs, n_el, n_az);
  return GSRF_OK;
}

gsrf_status gsrf_loss_spectrum(const float *signal, const float *target, int32_t n_pairs, int32_t n_el,
                               int32_t n_az, float power_scale, float lambda1, float lambda2, float *loss,
                               float *grad_signal, void *workspace, void *stream) {
  const gsrf_status st = check_spectrum(n_pairs, n_el, n_az);
  if (st != GSRF_OK) return st;
  if (!(power_scale > 0.f) || !isfinite(power_scale))
    return fail(GSRF_EINVAL, "power_scale = %g: must be finite and > 0", (double)power_scale);
  if (!isfinite(lambda1) || !isfinite(lambda2))
    return fail(GSRF_EINVAL, "lambda1 = %g, lambda2 = %g: must be finite", (double)lambda1, (double)lambda2);
  if (n_pairs > 0 && (!signal || !target || !loss || !workspace))
    return fail(GSRF_EINVAL, "signal, target, loss or workspace is NULL");
  return dev(launch_loss_spectrum(signal, target, n_pairs, n_el, n_az, power_scale, lambda1, lambda2, loss, grad_signal,
                                  workspace, (hipStream_t)stream),
             "gsrf_loss_spectrum");
}

gsrf_status gsrf_loss_spectrum_noalloc(const float *signal, const float *target, int32_t n_pairs, int32_t n_el,
                                       int32_t n_az, float power_scale, float lambda1, float lambda2, float *loss,
                                       float *grad_signal, void *stream) {
  const gsrf_status st = check_spectrum(n_pairs, n_el, n_az);
  if (st != GSRF_OK) return st;
  if (!(power_scale > 0.f) || !isfinite(power_scale))
    return fail(GSRF_EINVAL, "power_scale = %g: must be finite and > 0", (double)power_scale);
  if (!isfinite(lambda1) || !isfinite(lambda2))
    return fail(GSRF_EINVAL, "lambda1 = %g, lambda2 = %g: must be finite", (double)lambda1, (double)lambda2);
  const size_t need = loss_partials_bytes(n_pairs, n_el, n_az);
  if (need > loss_scratch_bytes())
    return fail(GSRF_ECAPACITY,
                "%d spectra of %d x %d rays need %zu bytes of partial sums; the fixed scratch holds %zu "
                "(use gsrf_loss_spectrum with a workspace)",
                n_pairs, n_el, n_az, need, loss_scratch_bytes());
  if (n_pairs > 0 && (!signal || !target || !loss)) return fail(GSRF_EINVAL, "signal, target or loss is NULL");
  if (n_pairs == 0) return GSRF_OK;
  void *ws = nullptr;
  const hipError_t e = loss_scratch_address((hipStream_t)stream, &ws);
  if (e == hipErrorInvalidDevice)
    return fail(GSRF_EINVAL, "the stream's device is not the current device (or the device index is above 63)");
  if (e != hipSuccess) return dev(e, "gsrf_loss_spectrum_noalloc: scratch address");
  return dev(launch_loss_spectrum(signal, target, n_pairs, n_el, n_az, power_scale, lambda1, lambda2, loss, grad_signal,
                                  ws, (hipStream_t)stream),
             "gsrf_loss_spectrum_noalloc");
}

gsrf_status gsrf_loss_single(const float *signal_sum, const float *target, int32_t n_pairs, int32_t kind,
                             float *loss, float *grad_sum, void *stream) {
  if (n_pairs < 0) return fail(GSRF_EINVAL, "n_pairs = %d is negative", n_pairs);
  if (kind != GSRF_LOSS_RSSI_DB && kind != GSRF_LOSS_COMPLEX_L2) return fail(GSRF_EINVAL, "loss kind %d", kind);
  if (n_pairs > 0 && (!signal_sum || !target || !loss)) return fail(GSRF_EINVAL, "signal_sum, target or loss is NULL");
  return dev(launch_loss_single(signal_sum, target, n_pairs, kind, loss, grad_sum, (hipStream_t)stream),
             "gsrf_loss_single");
}

gsrf_status gsrf_sgd_step(int64_t n_gauss, int32_t fle_L, float *means, float *log_scales, float *quats,
                          float *logits, float *coeffs, const float *d_means, const float *d_log_scales,
                          const float *d_quats, const float *d_logits, const float *d_coeffs,
                          const gsrf_sgd_lr *lr, int64_t iteration, void *stream) {
  if (n_gauss < 0 || n_gauss >= ((int64_t)1 << 31)) return fail(GSRF_EINVAL, "n_gauss = %lld", (long long)n_gauss);
  if (fle_L < 0 || fle_L > 6) return fail(GSRF_EINVAL, "fle_L = %d outside [0, 6]", fle_L);
  if (!lr) return fail(GSRF_EINVAL, "lr (host) is NULL");
  if (!(lr->mean_init > 0.0) || !(lr->mean_final > 0.0) || !isfinite(lr->mean_init) || !isfinite(lr->mean_final))
    return fail(GSRF_EINVAL, "mean learning rates must be finite and > 0");
  const double rest[4] = {lr->log_scale, lr->quat, lr->logit, lr->coeff};
  for (double r : rest)
    if (!(r >= 0.0) || !isfinite(r)) return fail(GSRF_EINVAL, "learning rates must be finite and >= 0");
  if (iteration < 0) return fail(GSRF_EINVAL, "iteration = %lld is negative", (long long)iteration);
  if (n_gauss > 0 && (!means || !log_scales || !quats || !logits || !coeffs || !d_means || !d_log_scales ||
                      !d_quats || !d_logits || !d_coeffs))
    return fail(GSRF_EINVAL, "a parameter or gradient pointer is NULL");
  double t = 1.0;
  if (lr->mean_steps > 0) t = fmin(fmax((double)iteration / (double)lr->mean_steps, 0.0), 1.0);
  const double eta_mu = exp((1.0 - t) * log(lr->mean_init) + t * log(lr->mean_final));
  float *const w[5] = {means, log_scales, quats, logits, coeffs};
  const float *const g[5] = {d_means, d_log_scales, d_quats, d_logits, d_coeffs};
  const float eta[5] = {(float)eta_mu, (float)lr->log_scale, (float)lr->quat, (float)lr->logit, (float)lr->coeff};
  return dev(launch_sgd(n_gauss, fle_K(fle_L), w, g, eta, (hipStream_t)stream), "gsrf_sgd_step");
}

gsrf_status gsrf_grad_stats_accumulate(int64_t n_gauss, const float *d_means, float *acc, int32_t *count,
                                       void *stream) {
  if (n_gauss < 0 || n_gauss >= ((int64_t)1 << 31)) return fail(GSRF_EINVAL, "n_gauss = %lld", (long long)n_gauss);
  if (n_gauss > 0 && (!d_means || !acc || !count)) return fail(GSRF_EINVAL, "d_means, acc or count is NULL");
  return dev(launch_grad_accum(n_gauss, d_means, acc, count, (hipStream_t)stream), "gsrf_grad_stats_accumulate");
}

gsrf_status gsrf_density_workspace_size(int64_t n_gauss, size_t *bytes) {
  if (!bytes) return fail(GSRF_EINVAL, "bytes is NULL");
  if (n_gauss < 0 || n_gauss >= ((int64_t)1 << 31)) return fail(GSRF_EINVAL, "n_gauss = %lld", (long long)n_gauss);
  *bytes = density_workspace_bytes(n_gauss);
  return GSRF_OK;
}

gsrf_status gsrf_density_control(int64_t n_gauss, int32_t fle_L, const float *means, const float *log_scales,
                                 const float *quats, const float *logits, const float *coeffs, const float *acc,
                                 const int32_t *count, const float *z_draws, const gsrf_density_params *params,
                                 int64_t out_capacity, float *o_means, float *o_log_scales, float *o_quats,
                                 float *o_logits, float *o_coeffs, float *o_acc, int32_t *o_count, int64_t *counts,
                                 void *workspace, void *stream) {
  if (n_gauss < 0 || n_gauss >= ((int64_t)1 << 30)) return fail(GSRF_EINVAL, "n_gauss = %lld", (long long)n_gauss);
  if (fle_L < 0 || fle_L > 6) return fail(GSRF_EINVAL, "fle_L = %d outside [0, 6]", fle_L);
  if (!params) return fail(GSRF_EINVAL, "params (host) is NULL");
  const gsrf_density_params &d = *params;
  if (!(d.eps_mu >= 0.0) || !isfinite(d.eps_mu) || !(d.eps_r >= 0.0) || !isfinite(d.eps_r) || !isfinite(d.eps_rho) ||
      !(d.phi > 1.0) || !isfinite(d.phi) || !isfinite(d.clone_step))
    return fail(GSRF_EINVAL, "density thresholds: need finite eps_mu, eps_r >= 0, eps_rho, clone_step and phi > 1");
  const int64_t need = d.densify ? 2 * n_gauss : n_gauss;
  if (out_capacity < need)
    return fail(GSRF_EINVAL, "out_capacity = %lld < %lld", (long long)out_capacity, (long long)need);
  if (!counts || !workspace) return fail(GSRF_EINVAL, "counts or workspace is NULL");
  if (n_gauss > 0 && (!means || !log_scales || !quats || !logits || !coeffs || !acc || !count ||
                      (d.densify && !z_draws) || !o_means || !o_log_scales || !o_quats || !o_logits || !o_coeffs ||
                      !o_acc || !o_count))
    return fail(GSRF_EINVAL, "an input or output pointer is NULL");
  DensityIO io{};
  io.means = means; io.log_scales = log_scales; io.quats = quats; io.logits = logits; io.coeffs = coeffs;
  io.acc = acc; io.cnt = count; io.z = z_draws;
  io.n = n_gauss; io.K = fle_K(fle_L);
  io.eps_mu = d.eps_mu; io.eps_r = d.eps_r; io.eps_rho = d.eps_rho; io.clone_step = d.clone_step;
  io.ln_phi = (float)log(d.phi); io.densify = d.densify != 0; io.prune = d.prune != 0;
  io.o_means = o_means; io.o_log_scales = o_log_scales; io.o_quats = o_quats; io.o_logits = o_logits;
  io.o_coeffs = o_coeffs; io.o_acc = o_acc; io.o_cnt = o_count;
  io.counts = counts;
  io.ws = workspace;
  return dev(launch_density_control(io, (hipStream_t)stream), "gsrf_density_control");
}

gsrf_status gsrf_set_kernel_events(void *fwd_start, void *fwd_stop, void *bwd_start, void *bwd_stop) {
  g_kernel_events[0] = (hipEvent_t)fwd_start;
  g_kernel_events[1] = (hipEvent_t)fwd_stop;
  g_kernel_events[2] = (hipEvent_t)bwd_start;
  g_kernel_events[3] = (hipEvent_t)bwd_stop;
  return GSRF_OK;
}

}  // extern "C"
