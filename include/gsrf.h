/*
 * gsrf.h -- C ABI of the MI355X (gfx950) GSRF hot-path library, libgsrf.so.
 *
 * GSRF (arXiv 2502.01826) renders complex-valued 3D Gaussians onto a
 * receiver's azimuth x elevation ray grid: orthographic splatting onto the 2D
 * receiving RF plane (Sec. 3.3), per-tile depth sorting with 64-bit
 * (tile | distance) keys (App. E, Alg. 1), and complex front-to-back ray
 * accumulation (Sec. 3.4 eq. rendering; App. A), plus its adjoint (App. C
 * backward kernel; App. D gradients).
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless the comment says HOST.  Arrays are
 *     row-major, FP32 unless stated, and owned by the caller; the library
 *     never allocates or frees memory.
 *   - Every call is asynchronous on the HIP stream passed as `stream`
 *     (a hipStream_t; NULL = the null stream) and does no host
 *     synchronisation, except gsrf_splat_count, which synchronises the stream.
 *     Calls on one problem must be issued in the order
 *     project -> bin_sort -> render_fwd [-> render_bwd] on one stream.
 *   - Arguments are validated on the host before anything is launched:
 *     GSRF_EINVAL means nothing was enqueued.  GSRF_EDEVICE reports a HIP
 *     launch error.  NaN or Inf parameters are not checked; they propagate.
 *   - A problem with no Gaussians, or pairs whose scene is empty, is valid and
 *     renders exact zeros.
 */
#ifndef GSRF_H_
#define GSRF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gsrf_status {
  GSRF_OK = 0,
  GSRF_EINVAL = 1,     /* bad argument; nothing enqueued */
  GSRF_ECAPACITY = 2,  /* more splats than splat_capacity (see gsrf_splat_count) */
  GSRF_EDEVICE = 3,    /* a HIP call or kernel launch failed */
  GSRF_ENOTSUP = 4     /* valid request this build does not implement */
} gsrf_status;

/*
 * Receiver ray grid and render constants.
 *   Rays sit at cell centres of the 2D receiving RF plane (Sec. 3.3 eqs.
 *   spherical coordinates and discretization): azimuth
 *   alpha_u = 2 pi (u + 1/2) / n_az, elevation
 *   beta_v = el_lo + (el_hi - el_lo)(v + 1/2) / n_el, direction
 *   fp32(cos b cos a, cos b sin a, sin b) evaluated in FP64.
 *   fle_L      Fourier-Legendre degree L of the radiance (Sec. 3.2 eq. FLE),
 *              K = (L+1)^2 complex coefficients per Gaussian; 0 <= L <= 6.
 *   r_rx       radius of the ray-emitting spherical surface (Sec. 3.3; the
 *              paper uses 1.0): a Gaussian counts only if its chord midpoint
 *              lies at ray parameter >= r_rx.
 *   t_min      a ray stops before the first hit whose transmittance < t_min.
 *   alpha_max  opacity clamp, in (0, 1).
 *   tile_w/h   rays per tile (App. E uses 16 x 16); tile_w * tile_h must be
 *              32 (two-phase traversal only), 64, 128 or 256.
 *   lanes_per_ray  traversal of a tile's depth-ordered list by the render
 *              kernels.  0 (recommended): two-phase traversal per staged
 *              batch, all (ray, entry) hit tests first, then the per-hit work
 *              on hits only, by 256 / (tile_w * tile_h) lanes per ray (8, 4,
 *              2 or 1).
 *              1, 2 or 4: direct traversal, that many lanes per ray, each
 *              testing and processing a different entry.  Every value gives
 *              the same hit decisions; the results agree to rounding.
 *   footprint  which rays' tiles a Gaussian is binned into (Sec. 3.3,
 *              splatting).  0 (default): a cap that bounds the 3-sigma
 *              ellipsoid exactly, so binning never drops a hit.  1: the
 *              paper's footprint, the bounding square of the circle of radius
 *              3 sqrt(lambda_max(J Sigma J^T)) around the projected centre,
 *              J the Jacobian of the ray-index map at mu.  It linearises that
 *              map, so hits of a ray outside the square are dropped.  Both
 *              keep the exact per-ray 3-sigma test of the render.
 *              GSRF_EINVAL for other values.
 * The paper-literal variants of the render (each 0 = the default reading;
 * GSRF_EINVAL for values other than 0 and 1; they need lanes_per_ray = 0;
 * gsrf_render_fwd supports them, while gsrf_render_bwd, gsrf_render_fwd_multi
 * and gsrf_render_stats return GSRF_ENOTSUP when any is set):
 *   depth_order    1: every ray takes its hits in increasing chord-midpoint
 *              parameter t_mid = -B/A (App. A.3: Gaussians sorted by their
 *              midpoint times), ties in depth-key order, instead of the
 *              per-tile distance-key order.  Needs hit_capacity (gsrf_problem).
 *   fle_eval       1: the radiance psi_k is the FLE evaluated once per
 *              (pair, Gaussian) at the direction of mu_k from the receiver,
 *              instead of at each ray's direction (Sec. 3.2 eq. FLE).
 *   transmittance  1: a hit's transmittance is the chord form of App. A.2,
 *              rho = exp(-alpha_k dt) with dt = t_out - t_in the 3-sigma
 *              chord and alpha_k = exp(opacity_logit) per metre, instead of
 *              1 - min(o G, alpha_max); the propagation phase is unchanged.
 */
typedef struct gsrf_grid {
  int32_t n_az, n_el;
  float el_lo, el_hi;
  int32_t fle_L;
  float r_rx;
  float t_min;
  float alpha_max;
  int32_t tile_w, tile_h;
  int32_t lanes_per_ray;
  int32_t footprint;
  int32_t depth_order;
  int32_t fle_eval;
  int32_t transmittance;
} gsrf_grid;

/*
 * One transmitter/receiver query (Sec. 3.1 problem formulation: TX at t,
 * RX at r).  40 bytes.  freq_hz is the carrier; wavelength = 3e8 / freq_hz.
 * scene indexes the CSR scene table.
 */
typedef struct gsrf_pair {
  float rx[3];
  float tx[3];
  double freq_hz;
  int32_t scene;
  int32_t reserved;
} gsrf_pair;

/*
 * A batch: S scenes of Gaussians concatenated in one parameter set, and P
 * pairs, each rendering one scene.  Gaussian parameters (Sec. 3.2 primitive
 * zeta_k = (mu, R, S, psi, rho)):
 *   means           [G,3]    mu
 *   log_scales      [G,3]    s = exp(log_scales); Sigma = R diag(s)^2 R^T
 *   quats           [G,4]    rotation (w,x,y,z), normalised in-kernel
 *   opacity_logits  [G]      o = sigmoid(logit); transmittance 1 - o G
 *   coeffs          [G,K,2]  complex FLE coefficients c_i, i = l^2 + l + m
 * scene_offsets (HOST) and scene_offsets_dev (DEVICE) hold the same S+1
 * non-decreasing values with scene_offsets[0] = 0, scene_offsets[S] = G.
 * pair_scene (HOST, [P]) repeats pairs[k].scene for host-side sizing.
 * workspace (DEVICE, workspace_bytes >= gsrf_workspace_size) holds every
 * intermediate; it must stay untouched between the calls of one render.
 */
typedef struct gsrf_problem {
  const float *means, *log_scales, *quats, *opacity_logits, *coeffs;
  int64_t n_gauss;
  int32_t n_scenes;
  const int64_t *scene_offsets;      /* HOST [S+1] */
  const int64_t *scene_offsets_dev;  /* DEVICE [S+1] */
  const gsrf_pair *pairs;            /* DEVICE [P] */
  const int32_t *pair_scene;         /* HOST [P] */
  int32_t n_pairs;
  gsrf_grid grid;
  int64_t splat_capacity;            /* max (tile, Gaussian) splats, < 2^32 */
  void *workspace;
  size_t workspace_bytes;
  int64_t hit_capacity;              /* depth_order = 1: max (ray, Gaussian) hit records, < 2^40;
                                        ignored (may be 0) otherwise */
} gsrf_problem;

/* Byte offsets of the workspace arrays that tests and tools may read.  Tile
 * tt of pair k (global tile k * n_tiles + tt) owns sorted entries
 * [tile_start[.], tile_end[.]) of sorted_klo / sorted_val. */
typedef struct gsrf_layout {
  size_t rec_key;      /* uint32 [R]      per (pair, Gaussian) depth key bits(fp32(|mu-r|^2)) */
  size_t rec_rect;     /* uint16 [R][4]   tile rectangle (tu0, ntu, tv0, ntv) */
  size_t rec_base;     /* int64  [P+1]    first record of each pair; R = rec_base[P] */
  size_t counters;     /* int64  [4]      [0] splat count, [1] = count if over capacity else 0 */
  size_t sorted_klo;   /* uint32 [cap]    depth key of each sorted splat */
  size_t sorted_val;   /* uint32 [cap]    Gaussian index of each sorted splat */
  size_t tile_start;   /* uint32 [P*T]    first sorted splat of each tile */
  size_t tile_end;     /* uint32 [P*T]    one past the last */
  int64_t n_records;   /* R */
  int32_t n_tiles;     /* T per pair */
  int32_t n_tiles_az;  /* tile columns (azimuth) */
} gsrf_layout;

/* Human-readable status name; never NULL. */
const char *gsrf_status_str(gsrf_status s);

/* Message of the last failing call in this thread (empty if none). */
const char *gsrf_last_error(void);

/*
 * Size of the workspace for `p` (only its sizes, grid and host arrays are
 * read; device pointers may be NULL).  HOST out.
 */
gsrf_status gsrf_workspace_size(const gsrf_problem *p, size_t *bytes);

/* Workspace offsets for `p` (same reading as gsrf_workspace_size). HOST out. */
gsrf_status gsrf_layout_of(const gsrf_problem *p, gsrf_layout *out);

/*
 * Steps a1 + a2: per-Gaussian activation (Sec. 2 Sigma = R S S^T R^T; App. A.3
 * normalised pdf) and orthographic splatting of every (pair, Gaussian)
 * (Sec. 3.3 splatting process; Alg. 1 sphericalGaussian/sphericalSplatting):
 * depth key, and the tile rectangle covered by the Gaussian's bounding cap of
 * radius 3 max(s) widened by 1e-5 rad -- conservative, so binning only culls.
 * Gaussians wholly inside the RESS or outside the elevation span are culled.
 * Ends with the splat count, readable by gsrf_splat_count.
 */
gsrf_status gsrf_project(const gsrf_problem *p, void *stream);

/*
 * Synchronises `stream` and returns (HOST) the number of splats the last
 * gsrf_project produced.  Returns GSRF_ECAPACITY if it exceeds
 * splat_capacity (the caller then re-sizes and re-runs from gsrf_project).
 */
gsrf_status gsrf_splat_count(const gsrf_problem *p, int64_t *n_splats, void *stream);

/*
 * depth_order = 1 only: synchronises `stream` and returns (HOST) the number of
 * (ray, Gaussian) hit records the last gsrf_render_fwd needed (every hit of
 * every ray, before termination).  GSRF_ECAPACITY if it exceeds
 * hit_capacity: that render wrote zeros; re-size and render again.
 */
gsrf_status gsrf_ray_hit_count(const gsrf_problem *p, int64_t *n_hits, void *stream);

/*
 * Steps a3 + a4 (Alg. 1 sphericalSplatting, the 64-bit key sort of App. E,
 * computeGridRange): one splat per covered tile, placed in its tile's range
 * (counted by gsrf_project), then each tile's list sorted by depth key with
 * ties broken by Gaussian index -- the order a sort of all splats by
 * (tile << 32 | depth key) would give.  If the splat count exceeds
 * splat_capacity the device-side overflow counter is set, every tile list is
 * left empty and renders give zeros; gsrf_splat_count reports it.  Each call
 * consumes the emission cursors (and, for more than 2048 (pair, tile) units,
 * the queue of long buckets) that the preceding gsrf_project left in the
 * workspace, so every gsrf_bin_sort follows its own gsrf_project.
 */
gsrf_status gsrf_bin_sort(const gsrf_problem *p, void *stream);

/*
 * Steps a5 + a6 (Sec. 3.4 eq. rendering; App. A; Alg. 1 Blend): for every
 * ray, in tile depth order, a Gaussian is hit iff B^2 - A(C - 9) >= 0 and the
 * chord midpoint t = -B/A >= r_rx (App. D.3.3); it adds T * N G(x_mid) * psi *
 * e^{-j 2 pi (|mu - tx| + t)/lambda} and multiplies T by
 * 1 - min(o G(x_mid), alpha_max); the ray stops before a hit with T < t_min.
 *   signal      [P, n_el, n_az, 2]  complex received signal per ray (re, im)
 *   signal_sum  [P, 2]              S_hat = sum over rays (Sec. 3.4 single antenna)
 *   rssi_dbm    [P] or NULL         10 log10 |S_hat|^2 (-inf when S_hat = 0)
 * Deterministic: repeated calls give bit-identical outputs.
 */
gsrf_status gsrf_render_fwd(const gsrf_problem *p, float *signal, float *signal_sum, float *rssi_dbm,
                            void *stream);

/*
 * Multi-carrier forward (OFDM subcarriers, the 5G CSI synthesis of Sec. 4;
 * each path's phase is 2 pi f tau, Sec. 2): the render of gsrf_render_fwd for
 * n_freq carriers per pair, carrier c of pair k at
 * pairs[k].freq_hz + c * freq_step_hz.  Hit decisions, transmittance, N G and
 * psi do not depend on the carrier, so one traversal serves up to 32
 * carriers and the propagation phase is the only per-carrier term.
 *   n_freq        1 .. 4096 carriers per pair
 *   freq_step_hz  carrier spacing, >= 0 (Hz)
 *   signal        [P, n_freq, n_el, n_az, 2]  complex received signal (re, im)
 *   signal_sum    [P, n_freq, 2]              S_hat per pair and carrier
 * Needs lanes_per_ray = 0 (GSRF_ENOTSUP otherwise).  Follows gsrf_bin_sort
 * like gsrf_render_fwd; it leaves the forward's hit masks untouched, so it
 * may sit between gsrf_render_fwd and gsrf_render_bwd.  Deterministic.
 */
gsrf_status gsrf_render_fwd_multi(const gsrf_problem *p, int32_t n_freq, double freq_step_hz, float *signal,
                                  float *signal_sum, void *stream);

/*
 * Steps a7 + a8 (App. C backward kernel; App. D gradients, including the
 * covariance chain the paper omits): recomputes each ray's transmittance
 * front to back and forms the gradient of L with respect to every
 * parameter, where the caller supplies dL/dS per ray and per pair.  Must
 * follow gsrf_render_fwd of the same prepared problem on the same workspace:
 * the remainder sum_{i>j} T_i c~_i of each hit is that forward's S minus the
 * running prefix, with S taken from the FP64 copy the forward leaves in the
 * workspace (so the remainder stays accurate to its own size, zero after a
 * ray's last hit, rather than to |S|); with lanes_per_ray = 0 it also reuses
 * the per-list-entry hit masks recorded there.  No other per-ray state is
 * kept between the passes.
 *   signal       [P, n_el, n_az, 2]  the render_fwd output for this problem
 *                (checked for NULL; the values used are the workspace's FP64
 *                copy of it)
 *   grad_signal  [P, n_el, n_az, 2]  dL/dRe S + j dL/dIm S
 *   grad_sum     [P, 2] or NULL      dL/dS_hat (added to every ray of the pair)
 * Outputs are OVERWRITTEN (not accumulated), summed over all pairs:
 *   d_means [G,3], d_log_scales [G,3], d_quats [G,4], d_logits [G], d_coeffs [G,K,2].
 * Discrete decisions (hit test, termination, clamp) are treated as constant.
 * Uses float atomics, so results are reproducible only to rounding.
 */
gsrf_status gsrf_render_bwd(const gsrf_problem *p, const float *signal, const float *grad_signal,
                            const float *grad_sum, float *d_means, float *d_log_scales, float *d_quats,
                            float *d_logits, float *d_coeffs, void *stream);

/*
 * Adjoint of the multi-carrier forward (the CSI vectors of Sec. 4 train one
 * set of Gaussians on every subcarrier; each path's phase is 2 pi f tau,
 * Sec. 2): the gradient of L = sum_c L_c with respect to every parameter,
 * where carrier c of pair k is at pairs[k].freq_hz + c * freq_step_hz and the
 * caller supplies each carrier's dL/dS per ray and per pair.  Equals the sum
 * over carriers of gsrf_render_bwd at each carrier's frequency, in one
 * traversal per 16 carriers instead of one per carrier: the carriers share
 * the hit decisions and transmittance, and the adjoint of every carrier's
 * phase is folded into two complex weights per hit.  Must follow
 * gsrf_render_fwd of the same prepared problem on the same workspace (it
 * reuses the hit masks recorded there; the hit decisions do not depend on the
 * carrier); the forward's multi-carrier output is not needed -- each chunk of
 * carriers first sums sum_c Re(conj(G_c) S_c) per ray in FP64 over the same
 * hits, so the remainders are accurate to their own size.
 *   n_freq        1 .. 4096 carriers per pair
 *   freq_step_hz  carrier spacing, >= 0 (Hz)
 *   grad_signal   [P, n_freq, n_el, n_az, 2]  dL/dRe S + j dL/dIm S per carrier
 *   grad_sum      [P, n_freq, 2] or NULL      dL/dS_hat per pair and carrier
 * Outputs OVERWRITTEN, summed over pairs and carriers, as gsrf_render_bwd.
 * Needs lanes_per_ray = 0 (GSRF_ENOTSUP otherwise, and for the paper-literal
 * variants).
 */
gsrf_status gsrf_render_bwd_multi(const gsrf_problem *p, int32_t n_freq, double freq_step_hz,
                                  const float *grad_signal, const float *grad_sum, float *d_means,
                                  float *d_log_scales, float *d_quats, float *d_logits, float *d_coeffs,
                                  void *stream);

/*
 * Instrumentation for the roofline: replays the render_fwd traversal of a
 * problem prepared by gsrf_project + gsrf_bin_sort without writing any
 * output, and stores (DEVICE, int64 [6], overwritten) the number of
 * (ray, Gaussian) hit tests made, processed hits, staged list entries, rays,
 * tile tests (sum over tiles of rays in the tile times list entries up to
 * the tile's termination: the tests the tiled method implies), and walk
 * slots (two-phase traversal only, else 0: 64 per step of a phase-2 wave, so
 * processed hits / walk slots is the share of phase-2 lanes doing per-hit work).
 */
gsrf_status gsrf_render_stats(const gsrf_problem *p, int64_t *counts, void *stream);

/*
 * Instrumentation for kernel timing: every later gsrf_render_fwd records
 * fwd_start / fwd_stop (hipEvent_t, caller-created; NULL = none) on its stream
 * immediately before and after its render kernel (gsrf_render_fwd_multi:
 * around all of its carrier-chunk traversals), and every gsrf_render_bwd
 * does the same with bwd_start / bwd_stop around its adjoint kernel.  The
 * setting is process-wide; pass NULLs to switch it off.  Never fails.
 */
gsrf_status gsrf_set_kernel_events(void *fwd_start, void *fwd_stop, void *bwd_start, void *bwd_stop);

/* ------------------------------------------------------------------------
 * Training steps either side of the render (Sec. 3.4 loss function;
 * App. Gaussian primitive optimization).  These take plain arrays, not a
 * problem, and follow the stream-order and validation rules above.
 * ------------------------------------------------------------------------ */

/*
 * Device workspace (bytes) that gsrf_loss_spectrum needs for n_pairs spectra
 * of n_el x n_az rays (per-tile FP64 partial sums).  0 when n_pairs = 0.
 */
gsrf_status gsrf_loss_workspace_size(int32_t n_pairs, int32_t n_el, int32_t n_az, size_t *bytes);

/*
 * Antenna-array loss (Sec. 3.4, loss function) of each pair's spatial
 * spectrum and its gradient with respect to the rendered rays.  The predicted
 * spectrum is the power x = power_scale * |S_uv|^2 of every ray (power_scale
 * > 0 a fixed normalisation, e.g. 1 / the largest measured power, since
 * spectra are compared as normalised images), the target y a measured
 * spectrum of the same shape, N = n_el * n_az:
 *   L = (1 - lambda1 - lambda2) L1 + lambda1 L_SSIM + lambda2 L_Fourier,
 *   L1 = (1/N) sum |x - y|,  L_SSIM = 1 - mean SSIM(x, y),
 *   L_Fourier = (1/N) sum over frequency pairs |F(x) - F(y)|^2 with F the
 *   unnormalised 2D DFT (by Parseval equal to sum (x - y)^2, which is what
 *   is computed).
 * SSIM: 11 x 11 Gaussian window of sigma 1.5, zero padding outside the
 * spectrum, C1 = 0.01^2, C2 = 0.03^2, averaged over all N pixels (the paper
 * gives no window or constants; these are the 3D Gaussian splatting ones).
 * The paper gives no values for lambda1, lambda2 either.
 *   signal       [P, n_el, n_az, 2]  rendered rays (gsrf_render_fwd output)
 *   target       [P, n_el, n_az]     target power spectra
 *   loss         [P, 4]              per pair: L, L1, L_SSIM, L_Fourier
 *   grad_signal  [P, n_el, n_az, 2] or NULL: dL_k/dRe S + j dL_k/dIm S for
 *                each pair's own loss L_k (= 2 power_scale dL_k/dx * S), the form
 *                gsrf_render_bwd takes; overwritten.  d|x - y|/dx at 0 is 0.
 *   workspace    gsrf_loss_workspace_size bytes (device), may be NULL when
 *                n_pairs = 0.
 * 1 <= n_el, n_az <= 65535, 0 <= n_pairs <= 65535, lambdas finite.
 * Deterministic (fixed-order sums).
 */
gsrf_status gsrf_loss_spectrum(const float *signal, const float *target, int32_t n_pairs, int32_t n_el,
                               int32_t n_az, float power_scale, float lambda1, float lambda2, float *loss,
                               float *grad_signal, void *workspace, void *stream);

/*
 * gsrf_loss_spectrum without a workspace argument and without any device
 * allocation, for callers that cannot allocate: code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Arguments, outputs,
 * validation and results are those of gsrf_loss_spectrum (the same kernels);
 * the per-tile FP64 partial sums live in a fixed 1 MiB device array of the
 * library instead (one copy per GPU, held until the process ends), so
 *   n_pairs * ceil(n_el / 16) * ceil(n_az / 32) * 24 bytes <= 1 MiB
 * (606 spectra of 360 x 90 rays) and larger calls fail with GSRF_ECAPACITY
 * before anything is enqueued.  The first call on a device looks the array's
 * address up (hipGetSymbolAddress, no allocation); call it with the stream's
 * device current (GSRF_EINVAL otherwise).  Every call on a GPU shares that
 * GPU's array: calls that may overlap on one GPU (different streams without
 * ordering between them) race and must not be issued.  Nothing in the array
 * has to start at zero; it keeps the last call's partial sums.
 */
gsrf_status gsrf_loss_spectrum_noalloc(const float *signal, const float *target, int32_t n_pairs, int32_t n_el,
                                       int32_t n_az, float power_scale, float lambda1, float lambda2, float *loss,
                                       float *grad_signal, void *stream);

/* Loss kinds of gsrf_loss_single. */
typedef enum gsrf_loss_kind {
  GSRF_LOSS_RSSI_DB = 0,      /* |10 log10 |S_hat|^2 - t|, t an RSSI in dBm (target [P]) */
  GSRF_LOSS_COMPLEX_L2 = 1    /* |S_hat - t|^2, t complex (target [P, 2]) */
} gsrf_loss_kind;

/*
 * Single-antenna loss (Sec. 3.4: L1 when the measurement is a power, squared
 * L2 when it is a complex signal) of each pair's S_hat = sum_uv S_uv.
 *   signal_sum  [P, 2]  (gsrf_render_fwd's S_hat)
 *   target      [P] (RSSI in dBm) or [P, 2] (complex), by kind
 *   loss        [P]     per pair
 *   grad_sum    [P, 2] or NULL: dL_k/dRe S_hat + j dL_k/dIm S_hat, the
 *               grad_sum argument of gsrf_render_bwd.  For GSRF_LOSS_RSSI_DB
 *               and S_hat = 0 the loss is +inf and the gradient 0.
 * Computed in FP64, rounded to FP32.  0 <= n_pairs; kind one of the above.
 */
gsrf_status gsrf_loss_single(const float *signal_sum, const float *target, int32_t n_pairs, int32_t kind,
                             float *loss, float *grad_sum, void *stream);

/*
 * Learning rates of gsrf_sgd_step (App. training gives mean 1.6e-4 decaying
 * exponentially to 1.6e-6 over 30000 iterations, scaling 0.01, rotation
 * 0.005, attenuation 0.01, emission 0.0025).
 */
typedef struct gsrf_sgd_lr {
  double mean_init, mean_final;  /* > 0 */
  int64_t mean_steps;            /* iterations of the decay; <= 0: final rate throughout */
  double log_scale, quat, logit, coeff;   /* >= 0 */
} gsrf_sgd_lr;

/*
 * SGD on every attribute of every Gaussian in one launch (App. attribute
 * updating, eq. updating): w <- w - eta_w * dL/dw, rounded once (FMA), in
 * place.  eta for the means at iteration j: exp((1 - t) ln mean_init +
 * t ln mean_final), t = min(j / mean_steps, 1), evaluated in FP64 on the host
 * and rounded to FP32 like the other rates.  The quaternion is updated as
 * stored (the render normalises it).
 *   means [G,3], log_scales [G,3], quats [G,4], logits [G], coeffs [G,K,2]
 *   (K = (fle_L + 1)^2) and the gradients in the same layouts
 *   (gsrf_render_bwd's outputs); lr HOST; iteration >= 0.
 */
gsrf_status gsrf_sgd_step(int64_t n_gauss, int32_t fle_L, float *means, float *log_scales, float *quats,
                          float *logits, float *coeffs, const float *d_means, const float *d_log_scales,
                          const float *d_quats, const float *d_logits, const float *d_coeffs,
                          const gsrf_sgd_lr *lr, int64_t iteration, void *stream);

/*
 * Adaptive density control (App. number of Gaussian updating).  Over a window
 * of N_mu iterations the caller accumulates each Gaussian's mean gradient;
 * then gsrf_density_control clones, splits and prunes in one pass.
 *
 * gsrf_grad_stats_accumulate: acc[G,3] += d_means[G,3] (one FP32 add per
 * component, so the sum is exact to the iteration order) and count[G] += 1
 * where d_means is not zero (the Gaussian was hit).  Start a window with both
 * zeroed; gsrf_density_control zeroes its outputs' statistics.
 */
gsrf_status gsrf_grad_stats_accumulate(int64_t n_gauss, const float *d_means, float *acc, int32_t *count,
                                       void *stream);

/* Thresholds of gsrf_density_control (App. parameter table: eps_mu = 0.0002,
 * eps_r = 10, eps_rho = 0.004, phi = 1.6). */
typedef struct gsrf_density_params {
  double eps_mu;      /* mean-gradient threshold: |acc / count| > eps_mu selects */
  double eps_r;       /* radius threshold: mean of diag Sigma > eps_r splits, else clones */
  double eps_rho;     /* attenuation threshold: sigmoid(logit) < eps_rho prunes */
  double phi;         /* split scale divisor (> 1) */
  double clone_step;  /* a clone's copy moves to mu - clone_step * acc / count */
  int32_t densify;    /* 0: no clone or split this call */
  int32_t prune;      /* 0: no pruning this call */
} gsrf_density_params;

/* Device workspace (bytes) of gsrf_density_control for n_gauss Gaussians. */
gsrf_status gsrf_density_workspace_size(int64_t n_gauss, size_t *bytes);

/*
 * Clone, split and prune (App. number of Gaussian updating), every decision
 * in FP64:
 *   selected  densify and count > 0 and |acc| > eps_mu * count;
 *   clone     selected with radius = mean of the diagonal of R S S^T R^T
 *             <= eps_r: the Gaussian and a copy whose mean is
 *             mu - clone_step * acc / count (the shift along the averaged
 *             gradient's descent direction);
 *   split     selected with radius > eps_r: two Gaussians with log-scales
 *             reduced by ln(phi) and means mu + R diag(s) z_c drawn from the
 *             original pdf, z = z_draws[i, c, :] (standard normal, caller's);
 *   pruned    prune and sigmoid(logit) < eps_rho (also when selected).
 * Every other attribute is copied.  Output order is stable: the outputs of
 * Gaussian i precede those of i + 1, an original precedes its copy.
 *   inputs     means [G,3], log_scales [G,3], quats [G,4], logits [G],
 *              coeffs [G,K,2] (K = (fle_L + 1)^2), acc [G,3], count [G],
 *              z_draws [G,2,3] (may be NULL when densify = 0)
 *   outputs    o_* in the same layouts with room for out_capacity Gaussians:
 *              out_capacity >= 2 G when densify, >= G otherwise; o_acc and
 *              o_count are zeroed for the new window.  Outputs must not
 *              overlap inputs.
 *   counts     [4] int64 (device): Gaussians out, clones, splits, pruned
 *   workspace  gsrf_density_workspace_size bytes (device)
 *   params     HOST
 * The new count is known on the device only: read counts[0] before using
 * the outputs.
 */
gsrf_status gsrf_density_control(int64_t n_gauss, int32_t fle_L, const float *means, const float *log_scales,
                                 const float *quats, const float *logits, const float *coeffs, const float *acc,
                                 const int32_t *count, const float *z_draws, const gsrf_density_params *params,
                                 int64_t out_capacity, float *o_means, float *o_log_scales, float *o_quats,
                                 float *o_logits, float *o_coeffs, float *o_acc, int32_t *o_count, int64_t *counts,
                                 void *workspace, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GSRF_H_ */
