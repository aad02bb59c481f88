"""ctypes binding of libgsrf.so (argument marshalling only).

The structures mirror include/gsrf.h field for field.  torch is imported
before the library is loaded so that libgsrf.so binds to the HIP runtime
torch already loaded (both carry the soname libamdhip64.so.7): one runtime
per process, so torch's device pointers and streams are valid for our
kernels.  A missing library raises immediately -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must load the HIP runtime first)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsrf.so")

GSRF_OK, GSRF_EINVAL, GSRF_ECAPACITY, GSRF_EDEVICE, GSRF_ENOTSUP = range(5)

c_i32, c_i64, c_f32, c_f64, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double,
                                          ctypes.c_void_p, ctypes.c_size_t)


class GsrfGrid(ctypes.Structure):
    _fields_ = [("n_az", c_i32), ("n_el", c_i32), ("el_lo", c_f32), ("el_hi", c_f32), ("fle_L", c_i32),
                ("r_rx", c_f32), ("t_min", c_f32), ("alpha_max", c_f32), ("tile_w", c_i32), ("tile_h", c_i32),
                ("lanes_per_ray", c_i32), ("footprint", c_i32), ("depth_order", c_i32), ("fle_eval", c_i32),
                ("transmittance", c_i32)]


class GsrfPair(ctypes.Structure):
    _fields_ = [("rx", c_f32 * 3), ("tx", c_f32 * 3), ("freq_hz", c_f64), ("scene", c_i32), ("reserved", c_i32)]


class GsrfProblem(ctypes.Structure):
    _fields_ = [("means", c_vp), ("log_scales", c_vp), ("quats", c_vp), ("opacity_logits", c_vp), ("coeffs", c_vp),
                ("n_gauss", c_i64), ("n_scenes", c_i32), ("scene_offsets", c_vp), ("scene_offsets_dev", c_vp),
                ("pairs", c_vp), ("pair_scene", c_vp), ("n_pairs", c_i32), ("grid", GsrfGrid),
                ("splat_capacity", c_i64), ("workspace", c_vp), ("workspace_bytes", c_sz), ("hit_capacity", c_i64)]


class GsrfLayout(ctypes.Structure):
    _fields_ = [("rec_key", c_sz), ("rec_rect", c_sz), ("rec_base", c_sz), ("counters", c_sz),
                ("sorted_klo", c_sz), ("sorted_val", c_sz), ("tile_start", c_sz),
                ("tile_end", c_sz), ("n_records", c_i64), ("n_tiles", c_i32), ("n_tiles_az", c_i32)]


class GsrfSgdLr(ctypes.Structure):
    _fields_ = [("mean_init", c_f64), ("mean_final", c_f64), ("mean_steps", c_i64), ("log_scale", c_f64),
                ("quat", c_f64), ("logit", c_f64), ("coeff", c_f64)]


class GsrfDensityParams(ctypes.Structure):
    _fields_ = [("eps_mu", c_f64), ("eps_r", c_f64), ("eps_rho", c_f64), ("phi", c_f64), ("clone_step", c_f64),
                ("densify", c_i32), ("prune", c_i32)]


assert ctypes.sizeof(GsrfPair) == 40

GSRF_LOSS_RSSI_DB, GSRF_LOSS_COMPLEX_L2 = 0, 1

EXPORTS = ["gsrf_status_str", "gsrf_last_error", "gsrf_workspace_size", "gsrf_layout_of", "gsrf_project",
           "gsrf_splat_count", "gsrf_ray_hit_count", "gsrf_bin_sort", "gsrf_render_fwd", "gsrf_render_fwd_multi", "gsrf_render_bwd",
           "gsrf_render_bwd_multi", "gsrf_render_stats",
           "gsrf_set_kernel_events", "gsrf_loss_workspace_size", "gsrf_loss_spectrum", "gsrf_loss_spectrum_noalloc",
           "gsrf_loss_single",
           "gsrf_sgd_step", "gsrf_grad_stats_accumulate", "gsrf_density_workspace_size", "gsrf_density_control"]

_lib = None


def lib() -> ctypes.CDLL:
    """Load libgsrf.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_01826_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.gsrf_status_str.restype = ctypes.c_char_p
    L.gsrf_status_str.argtypes = [c_i32]
    L.gsrf_last_error.restype = ctypes.c_char_p
    L.gsrf_last_error.argtypes = []
    L.gsrf_workspace_size.argtypes = [P(GsrfProblem), P(c_sz)]
    L.gsrf_layout_of.argtypes = [P(GsrfProblem), P(GsrfLayout)]
    L.gsrf_project.argtypes = [P(GsrfProblem), c_vp]
    L.gsrf_splat_count.argtypes = [P(GsrfProblem), P(c_i64), c_vp]
    L.gsrf_ray_hit_count.argtypes = [P(GsrfProblem), P(c_i64), c_vp]
    L.gsrf_bin_sort.argtypes = [P(GsrfProblem), c_vp]
    L.gsrf_render_fwd.argtypes = [P(GsrfProblem), c_vp, c_vp, c_vp, c_vp]
    L.gsrf_render_bwd.argtypes = [P(GsrfProblem), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]
    L.gsrf_render_bwd_multi.argtypes = [P(GsrfProblem), c_i32, c_f64] + [c_vp] * 8
    L.gsrf_render_stats.argtypes = [P(GsrfProblem), c_vp, c_vp]
    L.gsrf_render_fwd_multi.argtypes = [P(GsrfProblem), c_i32, c_f64, c_vp, c_vp, c_vp]
    L.gsrf_set_kernel_events.argtypes = [c_vp, c_vp, c_vp, c_vp]
    L.gsrf_loss_workspace_size.argtypes = [c_i32, c_i32, c_i32, P(c_sz)]
    L.gsrf_loss_spectrum.argtypes = [c_vp, c_vp, c_i32, c_i32, c_i32, c_f32, c_f32, c_f32, c_vp, c_vp, c_vp, c_vp]
    L.gsrf_loss_spectrum_noalloc.argtypes = [c_vp, c_vp, c_i32, c_i32, c_i32, c_f32, c_f32, c_f32, c_vp, c_vp, c_vp]
    L.gsrf_loss_single.argtypes = [c_vp, c_vp, c_i32, c_i32, c_vp, c_vp, c_vp]
    L.gsrf_sgd_step.argtypes = [c_i64, c_i32] + [c_vp] * 10 + [P(GsrfSgdLr), c_i64, c_vp]
    L.gsrf_grad_stats_accumulate.argtypes = [c_i64, c_vp, c_vp, c_vp, c_vp]
    L.gsrf_density_workspace_size.argtypes = [c_i64, P(c_sz)]
    L.gsrf_density_control.argtypes = ([c_i64, c_i32] + [c_vp] * 8 + [P(GsrfDensityParams), c_i64] + [c_vp] * 10)
    for n in EXPORTS[2:]:
        getattr(L, n).restype = c_i32
    _lib = L
    return L


class GsrfError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        self.status = status
        super().__init__(f"{where}: {L.gsrf_status_str(status).decode()}: {L.gsrf_last_error().decode()}")


def check(status: int, where: str) -> int:
    if status != GSRF_OK:
        raise GsrfError(status, where)
    return status
