"""Python API over libgsrf.so: device-resident problems, eager renders and a
``torch.autograd.Function``.

PyTorch supplies device memory and the stream; every step of the hot path
(activation, splatting, binning, radix sort, compositing, RSSI, adjoint and
chain rule) runs in the HIP kernels of libgsrf.so.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import GsrfGrid, GsrfLayout, GsrfProblem, check

FIELDS = ("means", "log_scales", "quats", "logits", "coeffs")


def multi_chunks(n_freq: int) -> list:
    """Carriers per traversal of gsrf_render_fwd_multi: 32 while more than 16
    remain, then 16 (the last chunk may be partly unused)."""
    out, left = [], n_freq
    while left > 0:
        c = 32 if left > 16 else 16
        out.append(c)
        left -= c
    return out


@dataclass
class GridSpec:
    """Receiver ray grid and render constants (mirrors ``gsrf_grid``)."""

    n_az: int = 360
    n_el: int = 90
    el_lo: float = 0.0
    el_hi: float = math.pi / 2
    fle_L: int = 2
    r_rx: float = 1.0
    t_min: float = 1.0e-4
    alpha_max: float = 0.99
    tile_w: int = 16
    tile_h: int = 16
    lanes_per_ray: int = 0
    footprint: int = 0
    depth_order: int = 0        # 1: per-ray chord-midpoint order (App. A.3)
    fle_eval: int = 0           # 1: radiance at each Gaussian's direction
    transmittance: int = 0      # 1: chord transmittance exp(-alpha dt) (App. A.2)

    @staticmethod
    def of(g) -> "GridSpec":
        return GridSpec(**{k: getattr(g, k, GridSpec.__dataclass_fields__[k].default)
                           for k in GridSpec.__dataclass_fields__})

    def c(self) -> GsrfGrid:
        return GsrfGrid(self.n_az, self.n_el, self.el_lo, self.el_hi, self.fle_L, self.r_rx, self.t_min,
                        self.alpha_max, self.tile_w, self.tile_h, self.lanes_per_ray, self.footprint,
                        self.depth_order, self.fle_eval, self.transmittance)

    @property
    def K(self) -> int:
        return (self.fle_L + 1) ** 2


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def pack_pairs(pairs) -> np.ndarray:
    """Pack (rx, tx, freq_hz, scene) records into the 40-byte ``gsrf_pair`` layout."""
    dt = np.dtype([("rx", "<f4", 3), ("tx", "<f4", 3), ("freq_hz", "<f8"), ("scene", "<i4"), ("reserved", "<i4")])
    assert dt.itemsize == 40
    a = np.zeros(len(pairs), dtype=dt)
    for i, p in enumerate(pairs):
        a[i]["rx"] = np.asarray(p.rx, np.float32)
        a[i]["tx"] = np.asarray(p.tx, np.float32)
        a[i]["freq_hz"] = float(p.freq_hz)
        a[i]["scene"] = int(getattr(p, "scene", 0))
    return a


class Problem:
    """A batch of scenes and TX/RX pairs resident on one GPU, plus its workspace.

    Parameters are FP32 device tensors (``set_params``); all scenes are
    concatenated with CSR ``scene_offsets``.  ``splat_capacity`` fixes the
    sort buffers; when None the first render sizes them from the measured
    splat count (one host synchronisation), and later renders grow them if a
    count ever exceeds the capacity.
    """

    def __init__(self, params: dict, pairs, grid, scene_offsets=None, splat_capacity=None, device="cuda",
                 hit_capacity=None):
        self.device = torch.device(device)
        self.grid = GridSpec.of(grid)
        self.set_params(**params)
        G = self.n_gauss
        offs = np.asarray([0, G] if scene_offsets is None else scene_offsets, dtype=np.int64)
        self.scene_offsets_host = np.ascontiguousarray(offs)
        self.scene_offsets_dev = torch.from_numpy(self.scene_offsets_host).to(self.device)
        packed = pack_pairs(pairs)
        self.n_pairs = len(pairs)
        self.pair_scene_host = np.ascontiguousarray(packed["scene"].astype(np.int32))
        self.pairs_dev = torch.from_numpy(packed.view(np.uint8).copy()).to(self.device)
        self.pairs = list(pairs)
        self.auto_capacity = splat_capacity is None
        self.cap = int(splat_capacity or 0)
        # per-ray midpoint order: (ray, Gaussian) hit records, sized by the first render
        self.auto_hit_capacity = hit_capacity is None
        self.hit_cap = int(hit_capacity or 0)
        self.ws = None
        self._alloc()

    # ---------------------------------------------------------------- setup --
    def set_params(self, means, log_scales, quats, logits, coeffs):
        t = lambda x: (x if isinstance(x, torch.Tensor) else torch.from_numpy(np.asarray(x))).to(
            self.device, torch.float32).contiguous()
        self.means, self.log_scales, self.quats = t(means), t(log_scales), t(quats)
        self.logits, self.coeffs = t(logits), t(coeffs)
        self.n_gauss = int(self.means.shape[0])
        assert self.coeffs.shape[1:] == (self.grid.K, 2), "coeffs must be [G, (L+1)^2, 2]"

    def _problem(self) -> GsrfProblem:
        p = GsrfProblem()
        p.means, p.log_scales, p.quats = self.means.data_ptr(), self.log_scales.data_ptr(), self.quats.data_ptr()
        p.opacity_logits, p.coeffs = self.logits.data_ptr(), self.coeffs.data_ptr()
        p.n_gauss = self.n_gauss
        p.n_scenes = len(self.scene_offsets_host) - 1
        p.scene_offsets = self.scene_offsets_host.ctypes.data
        p.scene_offsets_dev = self.scene_offsets_dev.data_ptr()
        p.pairs = self.pairs_dev.data_ptr() if self.n_pairs else None
        p.pair_scene = self.pair_scene_host.ctypes.data
        p.n_pairs = self.n_pairs
        p.grid = self.grid.c()
        p.splat_capacity = self.cap
        p.workspace = self.ws.data_ptr() if self.ws is not None else None
        p.workspace_bytes = self.ws.numel() if self.ws is not None else 0
        p.hit_capacity = self.hit_cap
        return p

    def workspace_bytes(self, cap=None) -> int:
        p = self._problem()
        if cap is not None:
            p.splat_capacity = int(cap)
        n = ctypes.c_size_t()
        check(_lib.lib().gsrf_workspace_size(ctypes.byref(p), ctypes.byref(n)), "gsrf_workspace_size")
        return int(n.value)

    def _alloc(self):
        nbytes = max(self.workspace_bytes(self.cap), 256)
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = None
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        assert self.ws.data_ptr() % 256 == 0

    def layout(self) -> GsrfLayout:
        lay = GsrfLayout()
        check(_lib.lib().gsrf_layout_of(ctypes.byref(self._problem()), ctypes.byref(lay)), "gsrf_layout_of")
        return lay

    def view(self, offset: int, dtype, count: int) -> torch.Tensor:
        """A typed view into the workspace (tests and tools)."""
        itemsize = torch.empty(0, dtype=dtype).element_size()
        return self.ws[offset:offset + count * itemsize].view(dtype)

    # ---------------------------------------------------------------- steps --
    def project(self, stream=None):
        check(_lib.lib().gsrf_project(ctypes.byref(self._problem()), _stream_handle(stream)), "gsrf_project")

    def splat_count(self, stream=None) -> tuple[int, bool]:
        n = ctypes.c_int64()
        st = _lib.lib().gsrf_splat_count(ctypes.byref(self._problem()), ctypes.byref(n), _stream_handle(stream))
        if st not in (_lib.GSRF_OK, _lib.GSRF_ECAPACITY):
            check(st, "gsrf_splat_count")
        return int(n.value), st == _lib.GSRF_OK

    def bin_sort(self, stream=None):
        check(_lib.lib().gsrf_bin_sort(ctypes.byref(self._problem()), _stream_handle(stream)), "gsrf_bin_sort")

    def render_fwd(self, signal=None, signal_sum=None, rssi=None, stream=None):
        g = self.grid
        P = self.n_pairs
        if signal is None:
            signal = torch.empty((P, g.n_el, g.n_az, 2), dtype=torch.float32, device=self.device)
        if signal_sum is None:
            signal_sum = torch.empty((P, 2), dtype=torch.float32, device=self.device)
        if rssi is None:
            rssi = torch.empty((P,), dtype=torch.float32, device=self.device)
        check(_lib.lib().gsrf_render_fwd(ctypes.byref(self._problem()), signal.data_ptr(), signal_sum.data_ptr(),
                                         rssi.data_ptr(), _stream_handle(stream)), "gsrf_render_fwd")
        return signal, signal_sum, rssi

    def render_fwd_multi(self, n_freq: int, freq_step_hz: float, signal=None, signal_sum=None, stream=None):
        """Forward for n_freq carriers per pair (carrier c at pair frequency + c * freq_step_hz):
        signal [P, n_freq, n_el, n_az, 2], signal_sum [P, n_freq, 2]."""
        g, P = self.grid, self.n_pairs
        if signal is None:
            signal = torch.empty((P, n_freq, g.n_el, g.n_az, 2), dtype=torch.float32, device=self.device)
        if signal_sum is None:
            signal_sum = torch.empty((P, n_freq, 2), dtype=torch.float32, device=self.device)
        check(_lib.lib().gsrf_render_fwd_multi(ctypes.byref(self._problem()), int(n_freq), float(freq_step_hz),
                                               signal.data_ptr(), signal_sum.data_ptr(), _stream_handle(stream)),
              "gsrf_render_fwd_multi")
        return signal, signal_sum

    def render_bwd(self, signal, grad_signal, grad_sum=None, out=None, stream=None):
        G, K = self.n_gauss, self.grid.K
        if out is None:
            e = lambda *s: torch.empty(s, dtype=torch.float32, device=self.device)
            out = (e(G, 3), e(G, 3), e(G, 4), e(G), e(G, K, 2))
        assert signal.is_contiguous() and grad_signal.is_contiguous()
        gs = grad_sum.contiguous() if grad_sum is not None else None
        check(_lib.lib().gsrf_render_bwd(ctypes.byref(self._problem()), signal.data_ptr(), grad_signal.data_ptr(),
                                         gs.data_ptr() if gs is not None else None,
                                         *(o.data_ptr() for o in out), _stream_handle(stream)), "gsrf_render_bwd")
        return out

    def render_bwd_multi(self, n_freq: int, freq_step_hz: float, grad_signal, grad_sum=None, out=None, stream=None):
        """Adjoint of render_fwd_multi after render_fwd: grad_signal [P, n_freq, n_el, n_az, 2],
        grad_sum [P, n_freq, 2] or None -> gradients summed over pairs and carriers."""
        G, K = self.n_gauss, self.grid.K
        if out is None:
            e = lambda *s: torch.empty(s, dtype=torch.float32, device=self.device)
            out = (e(G, 3), e(G, 3), e(G, 4), e(G), e(G, K, 2))
        assert grad_signal.is_contiguous() and tuple(grad_signal.shape) == (
            self.n_pairs, int(n_freq), self.grid.n_el, self.grid.n_az, 2)
        gs = grad_sum.contiguous() if grad_sum is not None else None
        check(_lib.lib().gsrf_render_bwd_multi(ctypes.byref(self._problem()), int(n_freq), float(freq_step_hz),
                                               grad_signal.data_ptr(), gs.data_ptr() if gs is not None else None,
                                               *(o.data_ptr() for o in out), _stream_handle(stream)),
              "gsrf_render_bwd_multi")
        return out

    def render_stats(self, stream=None) -> dict:
        """Counts of the forward traversal (instrumentation; run after prepare())."""
        c = torch.zeros(6, dtype=torch.int64, device=self.device)
        check(_lib.lib().gsrf_render_stats(ctypes.byref(self._problem()), c.data_ptr(), _stream_handle(stream)),
              "gsrf_render_stats")
        v = c.cpu().tolist()
        return dict(tests=v[0], hits=v[1], staged=v[2], rays=v[3], tile_tests=v[4], walk_slots=v[5])

    def prepare(self, stream=None):
        """project + bin_sort, growing the splat capacity when it is too small."""
        self.project(stream)
        if self.auto_capacity:
            n, ok = self.splat_count(stream)
            if not ok or self.cap == 0:
                self.cap = max(int(n * 1.25) + 1024, 4096)
                self._alloc()
                self.project(stream)
        self.bin_sort(stream)

    def ray_hit_count(self, stream=None) -> tuple[int, bool]:
        """depth_order = 1: hit records the last render needed, and whether they fit."""
        n = ctypes.c_int64()
        st = _lib.lib().gsrf_ray_hit_count(ctypes.byref(self._problem()), ctypes.byref(n), _stream_handle(stream))
        if st not in (_lib.GSRF_OK, _lib.GSRF_ECAPACITY):
            check(st, "gsrf_ray_hit_count")
        return int(n.value), st == _lib.GSRF_OK

    def forward(self, stream=None):
        self.prepare(stream)
        out = self.render_fwd(stream=stream)
        if self.grid.depth_order and self.auto_hit_capacity:
            n, ok = self.ray_hit_count(stream)
            if not ok:                      # the render wrote zeros: grow the records and render again
                self.hit_cap = max(int(n * 1.25) + 4096, 65536)
                self._alloc()               # a new workspace: project and bin_sort again
                self.prepare(stream)
                out = self.render_fwd(stream=stream)
        return out


class GSRFRender(torch.autograd.Function):
    """signal [P, n_el, n_az, 2], signal_sum [P, 2] = render(params); backward via gsrf_render_bwd.

    Complex values cross the boundary as real (re, im) views, so the adjoint
    receives dL/dRe S + j dL/dIm S and returns real parameter gradients.
    The problem's workspace holds the sorted tile lists between forward and
    backward: do not render the same Problem again before backward runs.
    """

    @staticmethod
    def forward(ctx, prob: Problem, means, log_scales, quats, logits, coeffs):
        prob.set_params(means.detach(), log_scales.detach(), quats.detach(), logits.detach(), coeffs.detach())
        signal, signal_sum, _ = prob.forward()
        ctx.prob = prob
        ctx.save_for_backward(signal)
        return signal, signal_sum

    @staticmethod
    def backward(ctx, g_signal, g_sum):
        (signal,) = ctx.saved_tensors
        prob = ctx.prob
        if g_signal is None:
            g_signal = torch.zeros_like(signal)
        grads = prob.render_bwd(signal, g_signal.contiguous(), None if g_sum is None else g_sum.contiguous())
        return (None, *grads)


def render(params: dict, pairs, grid, scene_offsets=None):
    """One-shot eager render: returns (signal complex64 [P, n_el, n_az], S_hat complex64 [P], rssi_dbm [P])."""
    prob = Problem(params, pairs, grid, scene_offsets)
    sig, ssum, rssi = prob.forward()
    return torch.view_as_complex(sig), torch.view_as_complex(ssum), rssi
