"""Binding of the training steps either side of the render (argument
marshalling only; the work runs in libgsrf.so):

* ``SpectrumLoss`` -- antenna-array loss (1 - l1 - l2) L1 + l1 L_SSIM +
  l2 L_Fourier of each pair's power spectrum c |S_uv|^2 and its gradient with
  respect to the rays (Sec. 3.4, loss function);
* ``loss_spectrum_noalloc`` -- the same loss without a workspace (fixed
  per-GPU scratch in the library, for callers that cannot allocate);
* ``loss_single`` -- single-antenna losses on S_hat (RSSI in dBm, or complex
  squared error; Sec. 3.4);
* ``sgd_step`` -- the per-attribute SGD update with the decaying mean
  learning rate (App. Gaussian primitive optimization; App. training);
* ``GradStats`` / ``density_control`` -- the mean-gradient statistics of a
  window of iterations and the clone / split / prune pass (App. number of
  Gaussian updating).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import GsrfDensityParams, GsrfSgdLr, check
from .render import FIELDS, _stream_handle

RSSI_DB, COMPLEX_L2 = _lib.GSRF_LOSS_RSSI_DB, _lib.GSRF_LOSS_COMPLEX_L2


def _ptr(t):
    return None if t is None else t.data_ptr()


def _f32(t, shape, name):
    assert t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == tuple(shape), \
        f"{name}: need a contiguous float32 tensor of shape {tuple(shape)}, got {t.dtype} {tuple(t.shape)}"


class SpectrumLoss:
    """Loss of [P, n_el, n_az] spectra x = power_scale |S|^2; owns the small
    workspace of partial sums."""

    def __init__(self, n_pairs: int, n_el: int, n_az: int, lambda1: float, lambda2: float, power_scale: float = 1.0,
                 device=None):
        self.P, self.n_el, self.n_az = int(n_pairs), int(n_el), int(n_az)
        self.lambda1, self.lambda2, self.power_scale = float(lambda1), float(lambda2), float(power_scale)
        self.device = torch.device(device or "cuda")
        nb = ctypes.c_size_t(0)
        check(_lib.lib().gsrf_loss_workspace_size(self.P, self.n_el, self.n_az, ctypes.byref(nb)),
              "gsrf_loss_workspace_size")
        self.ws = torch.empty(max(int(nb.value), 8), dtype=torch.uint8, device=self.device)

    def __call__(self, signal, target, loss=None, grad_signal=None, want_grad: bool = True, stream=None):
        """signal [P, n_el, n_az, 2], target [P, n_el, n_az] -> (loss [P, 4], grad_signal or None).
        loss[k] = (L, L1, L_SSIM, L_Fourier); grad_signal = dL_k/dRe S + j dL_k/dIm S."""
        P, ne, na = self.P, self.n_el, self.n_az
        _f32(signal, (P, ne, na, 2), "signal")
        _f32(target, (P, ne, na), "target")
        if loss is None:
            loss = torch.empty((P, 4), dtype=torch.float32, device=self.device)
        if want_grad and grad_signal is None:
            grad_signal = torch.empty_like(signal)
        g = _ptr(grad_signal) if want_grad else None
        check(_lib.lib().gsrf_loss_spectrum(signal.data_ptr(), target.data_ptr(), P, ne, na, self.power_scale,
                                            self.lambda1, self.lambda2, loss.data_ptr(), g, self.ws.data_ptr(),
                                            _stream_handle(stream)), "gsrf_loss_spectrum")
        return loss, (grad_signal if want_grad else None)


def loss_spectrum_noalloc(signal, target, lambda1: float, lambda2: float, power_scale: float = 1.0, loss=None,
                          grad_signal=None, want_grad: bool = True, stream=None):
    """The loss of ``SpectrumLoss`` through gsrf_loss_spectrum_noalloc: no
    workspace, the partial sums in the library's fixed per-GPU scratch (calls
    on one GPU must not overlap).  signal [P, n_el, n_az, 2], target
    [P, n_el, n_az] -> (loss [P, 4], grad_signal or None); pass loss and
    grad_signal to allocate nothing here either."""
    P, ne, na = signal.shape[0], signal.shape[1], signal.shape[2]
    _f32(signal, (P, ne, na, 2), "signal")
    _f32(target, (P, ne, na), "target")
    if loss is None:
        loss = torch.empty((P, 4), dtype=torch.float32, device=signal.device)
    if want_grad and grad_signal is None:
        grad_signal = torch.empty_like(signal)
    check(_lib.lib().gsrf_loss_spectrum_noalloc(signal.data_ptr(), target.data_ptr(), P, ne, na, float(power_scale),
                                                float(lambda1), float(lambda2), loss.data_ptr(),
                                                _ptr(grad_signal) if want_grad else None, _stream_handle(stream)),
          "gsrf_loss_spectrum_noalloc")
    return loss, (grad_signal if want_grad else None)


def loss_single(signal_sum, target, kind: int, loss=None, grad_sum=None, want_grad: bool = True, stream=None):
    """signal_sum [P, 2]; target [P] (RSSI_DB, dBm) or [P, 2] (COMPLEX_L2) -> (loss [P], grad_sum [P, 2])."""
    P = signal_sum.shape[0]
    _f32(signal_sum, (P, 2), "signal_sum")
    _f32(target, (P,) if kind == RSSI_DB else (P, 2), "target")
    if loss is None:
        loss = torch.empty((P,), dtype=torch.float32, device=signal_sum.device)
    if want_grad and grad_sum is None:
        grad_sum = torch.empty_like(signal_sum)
    check(_lib.lib().gsrf_loss_single(signal_sum.data_ptr(), target.data_ptr(), P, int(kind), loss.data_ptr(),
                                      _ptr(grad_sum) if want_grad else None, _stream_handle(stream)),
          "gsrf_loss_single")
    return loss, (grad_sum if want_grad else None)


@dataclass
class LearningRates:
    """App. training: mean 1.6e-4 -> 1.6e-6 over 30000 iterations (exponential),
    scaling 0.01, rotation 0.005, attenuation 0.01, emission 0.0025."""
    mean_init: float = 1.6e-4
    mean_final: float = 1.6e-6
    mean_steps: int = 30_000
    log_scale: float = 0.01
    quat: float = 0.005
    logit: float = 0.01
    coeff: float = 0.0025

    def c(self) -> GsrfSgdLr:
        return GsrfSgdLr(self.mean_init, self.mean_final, int(self.mean_steps), self.log_scale, self.quat,
                         self.logit, self.coeff)


def sgd_step(params, grads, iteration: int, fle_L: int, lr: LearningRates | None = None, stream=None):
    """In-place SGD on (means, log_scales, quats, logits, coeffs) -- dicts keyed
    by FIELDS or 5-tuples in that order -- with gradients in the same layouts."""
    p = [params[k] for k in FIELDS] if isinstance(params, dict) else list(params)
    g = [grads[k] for k in FIELDS] if isinstance(grads, dict) else list(grads)
    G = p[0].shape[0]
    K = (fle_L + 1) ** 2
    for t, shape, name in zip(p + g, [(G, 3), (G, 3), (G, 4), (G,), (G, K, 2)] * 2, [*FIELDS, *FIELDS]):
        _f32(t, shape, name)
    lr = lr or LearningRates()
    c = lr.c()
    check(_lib.lib().gsrf_sgd_step(G, int(fle_L), *(t.data_ptr() for t in p), *(t.data_ptr() for t in g),
                                   ctypes.byref(c), int(iteration), _stream_handle(stream)), "gsrf_sgd_step")


class GradStats:
    """Per-Gaussian running sum of dL/dmu and the number of iterations with a
    nonzero one, over a densification window."""

    def __init__(self, n_gauss: int, device=None, acc=None, count=None):
        dev = torch.device(device or "cuda")
        self.acc = acc if acc is not None else torch.zeros((n_gauss, 3), dtype=torch.float32, device=dev)
        self.count = count if count is not None else torch.zeros((n_gauss,), dtype=torch.int32, device=dev)

    def accumulate(self, d_means, stream=None):
        G = self.acc.shape[0]
        _f32(d_means, (G, 3), "d_means")
        check(_lib.lib().gsrf_grad_stats_accumulate(G, d_means.data_ptr(), self.acc.data_ptr(), self.count.data_ptr(),
                                                    _stream_handle(stream)), "gsrf_grad_stats_accumulate")


@dataclass
class DensityParams:
    """App. parameter table: eps_mu = 0.0002, eps_r = 10, eps_rho = 0.004, phi = 1.6."""
    eps_mu: float = 0.0002
    eps_r: float = 10.0
    eps_rho: float = 0.004
    phi: float = 1.6
    clone_step: float = 1.6e-4
    densify: bool = True
    prune: bool = True

    def c(self) -> GsrfDensityParams:
        return GsrfDensityParams(self.eps_mu, self.eps_r, self.eps_rho, self.phi, self.clone_step, int(self.densify),
                                 int(self.prune))


def density_control(params, stats: GradStats, z_draws, fle_L: int, dp: DensityParams | None = None, stream=None,
                    read_counts: bool = True):
    """Clone / split / prune.  params: 5-tuple or dict (FIELDS order);
    z_draws [G, 2, 3] standard normal (None when not densifying).  Returns
    (new params tuple, new GradStats, dict(n, clones, splits, pruned)); reads
    the new count back (one host synchronisation).  With read_counts=False it
    returns the capacity-sized outputs and the device counts tensor instead,
    without synchronising."""
    dp = dp or DensityParams()
    p = [params[k] for k in FIELDS] if isinstance(params, dict) else list(params)
    G = p[0].shape[0]
    K = (fle_L + 1) ** 2
    for t, shape, name in zip(p, [(G, 3), (G, 3), (G, 4), (G,), (G, K, 2)], FIELDS):
        _f32(t, shape, name)
    if dp.densify:
        _f32(z_draws, (G, 2, 3), "z_draws")
    dev = p[0].device
    cap = 2 * G if dp.densify else G
    e = lambda *s_: torch.empty(s_, dtype=torch.float32, device=dev)
    out = [e(cap, 3), e(cap, 3), e(cap, 4), e(cap), e(cap, K, 2)]
    o_acc = e(cap, 3)
    o_cnt = torch.empty((cap,), dtype=torch.int32, device=dev)
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    nb = ctypes.c_size_t(0)
    check(_lib.lib().gsrf_density_workspace_size(G, ctypes.byref(nb)), "gsrf_density_workspace_size")
    ws = torch.empty(max(int(nb.value), 8), dtype=torch.uint8, device=dev)
    c = dp.c()
    check(_lib.lib().gsrf_density_control(G, int(fle_L), *(t.data_ptr() for t in p), stats.acc.data_ptr(),
                                          stats.count.data_ptr(), _ptr(z_draws) if dp.densify else None,
                                          ctypes.byref(c), cap, *(t.data_ptr() for t in out), o_acc.data_ptr(),
                                          o_cnt.data_ptr(), counts.data_ptr(), ws.data_ptr(), _stream_handle(stream)),
          "gsrf_density_control")
    if not read_counts:
        return tuple(out), (o_acc, o_cnt), counts
    n, clones, splits, pruned = (int(v) for v in counts.cpu())
    new = tuple(t[:n] for t in out)
    return new, GradStats(n, dev, o_acc[:n], o_cnt[:n]), dict(n=n, clones=clones, splits=splits, pruned=pruned)
