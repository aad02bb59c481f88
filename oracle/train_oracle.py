"""FP64 CPU oracle for the steps either side of the render in a training
iteration of GSRF (arXiv 2502.01826): the losses and the attribute update.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP path.

It is the plain definition: the SSIM statistics are 2D convolutions with the
window, the Fourier term is a literal 2D FFT of both spectra, and every
gradient is autograd of the loss as written.  Library primitives used as
steps: conv2d, fft2, exp/log and autograd.

Paper passages followed:
  * antenna-array loss (1 - l1 - l2) L1 + l1 L_SSIM + l2 L_Fourier,
    L1 = mean |S_hat - S|, L_Fourier = (1/(N_az N_el)) sum |F(S_hat) - F(S)|^2
                                                  -- Sec. 3.4 (loss function)
  * single antenna: S_hat = sum_uv S_hat_uv, L = |S_hat - S| for a power,
    |S_hat - S|^2 for a complex signal            -- Sec. 3.4 (single antenna)
  * SGD per attribute w <- w - eta_w grad_w, learning-rate table, mean
    learning rate decaying exponentially 1.6e-4 -> 1.6e-6 over 30000
    iterations                                    -- App. (Gaussian primitive
                                                     optimization, attribute
                                                     updating); App. (training)

Readings taken where the paper is silent:
  L1  the spatial spectrum of a pair is the power of its rays, an [n_el, n_az]
      image c |S_uv|^2 with a fixed normalisation constant c > 0 (measured
      spectra are compared as normalised images); the target is a spectrum of
      the same shape.
  L2  SSIM as in the 3D Gaussian splatting method the paper builds on: an
      11 x 11 Gaussian window of sigma 1.5 (normalised), zero padding outside
      the image, C1 = 0.01^2, C2 = 0.03^2, the map averaged over all pixels;
      L_SSIM = 1 - mean SSIM.
  L3  F is the unnormalised 2D DFT (sum over all pixels, no 1/N).
  L4  single antenna, power case: the received power is the RSSI in dBm,
      10 log10 |S_hat|^2, against a measured RSSI in dBm.
  L5  the mean's learning rate is log-linear in the iteration j from 1.6e-4
      at j = 0 to 1.6e-6 at j = 30000 and held afterwards; learning rates are
      rounded to FP32, the parameters' type, and the update is
      w - eta * g rounded once to FP32.
  L6  the derivative of |x| at x = 0 is 0.
  The weights l1, l2 are not given in the paper; they are arguments.
  D1  the mean gradient of a Gaussian over a densification window is the
      FP32 running sum of its dL/dmu, one FP32 add per component and
      iteration, divided by the number of iterations in which that gradient
      was not zero (the Gaussian was hit); it is selected when the norm of
      that average exceeds eps_mu (decided in FP64 from the FP32 sum).
  D2  the radius is the mean of the diagonal of Sigma = R S S^T R^T; a
      selected Gaussian is large when the radius exceeds eps_r.
  D3  clone: the original stays and its copy's mean moves one step of
      size `clone_step` against the average gradient, mu - step * g_avg
      ("in the direction of the gradient" read as the descent direction).
  D4  split: the original is replaced by two Gaussians whose log-scales are
      reduced by ln(phi) (one FP32 subtraction) and whose means are draws
      mu + R diag(s) z from the original pdf, z ~ N(0, I) passed in; every
      other attribute is copied.
  D5  prune: a Gaussian whose attenuation rho = sigmoid(logit) is below
      eps_rho is removed; pruning follows densification and applies to the
      new Gaussians too.
  D6  output order: the survivors of Gaussian i come before those of i + 1;
      a clone's original precedes its copy, a split's first child its
      second; the gradient statistics restart at zero.

  * adaptive density control: every N_mu iterations Gaussians whose mean
    gradient exceeds eps_mu are cloned (radius <= eps_r) or split in two
    (scales divided by phi, means drawn from the pdf); every N_rho iterations
    Gaussians with attenuation below eps_rho are removed; eps_mu = 0.0002,
    eps_r = 10, eps_rho = 0.004, phi = 1.6      -- App. (number of Gaussian
                                                   updating), App. (training,
                                                   parameter table)

Parity pinning: tests/test_oracle_train.py pins SSIM against a pure-Python
windowed-statistics loop and closed forms, the Fourier term against a literal
double-sum DFT, every gradient against FP64 central differences, the
learning-rate schedule at its end points, and density control against
hand-built cases (each action, ordering, thresholds from both sides) and the
sample covariance of split draws.
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64
SSIM_SIZE = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2

# App. (training): per-attribute learning rates
LR_MEAN_INIT = 1.6e-4
LR_MEAN_FINAL = 1.6e-6
LR_MEAN_STEPS = 30_000
LR_LOG_SCALE = 0.01     # scaling matrix
LR_QUAT = 0.005         # rotation
LR_LOGIT = 0.01         # attenuation
LR_COEFF = 0.0025       # emission (FLE coefficients)


def ssim_window() -> torch.Tensor:
    """11 x 11 Gaussian window, sigma 1.5, summing to 1 (reading L2)."""
    r = torch.arange(SSIM_SIZE, dtype=F64) - (SSIM_SIZE // 2)
    g = torch.exp(-(r * r) / (2.0 * SSIM_SIGMA ** 2))
    g = g / g.sum()
    return torch.outer(g, g)


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Per-pixel SSIM of two [H, W] images (zero padding, reading L2)."""
    w = ssim_window()[None, None]
    pad = SSIM_SIZE // 2

    def blur(z):
        return torch.nn.functional.conv2d(z[None, None], w, padding=pad)[0, 0]

    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def fourier_term(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """(1/(N_az N_el)) sum over frequency pairs of |F(x) - F(y)|^2 (Sec. 3.4, reading L3)."""
    d = torch.fft.fft2(x) - torch.fft.fft2(y)
    return (d.real ** 2 + d.imag ** 2).sum() / x.numel()


def spectrum_loss_terms(signal: np.ndarray, target: np.ndarray, lam1: float, lam2: float, *, power_scale: float = 1.0,
                        grad: bool = True):
    """Antenna-array loss of one pair (Sec. 3.4).

    signal  [n_el, n_az] complex (the rendered rays S_uv)
    target  [n_el, n_az] real    (the measured spectrum)
    power_scale  c of reading L1: the predicted spectrum is c |S_uv|^2
    Returns dict(total, l1, ssim_loss, fourier) and, with grad, G = dL/dRe S +
    j dL/dIm S as complex [n_el, n_az].
    """
    re = torch.tensor(np.real(signal), dtype=F64, requires_grad=grad)
    im = torch.tensor(np.imag(signal), dtype=F64, requires_grad=grad)
    t = torch.tensor(target, dtype=F64)
    p = power_scale * (re * re + im * im)                  # reading L1: power spectrum
    l1 = (p - t).abs().mean()
    ls = 1.0 - ssim_map(p, t).mean()
    lf = fourier_term(p, t)
    total = (1.0 - lam1 - lam2) * l1 + lam1 * ls + lam2 * lf
    out = dict(total=total.item(), l1=l1.item(), ssim_loss=ls.item(), fourier=lf.item())
    if grad:
        gr, gi = torch.autograd.grad(total, (re, im))
        out["G"] = gr.numpy() + 1j * gi.numpy()
    return out


def single_loss_terms(s_hat: complex, target, kind: str, *, grad: bool = True):
    """Single-antenna loss of one pair (Sec. 3.4).

    kind "rssi":    |10 log10 |S_hat|^2 - target| with target in dBm (reading L4)
    kind "complex": |S_hat - target|^2 with a complex target
    Returns dict(loss) and, with grad, G = dL/dRe S_hat + j dL/dIm S_hat.
    """
    re = torch.tensor(float(np.real(s_hat)), dtype=F64, requires_grad=grad)
    im = torch.tensor(float(np.imag(s_hat)), dtype=F64, requires_grad=grad)
    if kind == "rssi":
        loss = (10.0 * torch.log10(re * re + im * im) - float(target)).abs()
    elif kind == "complex":
        loss = (re - float(np.real(target))) ** 2 + (im - float(np.imag(target))) ** 2
    else:
        raise ValueError(kind)
    out = dict(loss=loss.item())
    if grad:
        gr, gi = torch.autograd.grad(loss, (re, im))
        out["G"] = complex(float(gr), float(gi))
    return out


def mean_lr(iteration: int, init: float = LR_MEAN_INIT, final: float = LR_MEAN_FINAL,
            steps: int = LR_MEAN_STEPS) -> float:
    """The mean's learning rate at iteration j (App. training; reading L5), FP64."""
    t = min(max(iteration / steps, 0.0), 1.0) if steps > 0 else 1.0
    return math.exp((1.0 - t) * math.log(init) + t * math.log(final))


def sgd_step(params: dict, grads: dict, iteration: int, lrs: dict | None = None) -> dict:
    """w <- w - eta_w grad_w for every attribute (App. attribute updating, eq. updating).

    params/grads: FP32 arrays keyed means, log_scales, quats, logits, coeffs.
    The difference is formed exactly in FP64 from the FP32 operands and rounded
    once to FP32 (reading L5).
    """
    lrs = dict(lrs or {})
    eta = dict(means=mean_lr(iteration, lrs.get("mean_init", LR_MEAN_INIT), lrs.get("mean_final", LR_MEAN_FINAL),
                             lrs.get("mean_steps", LR_MEAN_STEPS)),
               log_scales=lrs.get("log_scale", LR_LOG_SCALE), quats=lrs.get("quat", LR_QUAT),
               logits=lrs.get("logit", LR_LOGIT), coeffs=lrs.get("coeff", LR_COEFF))
    out = {}
    for k, w in params.items():
        e32 = np.float64(np.float32(eta[k]))
        # the FP32 x FP32 product is exact in FP64 (48 significant bits) and so
        # is its difference with w unless their exponents lie more than 29
        # apart; then the FP64 rounding precedes the FP32 one, which differs
        # from a single rounding only at exact FP32 ties
        out[k] = (np.asarray(w, np.float64) - e32 * np.asarray(grads[k], np.float64)).astype(np.float32)
    return out


# --------------------------------------------------------------------------
# Adaptive density control (App. number of Gaussian updating; parameter table)
# --------------------------------------------------------------------------

EPS_MU = 0.0002
EPS_R = 10.0
EPS_RHO = 0.004
PHI = 1.6


def accumulate_grad_stats(acc: np.ndarray, cnt: np.ndarray, d_means: np.ndarray):
    """One iteration of the window (reading D1): acc += dL/dmu in FP32, cnt += 1
    where the gradient is not zero.  Returns new (acc, cnt)."""
    g = np.asarray(d_means, np.float32)
    acc = (np.asarray(acc, np.float32) + g).astype(np.float32)      # one IEEE FP32 add per component
    cnt = np.asarray(cnt, np.int32) + np.any(g != 0, axis=1).astype(np.int32)
    return acc, cnt


def density_control(params: dict, acc: np.ndarray, cnt: np.ndarray, z: np.ndarray, *, clone_step: float,
                    eps_mu: float = EPS_MU, eps_r: float = EPS_R, eps_rho: float = EPS_RHO, phi: float = PHI,
                    densify: bool = True, prune: bool = True):
    """Clone / split / prune (readings D1-D6).

    params: FP32 arrays keyed means [G,3], log_scales [G,3], quats [G,4],
    logits [G], coeffs [G,K,2]; acc [G,3] FP32 and cnt [G] the window's
    statistics; z [G,2,3] FP32 standard normal draws for the split children.
    Returns (new params, dict(clones, splits, pruned)): clones and splits count
    selected Gaussians that survive pruning, pruned the removed originals.
    """
    from .gsrf_oracle import rotation_matrix
    G = params["means"].shape[0]
    mu = params["means"].astype(np.float64)
    ls = params["log_scales"].astype(np.float64)
    q = torch.tensor(params["quats"], dtype=F64)
    R = rotation_matrix(q).numpy() if G else np.zeros((0, 3, 3))
    s = np.exp(ls)
    Sigma = R @ (s[:, :, None] ** 2 * np.transpose(R, (0, 2, 1)))   # R S S^T R^T
    radius = np.trace(Sigma, axis1=1, axis2=2) / 3.0
    a64 = np.asarray(acc, np.float32).astype(np.float64)
    n = np.asarray(cnt, np.int64)
    sel = densify & (n > 0) & ((a64 * a64).sum(1) > (eps_mu * n.astype(np.float64)) ** 2)
    big = radius > eps_r
    rho = 1.0 / (1.0 + np.exp(-params["logits"].astype(np.float64)))
    gone = prune & (rho < eps_rho)
    out = {k: [] for k in params}
    stats = dict(clones=0, splits=0, pruned=0)
    ln_phi = np.float32(math.log(phi))
    for i in range(G):
        if sel[i] and not big[i]:
            kids = [("keep", None), ("clone", None)]
        elif sel[i]:
            kids = [("split", 0), ("split", 1)]
        else:
            kids = [("keep", None)]
        if gone[i]:
            stats["pruned"] += 1
            continue
        if sel[i]:
            stats["splits" if big[i] else "clones"] += 1
        for kind, c in kids:
            m = params["means"][i]
            l = params["log_scales"][i]
            if kind == "clone":
                m = (mu[i] - clone_step * (a64[i] / n[i])).astype(np.float32)
            elif kind == "split":
                m = (mu[i] + R[i] @ (s[i] * z[i, c].astype(np.float64))).astype(np.float32)
                l = (params["log_scales"][i] - ln_phi).astype(np.float32)     # FP32 subtraction
            out["means"].append(np.asarray(m, np.float32))
            out["log_scales"].append(np.asarray(l, np.float32))
            out["quats"].append(params["quats"][i])
            out["logits"].append(params["logits"][i])
            out["coeffs"].append(params["coeffs"][i])
    K = params["coeffs"].shape[1]
    shapes = dict(means=(0, 3), log_scales=(0, 3), quats=(0, 4), logits=(0,), coeffs=(0, K, 2))
    res = {k: (np.stack(v).astype(np.float32) if v else np.zeros(shapes[k], np.float32)) for k, v in out.items()}
    return res, stats
