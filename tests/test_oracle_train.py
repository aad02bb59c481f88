"""Pins of the loss and attribute-update oracle (CPU only).

Each pin checks the oracle against something other than itself: a pure-Python
loop over the SSIM windows with explicit zero padding, closed forms of SSIM on
constant images, a literal double-sum DFT, FP64 central differences of every
gradient, the learning-rate schedule's end points (App. training) and exact
rational arithmetic for the update.
"""
from fractions import Fraction
import math

import numpy as np
import pytest
import torch

from oracle import train_oracle as to


def _ssim_loops(x, y):
    """SSIM map by explicit loops over each pixel's 11 x 11 window (zero outside)."""
    H, W = x.shape
    r = np.arange(11) - 5
    g = np.exp(-(r * r) / (2 * 1.5 ** 2))
    g = g / g.sum()
    out = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            sx = sy = sxx = syy = sxy = 0.0
            for a in range(11):
                for b in range(11):
                    ii, jj = i + a - 5, j + b - 5
                    if 0 <= ii < H and 0 <= jj < W:
                        w = g[a] * g[b]
                        xv, yv = x[ii, jj], y[ii, jj]
                        sx += w * xv
                        sy += w * yv
                        sxx += w * xv * xv
                        syy += w * yv * yv
                        sxy += w * xv * yv
            vx, vy, cxy = sxx - sx * sx, syy - sy * sy, sxy - sx * sy
            c1, c2 = 0.01 ** 2, 0.03 ** 2
            out[i, j] = (2 * sx * sy + c1) * (2 * cxy + c2) / ((sx * sx + sy * sy + c1) * (vx + vy + c2))
    return out


def test_ssim_window_is_normalised_gaussian():
    w = to.ssim_window().numpy()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])
    # ratio of neighbouring taps on the axis is exp(-(2k+1)/(2 sigma^2))
    assert math.isclose(w[5, 6] / w[5, 5], math.exp(-1 / 4.5), rel_tol=1e-14)


def test_ssim_map_matches_window_loops():
    rng = np.random.default_rng(3)
    x, y = rng.uniform(0, 1, (7, 13)), rng.uniform(0, 1, (7, 13))
    ref = _ssim_loops(x, y)
    got = to.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13)


def test_ssim_identical_and_constant_images():
    rng = np.random.default_rng(4)
    x = torch.tensor(rng.uniform(0, 1, (20, 30)))
    assert torch.allclose(to.ssim_map(x, x), torch.ones_like(x), atol=1e-14)
    # constant images a, b: away from the border the windows see no padding, the
    # variances and covariance vanish, SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.7, 0.2
    m = to.ssim_map(torch.full((30, 30), a, dtype=torch.float64), torch.full((30, 30), b, dtype=torch.float64))
    want = (2 * a * b + to.SSIM_C1) / (a * a + b * b + to.SSIM_C1)
    assert abs(float(m[15, 15]) - want) < 1e-12
    assert abs(float(m[0, 0]) - want) > 1e-3      # the zero padding reaches the corner


def test_fourier_term_matches_double_sum_dft():
    rng = np.random.default_rng(5)
    x, y = rng.uniform(0, 1, (4, 5)), rng.uniform(0, 1, (4, 5))
    H, W = x.shape
    tot = 0.0
    for fu in range(H):
        for fv in range(W):
            fx = fy = 0j
            for u in range(H):
                for v in range(W):
                    e = np.exp(-2j * np.pi * (fu * u / H + fv * v / W))
                    fx += x[u, v] * e
                    fy += y[u, v] * e
            tot += abs(fx - fy) ** 2
    got = float(to.fourier_term(torch.tensor(x), torch.tensor(y)))
    assert math.isclose(got, tot / (H * W), rel_tol=1e-12)
    # Parseval: with the unnormalised DFT the term equals the sum of squared differences
    assert math.isclose(got, float(((x - y) ** 2).sum()), rel_tol=1e-12)


def _signal(shape, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(0, 0.5, shape) + 1j * rng.normal(0, 0.5, shape))


def test_spectrum_loss_terms_values():
    s = _signal((6, 9), 6)
    t = np.abs(_signal((6, 9), 7)) ** 2
    p = np.abs(s) ** 2
    r = to.spectrum_loss_terms(s, t, 0.2, 0.1, grad=False)
    assert math.isclose(r["l1"], np.abs(p - t).mean(), rel_tol=1e-13)
    assert math.isclose(r["ssim_loss"], 1 - _ssim_loops(p, t).mean(), rel_tol=1e-11)
    assert math.isclose(r["fourier"], ((p - t) ** 2).sum(), rel_tol=1e-12)
    assert math.isclose(r["total"], 0.7 * r["l1"] + 0.2 * r["ssim_loss"] + 0.1 * r["fourier"], rel_tol=1e-13)
    assert to.spectrum_loss_terms(s, p, 0.2, 0.1, grad=False)["total"] < 1e-14


@pytest.mark.parametrize("lam1,lam2", [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (0.2, 0.05)])
def test_spectrum_loss_gradient_vs_central_differences(lam1, lam2):
    s = _signal((5, 8), 8)
    t = np.abs(_signal((5, 8), 9)) ** 2
    G = to.spectrum_loss_terms(s, t, lam1, lam2)["G"]
    h = 1e-6
    rng = np.random.default_rng(10)
    for _ in range(12):
        i, j = rng.integers(0, 5), rng.integers(0, 8)
        for unit, part in ((1.0, "re"), (1j, "im")):
            sp, sm = s.copy(), s.copy()
            sp[i, j] += h * unit
            sm[i, j] -= h * unit
            fd = (to.spectrum_loss_terms(sp, t, lam1, lam2, grad=False)["total"]
                  - to.spectrum_loss_terms(sm, t, lam1, lam2, grad=False)["total"]) / (2 * h)
            an = G[i, j].real if part == "re" else G[i, j].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (i, j, part, fd, an)


def test_single_antenna_losses():
    s, tc = 0.3 - 0.4j, 0.1 + 0.2j
    r = to.single_loss_terms(s, tc, "complex")
    assert math.isclose(r["loss"], abs(s - tc) ** 2, rel_tol=1e-14)
    assert abs(r["G"] - 2 * (s - tc)) < 1e-15                  # closed form 2 (S_hat - S)
    r = to.single_loss_terms(s, -12.0, "rssi")
    p_db = 10 * math.log10(abs(s) ** 2)
    assert math.isclose(r["loss"], abs(p_db + 12.0), rel_tol=1e-14)
    # d/dS of |10 log10 |S|^2 - t| = sign * 20 / ln 10 * S / |S|^2
    want = math.copysign(1.0, p_db + 12.0) * 20 / math.log(10) * s / abs(s) ** 2
    assert abs(r["G"] - want) < 1e-13
    h = 1e-7
    fd = (to.single_loss_terms(s + h, -12.0, "rssi", grad=False)["loss"]
          - to.single_loss_terms(s - h, -12.0, "rssi", grad=False)["loss"]) / (2 * h)
    assert abs(fd - r["G"].real) < 1e-6


def test_mean_learning_rate_schedule():
    assert math.isclose(to.mean_lr(0), 1.6e-4, rel_tol=1e-15)
    assert math.isclose(to.mean_lr(30_000), 1.6e-6, rel_tol=1e-14)
    assert math.isclose(to.mean_lr(15_000), math.sqrt(1.6e-4 * 1.6e-6), rel_tol=1e-14)   # exponential decay
    assert to.mean_lr(90_000) == to.mean_lr(30_000)
    r = [to.mean_lr(j) for j in (0, 1000, 2000)]
    assert math.isclose(r[1] / r[0], r[2] / r[1], rel_tol=1e-12)                        # constant ratio per step


def test_sgd_step_rounds_once():
    rng = np.random.default_rng(11)
    params = {k: rng.normal(0, 1, n).astype(np.float32) for k, n in
              (("means", 12), ("log_scales", 12), ("quats", 16), ("logits", 4), ("coeffs", 72))}
    grads = {k: rng.normal(0, 3, v.shape).astype(np.float32) for k, v in params.items()}
    out = to.sgd_step(params, grads, 1234)
    etas = dict(means=to.mean_lr(1234), log_scales=0.01, quats=0.005, logits=0.01, coeffs=0.0025)
    for k in params:
        e = Fraction(float(np.float32(etas[k])))
        for w, g, o in zip(params[k], grads[k], out[k]):
            exact = Fraction(float(w)) - e * Fraction(float(g))
            # o is the FP32 value nearest to the exact result
            lo, hi = np.nextafter(o, np.float32(-np.inf)), np.nextafter(o, np.float32(np.inf))
            d = abs(Fraction(float(o)) - exact)
            assert d <= abs(Fraction(float(lo)) - exact) and d <= abs(Fraction(float(hi)) - exact)
