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


def _gauss(n, K=1):
    return dict(means=np.zeros((n, 3), np.float32), log_scales=np.full((n, 3), -2.0, np.float32),
                quats=np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)), logits=np.zeros(n, np.float32),
                coeffs=np.zeros((n, K, 2), np.float32))


def test_grad_stats_accumulate_in_fp32_and_count_hits():
    acc, cnt = np.zeros((3, 3), np.float32), np.zeros(3, np.int32)
    g1 = np.array([[1e8, 0, 0], [0, 0, 0], [1, 2, 3]], np.float32)
    g2 = np.array([[1, 0, 0], [0, 0, 0], [0, 0, -1]], np.float32)
    acc, cnt = to.accumulate_grad_stats(acc, cnt, g1)
    acc, cnt = to.accumulate_grad_stats(acc, cnt, g2)
    assert acc[0, 0] == np.float32(1e8)          # 1e8 + 1 rounds back in FP32
    assert list(cnt) == [2, 0, 2] and np.array_equal(acc[2], np.array([1, 2, 2], np.float32))


def test_density_control_actions_by_hand():
    p = _gauss(6)
    p["means"][:] = np.arange(18, dtype=np.float32).reshape(6, 3)
    p["coeffs"][:, 0, 0] = np.arange(6)
    p["log_scales"][2] = np.log(4.0)              # radius = mean of diag Sigma = 16 > 10: large
    p["logits"][3] = -8.0                         # rho = 3.4e-4 < 0.004: pruned
    p["logits"][5] = -8.0
    eps = 0.0002
    acc = np.zeros((6, 3), np.float32)
    cnt = np.array([0, 2, 4, 1, 2, 3], np.int32)
    acc[1] = [0.004, 0.0, 0.0]                   # average 0.002 > eps: clone
    acc[2] = [0.0, 0.0, -0.008]                  # average 0.002: split (large)
    acc[3] = [1.0, 0.0, 0.0]
    acc[4] = [2 * eps * 0.999, 0.0, 0.0]         # just below the threshold: kept as is
    acc[5] = [1.0, 1.0, 1.0]                     # selected but pruned: nothing survives
    z = np.zeros((6, 2, 3), np.float32)
    z[2, 0] = [1.0, 0.0, 0.0]
    z[2, 1] = [0.0, -0.5, 2.0]
    out, st = to.density_control(p, acc, cnt, z, clone_step=0.5)
    assert st == dict(clones=1, splits=1, pruned=2)
    # order: 0, 1, copy of 1, children of 2, 4
    assert np.array_equal(out["coeffs"][:, 0, 0], np.array([0, 1, 1, 2, 2, 4], np.float32))
    assert np.array_equal(out["means"][0], p["means"][0]) and np.array_equal(out["means"][1], p["means"][1])
    assert np.allclose(out["means"][2], p["means"][1] - 0.5 * np.array([0.002, 0, 0]), rtol=0, atol=1e-6)
    # split with R = I: mu + s * z, log-scale reduced by ln 1.6
    assert np.allclose(out["means"][3], p["means"][2] + 4.0 * np.array([1.0, 0, 0]), atol=1e-6)
    assert np.allclose(out["means"][4], p["means"][2] + 4.0 * np.array([0.0, -0.5, 2.0]), atol=1e-6)
    assert np.allclose(out["log_scales"][3:5], np.log(4.0) - np.log(1.6), atol=1e-6)
    assert np.array_equal(out["log_scales"][2], p["log_scales"][1])
    assert np.array_equal(out["means"][5], p["means"][4])
    # switches: no densification keeps every selected one, no pruning keeps the faint ones
    out2, st2 = to.density_control(p, acc, cnt, z, clone_step=0.5, densify=False)
    assert st2 == dict(clones=0, splits=0, pruned=2) and out2["means"].shape == (4, 3)
    out3, st3 = to.density_control(p, acc, cnt, z, clone_step=0.5, prune=False)
    assert st3 == dict(clones=3, splits=1, pruned=0) and out3["means"].shape == (10, 3)   # 1, 3, 5 cloned


def test_split_rotates_the_draw_and_matches_the_pdf():
    from scipy.spatial.transform import Rotation
    # 90 degrees about z: the body x axis points along world y
    p = _gauss(1)
    p["quats"][0] = [np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)]
    p["log_scales"][0] = np.log([8.0, 1.0, 1.0])
    acc, cnt = np.array([[1.0, 0, 0]], np.float32), np.array([1], np.int32)
    z = np.array([[[1.0, 0, 0], [0, 0, 1.0]]], np.float32)
    out, st = to.density_control(p, acc, cnt, z, clone_step=0.0)
    assert st["splits"] == 1
    assert np.allclose(out["means"][0], [0, 8.0, 0], atol=1e-5) and np.allclose(out["means"][1], [0, 0, 1.0], atol=1e-6)
    # many splits of one random Gaussian: the children's sample covariance is Sigma
    rng = np.random.default_rng(30)
    n = 20000
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    s = np.array([3.0, 2.0, 5.0])
    p = _gauss(n)
    p["quats"][:] = q.astype(np.float32)
    p["log_scales"][:] = np.log(s).astype(np.float32)
    acc = np.ones((n, 3), np.float32)
    cnt = np.ones(n, np.int32)
    z = rng.normal(size=(n, 2, 3)).astype(np.float32)
    out, _ = to.density_control(p, acc, cnt, z, clone_step=0.0)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    sigma = R @ np.diag(np.exp(2 * np.log(s.astype(np.float32).astype(np.float64)))) @ R.T
    emp = np.cov(out["means"].astype(np.float64).T)
    assert np.allclose(emp, sigma, atol=0.05 * np.abs(sigma).max())


def test_radius_threshold_is_rotation_invariant():
    p = _gauss(2)
    p["log_scales"][:] = np.log([np.sqrt(10.5), np.sqrt(10.5), np.sqrt(10.5)]).astype(np.float32)  # radius 10.5
    p["quats"][1] = [0.3, -0.5, 0.7, 0.1]
    acc, cnt = np.ones((2, 3), np.float32), np.ones(2, np.int32)
    z = np.zeros((2, 2, 3), np.float32)
    _, st = to.density_control(p, acc, cnt, z, clone_step=0.0)
    assert st["splits"] == 2
    p["log_scales"][:] = np.log([np.sqrt(9.5)] * 3).astype(np.float32)
    _, st = to.density_control(p, acc, cnt, z, clone_step=0.0)
    assert st["clones"] == 2
