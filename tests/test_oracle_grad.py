"""CPU pins of the oracle's gradients (T10): autograd vs FP64 central differences,
and the midpoint identities of App. D.3 (no GPU)."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from synth import Grid, Pair, Scene


def _loss(scene, pair, grid, G):
    r = oracle.render(scene, pair, grid)
    return float((G[:, 0] * r["S"].real + G[:, 1] * r["S"].imag).sum()), r["active_sig"], r["n_active"]


def test_autograd_matches_central_differences():
    b = synth.tiny()
    g = Grid(n_az=24, n_el=6, fle_L=2)
    sc = b.scenes[0].subset(slice(0, 400))
    sc = synth.Scene(*(getattr(sc, f).astype(np.float64) for f in ("means", "log_scales", "quats", "logits", "coeffs")))
    p = b.pairs[0]
    G = synth.cotangent((g.n_el * g.n_az,), seed=3).astype(np.float64)
    grads = oracle.vjp(sc, p, g, G)
    base = oracle.render(sc, p, g)
    # Gaussians that actually contribute
    contrib = set()
    for k in range(0, g.n_el * g.n_az, 5):
        v, u = divmod(k, g.n_az)
        sq = oracle.ray_sequence(sc, p, g, u, v)
        contrib |= set(sq["order"][sq["active"]].tolist())
    contrib = sorted(contrib)
    assert len(contrib) > 20
    rng = np.random.default_rng(11)
    fields = [("means", 3), ("log_scales", 3), ("quats", 4), ("logits", None), ("coeffs", None)]
    checked = 0
    for trial in range(60):
        gi = int(rng.choice(contrib))
        name, width = fields[trial % len(fields)]
        arr = getattr(sc, name)
        idx = (gi,) + tuple(int(rng.integers(0, s)) for s in arr.shape[1:])
        h = 1e-6 * max(1.0, abs(float(arr[idx])))
        vals = []
        sigs = []
        for sgn in (+1, -1):
            a2 = arr.copy()
            a2[idx] += sgn * h
            sc2 = synth.Scene(**{**sc.__dict__, name: a2})
            L, sig, na = _loss(sc2, p, g, G)
            vals.append(L)
            sigs.append((sig, na))
        if not (np.array_equal(sigs[0][0], sigs[1][0]) and np.array_equal(sigs[0][1], sigs[1][1])
                and np.array_equal(sigs[0][0], base["active_sig"])):
            continue            # a discrete decision moved within +-h: FD is not defined there
        fd = (vals[0] - vals[1]) / (2 * h)
        ad = float(grads[name][idx])
        scale = max(abs(fd), 1e-3 * np.abs(grads[name]).max())
        assert abs(ad - fd) <= 2e-5 * scale + 1e-7, (name, idx, ad, fd)
        checked += 1
    assert checked >= 40


def test_midpoint_envelope_identities():
    """dp/dmu = p M (x_mid - mu) (the chord midpoint maximises the density along
    the ray), and dt_mid/dmu = M v / A (the +-sqrt terms of the two roots cancel)."""
    rng = np.random.default_rng(5)
    for _ in range(5):
        q = torch.tensor(rng.normal(size=(1, 4)))
        ls = torch.tensor(rng.normal(-1.5, 0.3, size=(1, 3)))
        mu = torch.tensor(rng.normal(size=(1, 3)) * 0.1 + np.array([[2.0, 0.5, 0.3]]), requires_grad=True)
        rx = torch.zeros(3, dtype=torch.float64)
        v = torch.tensor([1.0, 0.1, 0.05], dtype=torch.float64)
        v = v / torch.linalg.norm(v)
        P = oracle.Params(mu, ls, q, torch.zeros(1, dtype=torch.float64), torch.zeros(1, 1, 2, dtype=torch.float64))
        M, Nn, _ = oracle.activate(P)
        M = M[0]
        delta = rx - mu[0]
        A = v @ M @ v
        B = v @ M @ delta
        C = delta @ M @ delta
        t = -B / A
        Q = C - B * B / A
        p = Nn[0] * torch.exp(-Q / 2)
        (gp,) = torch.autograd.grad(p, mu, retain_graph=True)
        (gt,) = torch.autograd.grad(t, mu)
        xm = rx + t.detach() * v
        np.testing.assert_allclose(gp[0].numpy(), (p.detach() * M.detach() @ (xm - mu[0].detach())).numpy(), rtol=1e-10)
        np.testing.assert_allclose(gt[0].numpy(), (M.detach() @ v / A.detach()).numpy(), rtol=1e-10)
        # and the paper's route through both roots gives the same midpoint
        disc = B * B - A * (C - 9)
        if disc > 0:
            d1 = (-B + torch.sqrt(disc)) / A
            d2 = (-B - torch.sqrt(disc)) / A
            assert float((d1 + d2) / 2) == pytest.approx(float(t), rel=1e-12)


def test_vjp_sum_cotangent_equals_broadcast():
    """d(Re conj(g) S_hat)/dtheta with S_hat = sum S_uv equals the per-ray cotangent g on every ray."""
    b = synth.tiny()
    g = Grid(n_az=12, n_el=3, fle_L=1)
    sc = b.scenes[0].subset(slice(0, 150))
    sc = synth.Scene(**{**sc.__dict__, "coeffs": sc.coeffs[:, :g.K]})
    R = g.n_az * g.n_el
    gs = np.array([0.3, -1.1])
    a = oracle.vjp(sc, b.pairs[0], g, np.zeros((R, 2)), g_sum=gs)
    c = oracle.vjp(sc, b.pairs[0], g, np.tile(gs, (R, 1)))
    for k in a:
        np.testing.assert_allclose(a[k], c[k], rtol=1e-12, atol=1e-14)
