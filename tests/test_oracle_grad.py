"""CPU pins of the oracle's gradients (T10): autograd vs FP64 central differences,
and the midpoint identities of App. D.3 (no GPU)."""
import json
import math
import os

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


def test_vjp_abs_scale_is_the_sum_of_group_magnitudes():
    """vjp_abs: its gradient is vjp's (superposition over ray groups); with one
    ray per group its scale is sum_r |dL_r/dtheta + j dL'_r/dtheta| (L' with the
    cotangent j G); a ray listed twice with opposite cotangents cancels the
    gradient exactly while the scale doubles."""
    b = synth.tiny()
    g = Grid(n_az=24, n_el=6, fle_L=2)
    sc = b.scenes[0].subset(slice(0, 300))
    sc = synth.Scene(*(getattr(sc, f).astype(np.float64) for f in ("means", "log_scales", "quats", "logits", "coeffs")))
    p = b.pairs[0]
    G = synth.cotangent((g.n_el * g.n_az,), seed=5).astype(np.float64)
    tot, scl = oracle.vjp_abs(sc, p, g, G, ray_chunk=16)
    ref = oracle.vjp(sc, p, g, G)
    uv = np.array([[3, 1], [10, 2], [17, 4], [22, 5]])
    Gs = G[uv[:, 1] * g.n_az + uv[:, 0]]
    jGs = np.stack([-Gs[:, 1], Gs[:, 0]], 1)
    tot1, scl1 = oracle.vjp_abs(sc, p, g, Gs, rays_uv=uv, ray_chunk=1)
    per_ray = [oracle.vjp(sc, p, g, Gs[i:i + 1], rays_uv=uv[i:i + 1]) for i in range(len(uv))]
    per_ray_j = [oracle.vjp(sc, p, g, jGs[i:i + 1], rays_uv=uv[i:i + 1]) for i in range(len(uv))]
    twice = np.concatenate([uv[1:2], uv[1:2]])
    tot2, scl2 = oracle.vjp_abs(sc, p, g, np.concatenate([Gs[1:2], -Gs[1:2]]), rays_uv=twice, ray_chunk=1)
    hits = 0
    for nm in ("means", "log_scales", "quats", "logits", "coeffs"):
        np.testing.assert_allclose(tot[nm], ref[nm], rtol=1e-10, atol=1e-12 * np.abs(ref[nm]).max())
        assert np.all(scl[nm] >= np.abs(tot[nm]) * (1 - 1e-12))
        mag = [np.hypot(a[nm], c[nm]) for a, c in zip(per_ray, per_ray_j)]
        np.testing.assert_allclose(scl1[nm], sum(mag), rtol=1e-12, atol=0)
        np.testing.assert_allclose(tot1[nm], sum(r[nm] for r in per_ray), rtol=1e-10,
                                   atol=1e-12 * np.abs(tot1[nm]).max(initial=0.0))
        assert np.abs(tot2[nm]).max() <= 1e-12 * np.abs(per_ray[1][nm]).max(initial=0.0)
        np.testing.assert_allclose(scl2[nm], 2 * mag[1], rtol=1e-12, atol=0)
        hits += int((mag[1] > 0).sum())
    assert hits > 0


def test_vjp_abs_scale_of_a_coefficient_is_the_closed_form_magnitude():
    """One isotropic Gaussian, L = 0: per ray dS/dRe(c00) = p e^{-j phi} with
    p = N exp(-rho^2 / 2 s^2) (the point-line distance rho), so with one ray per
    group the scale of Re(c00) and Im(c00) is sum_r |G_r| p_r, whatever the
    phase -- while the gradient itself is only its real projection."""
    g = Grid(n_az=72, n_el=18, fle_L=0)
    rx, tx, mu, s = np.array([1.0, 2.0, 1.0]), np.array([3.0, 0.5, 2.0]), np.array([2.3, 2.9, 2.1]), 0.2
    sc = synth.Scene(mu[None, :], np.full((1, 3), math.log(s)), np.array([[1.0, 0.0, 0.0, 0.0]]),
                     np.array([-30.0]), np.array([[[0.3, -0.2]]]))
    p = Pair(rx, tx, 2.4e9)
    dirs = oracle.ray_dirs(g).reshape(-1, 3)
    w = mu - rx
    nv2 = (dirs * dirs).sum(1)
    rho = np.linalg.norm(np.cross(dirs, w), axis=1) / np.sqrt(nv2)
    hit = (rho <= 3 * s) & (dirs @ w / nv2 >= 1.0) & (np.abs(rho / s - 3) > 1e-6)
    idx = np.nonzero(hit)[0]
    assert len(idx) >= 6
    uv = np.stack([idx % g.n_az, idx // g.n_az], 1)
    G = synth.cotangent((len(idx),), seed=8).astype(np.float64)
    tot, scl = oracle.vjp_abs(sc, p, g, G, rays_uv=uv, ray_chunk=1)
    pr = (2 * math.pi) ** -1.5 / s ** 3 * np.exp(-rho[idx] ** 2 / (2 * s * s))
    want = float((np.hypot(G[:, 0], G[:, 1]) * pr).sum())
    # alpha = sigmoid(-30) G makes T = 1 - O(1e-13) for the one hit on each ray
    assert scl["coeffs"][0, 0, 0] == pytest.approx(want, rel=1e-9)
    assert scl["coeffs"][0, 0, 1] == pytest.approx(want, rel=1e-9)
    assert abs(tot["coeffs"][0, 0, 0]) < 0.9 * want


def test_paper_scale_stored_differences_match_oracle_gradient():
    """The stored reference of the paper-scale gradient test: for each of the
    500 Gaussians and attributes, the oracle's autograd gradient along the
    stored direction equals the FP64 central difference along it (both made
    by tests/golden/make_paper_scale_fd.py), and the per-entry scales bound
    the gradients."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_scale_fd.json")
    with open(path) as fh:
        d = json.load(fh)
    assert len(d["gaussians"]) == 500 and d["grid"]["n_az"] == 360 and d["grid"]["n_el"] == 90
    n_fd = 0
    for rec in d["gaussians"]:
        for n in ("means", "log_scales", "quats", "logits", "coeffs"):
            e = rec[n]
            gr, sc, v = np.asarray(e["grad"]), np.asarray(e["scale"]), np.asarray(e["v"])
            assert np.all(sc >= np.abs(gr) * (1 - 1e-12))
            assert abs(np.linalg.norm(v) - 1.0) <= 1e-12
            if e["fd"] is not None:
                # FD truncation ~h^2 and round-off ~1e-16 |L| / h with h = 1e-6 of the parameter
                # and |L| up to ~1e3 over the Gaussian's rays: ~1e-7 absolute
                assert abs(float(gr @ v) - e["fd"]) <= 1e-5 * float(np.abs(v) @ sc) + 1e-6, (rec["index"], n)
                n_fd += 1
    assert n_fd >= 0.9 * 5 * len(d["gaussians"])
