"""CPU pins of the FP64 oracle (no GPU).

Each test pins a part of the oracle to something other than itself: the
paper's worked example (golden fixture), closed forms, library routines,
symmetry, or an independent high-precision brute force.  A plausible slip in
the oracle (dropped term, wrong sign or index, transposed operand) fails at
least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.special
import scipy.stats
import torch
from scipy.spatial.transform import Rotation

import oracle
import synth
from synth import Grid, Pair, Scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_gaussian(mu, s, coeff00, K, logit=0.0, quat=(1.0, 0.0, 0.0, 0.0), dtype=np.float64):
    c = np.zeros((1, K, 2), dtype)
    c[0, 0] = coeff00
    return Scene(np.array([mu], dtype), np.full((1, 3), math.log(s), dtype), np.array([quat], dtype),
                 np.array([logit], dtype), c)


def stack(scenes):
    return Scene(*(np.concatenate([getattr(s, f) for s in scenes]) for f in
                   ("means", "log_scales", "quats", "logits", "coeffs")))


# A grid with one exactly-representable ray: n_az odd puts a cell centre at
# alpha = pi, and a symmetric elevation span with n_el odd puts one at beta = 0,
# so ray (u=(n_az-1)/2, v=(n_el-1)/2) points along -x with |v| = 1 in FP64.
def axis_grid(L=0):
    return Grid(n_az=3, n_el=1, el_lo=-0.5, el_hi=0.5, fle_L=L, tile_w=16, tile_h=16)


def axis_ray(grid):
    d = oracle.ray_dirs(grid)[0, 1]
    assert d[0] == -1.0 and d[2] == 0.0 and abs(d[1]) < 1e-15
    return d


# ---------------------------------------------------------------- T1 -------
def test_empty_scene_is_exactly_zero():
    g = Grid(n_az=12, n_el=4, fle_L=2)
    empty = Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros((0, 4), np.float32),
                  np.zeros((0,), np.float32), np.zeros((0, g.K, 2), np.float32))
    p = Pair(np.array([1, 1, 1], np.float32), np.array([2, 2, 2], np.float32), 2.4e9)
    r = oracle.render(empty, p, g)
    assert np.all(r["S"] == 0) and r["S_sum"] == 0
    assert oracle.rssi_dbm(r["S_sum"]) == -math.inf


# ---------------------------------------------------------- activation -----
def test_activation_matches_scipy_rotation_and_inverse():
    rng = np.random.default_rng(0)
    n = 64
    q = rng.normal(size=(n, 4)) * rng.uniform(0.5, 2.0, size=(n, 1))   # unnormalised on purpose
    ls = rng.normal(-2.0, 0.5, size=(n, 3))
    a = rng.normal(size=n)
    P = oracle.Params(*(torch.tensor(x) for x in (np.zeros((n, 3)), ls, q, a, np.zeros((n, 1, 2)))))
    M, Nn, o = oracle.activate(P)
    for i in range(n):
        # scipy quaternions are (x, y, z, w)
        R = Rotation.from_quat(np.r_[q[i, 1:], q[i, 0]]).as_matrix()
        Sig = R @ np.diag(np.exp(2 * ls[i])) @ R.T
        np.testing.assert_allclose(M[i].numpy(), np.linalg.inv(Sig), rtol=1e-10, atol=1e-10 * np.abs(M[i].numpy()).max())
        pdf0 = scipy.stats.multivariate_normal(mean=np.zeros(3), cov=Sig).pdf(np.zeros(3))
        assert Nn[i].item() == pytest.approx(pdf0, rel=1e-10)
    np.testing.assert_allclose(o.numpy(), scipy.special.expit(a), rtol=1e-14)


def test_quaternion_sign_and_isotropy():
    rng = np.random.default_rng(1)
    q = rng.normal(size=(8, 4))
    R1 = oracle.rotation_matrix(torch.tensor(q))
    R2 = oracle.rotation_matrix(torch.tensor(-q))
    np.testing.assert_allclose(R1.numpy(), R2.numpy(), atol=1e-14)
    # isotropic scale: M = I / s^2 whatever the rotation
    P = oracle.Params(torch.zeros(8, 3, dtype=torch.float64), torch.full((8, 3), math.log(0.2), dtype=torch.float64),
                      torch.tensor(q), torch.zeros(8, dtype=torch.float64), torch.zeros(8, 1, 2, dtype=torch.float64))
    M, _, _ = oracle.activate(P)
    np.testing.assert_allclose(M.numpy(), np.broadcast_to(np.eye(3) / 0.04, (8, 3, 3)), atol=1e-12)


# ------------------------------------------------------------- T8 FLE ------
def test_legendre_closed_forms():
    x = np.linspace(-1, 1, 41)
    sq = np.sqrt(1 - x * x)
    closed = {
        (0, 0): np.ones_like(x),
        (1, 0): x, (1, 1): -sq,
        (2, 0): 0.5 * (3 * x * x - 1), (2, 1): -3 * x * sq, (2, 2): 3 * (1 - x * x),
    }
    for (l, m), ref in closed.items():
        np.testing.assert_allclose(oracle.assoc_legendre(l, m, x), ref, atol=1e-14)
    # negative orders from the textbook relation, checked on l=1, 2 by hand
    np.testing.assert_allclose(oracle.assoc_legendre(1, -1, x), 0.5 * sq, atol=1e-14)
    np.testing.assert_allclose(oracle.assoc_legendre(2, -1, x), 0.5 * x * sq, atol=1e-14)
    np.testing.assert_allclose(oracle.assoc_legendre(2, -2, x), 0.125 * (1 - x * x), atol=1e-14)


def test_legendre_matches_scipy_lpmv():
    x = np.linspace(-0.999, 0.999, 57)
    for l in range(7):
        for m in range(0, l + 1):
            ref = scipy.special.lpmv(m, l, x)
            np.testing.assert_allclose(oracle.assoc_legendre(l, m, x), ref, rtol=1e-11, atol=1e-11 * max(1, np.abs(ref).max()))


def test_fle_basis_index_and_discrete_orthogonality():
    g = Grid(n_az=36, n_el=9, fle_L=3)
    Y = oracle.ray_basis(g)                       # [n_el, n_az, K]
    alpha, beta = oracle.ray_angles(g)
    # index l^2 + l + m, azimuth factor e^{+j m alpha}
    for l in range(4):
        for m in range(-l, l + 1):
            ref = np.exp(1j * m * alpha)[None, :] * oracle.assoc_legendre(l, m, np.sin(beta))[:, None]
            np.testing.assert_allclose(Y[:, :, l * l + l + m], ref, atol=1e-13)
    # sum over cell-centre azimuths of e^{j (m - m') alpha_u} vanishes for m != m'
    for dm in range(1, 7):
        assert abs(np.exp(1j * dm * alpha).sum()) < 1e-12


# ----------------------------------------------------- T2 closed form ------
@pytest.mark.parametrize("s", [0.05, 0.12])
def test_single_isotropic_gaussian_closed_form(s):
    g = Grid(n_az=72, n_el=18, fle_L=1)
    rx = np.array([1.0, 2.0, 1.0])
    tx = np.array([3.0, 0.5, 2.0])
    mu = np.array([2.3, 2.9, 2.1])
    c00 = np.array([0.3, -0.2])
    sc = one_gaussian(mu, s, c00, g.K, logit=0.7)
    p = Pair(rx, tx, 2.4e9)
    r = oracle.render(sc, p, g)
    dirs = oracle.ray_dirs(g).reshape(-1, 3)
    lam = 3e8 / 2.4e9
    w = mu - rx
    nv2 = (dirs * dirs).sum(1)
    rho = np.linalg.norm(np.cross(dirs, w), axis=1) / np.sqrt(nv2)    # point-line distance
    tpar = dirs @ w / nv2
    path = np.linalg.norm(mu - tx) + tpar
    N = (2 * math.pi) ** -1.5 / s ** 3
    val = N * np.exp(-rho ** 2 / (2 * s * s)) * (c00[0] + 1j * c00[1]) * np.exp(-2j * math.pi * path / lam)
    hit = (rho <= 3 * s) & (tpar >= 1.0)
    ref = np.where(hit, val, 0)
    assert hit.sum() >= 4
    edge = np.abs(rho / s - 3) < 1e-6
    ok = ~edge
    np.testing.assert_allclose(r["S"][ok], ref[ok], rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_hit_requires_midpoint_beyond_ress():
    # Gaussian centred 0.5 m from the RX (inside the RESS of radius 1): no ray counts it
    g = axis_grid()
    rx = np.array([0.0, 0.0, 0.0])
    sc = one_gaussian(rx + np.array([-0.5, 0, 0]), 0.05, np.array([1.0, 0.0]), 1)
    r = oracle.render(sc, Pair(rx, rx, 2.4e9), g)
    assert np.all(r["S"] == 0)
    sc2 = one_gaussian(rx + np.array([-1.5, 0, 0]), 0.05, np.array([1.0, 0.0]), 1)
    r2 = oracle.render(sc2, Pair(rx, rx, 2.4e9), g)
    assert abs(r2["S"][1]) > 0


# ------------------------------------------- T3 paper's worked example -----
def test_worked_example_two_paths_cancel():
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    # the printed delays fix c to the printed precision
    assert ex["d1_m"] / oracle.C0 * 1e9 == pytest.approx(ex["tau1_ns"], abs=5e-4)
    assert ex["d2_m"] / oracle.C0 * 1e9 == pytest.approx(ex["tau2_ns"], abs=5e-4)
    lam = oracle.C0 / ex["f_c_hz"]
    phi1 = 2 * math.pi * ex["d1_m"] / lam
    phi2 = 2 * math.pi * ex["d2_m"] / lam
    assert math.remainder(phi1, 2 * math.pi) == pytest.approx(ex["phi1_rad"], abs=1e-9)
    assert abs(math.remainder(phi2 - phi1, 2 * math.pi)) == pytest.approx(ex["phi2_rad_over_pi"] * math.pi, abs=1e-9)
    # two identical, nearly transparent Gaussians on one ray; TX at the RX so the
    # path lengths are 2*D = 3 m and 3.0625 m
    g = axis_grid()
    v = axis_ray(g)
    rx = np.array([0.25, -0.5, 1.0])
    D1, D2 = ex["d1_m"] / 2, ex["d2_m"] / 2
    sc = stack([one_gaussian(rx + D * v, 0.004, np.array([0.7, 0.1]), 1, logit=-30.0) for D in (D1, D2)])
    r = oracle.render(sc, Pair(rx, rx, ex["f_c_hz"]), g)
    S, A = r["S"][1], r["A_uv"][1]
    assert r["n_active"][1] == 2
    assert abs(S) <= 1e-12 * A
    # with only one path there is no cancellation
    r1 = oracle.render(sc.subset(slice(0, 1)), Pair(rx, rx, ex["f_c_hz"]), g)
    assert abs(r1["S"][1]) == pytest.approx(r1["A_uv"][1], rel=1e-12)


# ---------------------------------------------- T4 translation -------------
@pytest.mark.parametrize("colocated", [True, False])
def test_translation_along_ray_rotates_phase(colocated):
    g = axis_grid()
    v = axis_ray(g)
    rx = np.array([0.1, 0.2, 0.3])
    tx = rx.copy() if colocated else np.array([2.0, -1.0, 0.7])
    f = 5.0e9
    lam = oracle.C0 / f
    mu0 = rx + 2.0 * v + np.array([0.0, 0.01, -0.005])
    out = []
    for delta in (0.0, 0.0137, 0.4):
        mu = mu0 + delta * v
        sc = one_gaussian(mu, 0.06, np.array([0.4, 0.25]), 1)
        out.append((oracle.render(sc, Pair(rx, tx, f), g)["S"][1], np.linalg.norm(mu - tx)))
    S0, dtx0 = out[0]
    for (S, dtx), delta in zip(out[1:], (0.0137, 0.4)):
        extra = delta + (dtx - dtx0)
        if colocated:
            assert extra == pytest.approx(2 * delta, rel=1e-4)   # centre sits 1 cm off the ray
        np.testing.assert_allclose(S, S0 * np.exp(-2j * math.pi * extra / lam), rtol=1e-10)


# -------------------------------------------- T5 transmittance -------------
def test_transmittance_monotone_and_bounded():
    b = synth.tiny()
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    for (u, v) in [(0, 0), (5, 3), (20, 8), (35, 4)]:
        sq = oracle.ray_sequence(sc, p, g, u, v)
        T = sq["T"]
        assert np.all(np.diff(T) <= 0) and T[0] == 1.0 and np.all(T > 0)
        # T falls only at hits, by exactly (1 - alpha)
        h = sq["hit"]
        ratio = T[1:] / T[:-1]
        np.testing.assert_allclose(ratio[~h[:-1]], 1.0)
        np.testing.assert_allclose(ratio[h[:-1]], 1.0 - sq["alpha"][:-1][h[:-1]], rtol=1e-12)
    # without termination, adding a Gaussian never raises any ray's final T
    g0 = Grid(**{**g.__dict__, "t_min": 0.0})
    base = oracle.render(sc, p, g0)
    extra = Scene(np.array([[3.5, 3.0, 2.6]], np.float32), np.full((1, 3), -1.5, np.float32),
                  np.array([[1, 0, 0, 0]], np.float32), np.array([2.0], np.float32), np.zeros((1, g.K, 2), np.float32))
    more = oracle.render(stack([sc, extra]), p, g0)
    assert np.all(more["T_end"] <= base["T_end"] * (1 + 1e-12))
    assert np.any(more["T_end"] < base["T_end"] * (1 - 1e-3))
    assert np.all((base["T_end"] > 0) & (base["T_end"] <= 1))


# ----------------------------------- T6 compositing / termination closed form
@pytest.mark.parametrize("logit,n", [(-1.0, 5), (0.5, 40), (2.0, 40), (6.0, 12)])
def test_stack_on_axis_geometric_series(logit, n):
    g = axis_grid()
    v = axis_ray(g)
    rx = np.zeros(3)
    s = 0.01
    c00 = 0.8
    sc = stack([one_gaussian(rx + (2.0 + 0.1 * i) * v, s, np.array([c00, 0.0]), 1, logit=logit) for i in range(n)])
    r = oracle.render(sc, Pair(rx, rx, 1e-3), g)          # f -> 0: every phase vanishes (3DGS reduction)
    o = 1 / (1 + math.exp(-logit))
    a = min(o, float(np.float32(0.99)))
    t_min = float(np.float32(1e-4))
    n_eff = min(n, sum(1 for i in range(n) if (1 - a) ** i >= t_min))
    N = (2 * math.pi) ** -1.5 / s ** 3
    ref = N * c00 * (1 - (1 - a) ** n_eff) / a
    assert r["n_active"][1] == n_eff
    assert r["S"][1].real == pytest.approx(ref, rel=1e-9)
    assert abs(r["S"][1].imag) < 1e-6 * ref


def test_front_to_back_order():
    g = axis_grid()
    v = axis_ray(g)
    rx = np.zeros(3)
    s1, s2 = 0.02, 0.03
    near = one_gaussian(rx + 2.0 * v, s1, np.array([1.0, 0.0]), 1, logit=1.0)
    far = one_gaussian(rx + 3.0 * v, s2, np.array([0.0, 2.0]), 1, logit=-0.5)
    N1, N2 = [(2 * math.pi) ** -1.5 / s ** 3 for s in (s1, s2)]
    o1 = 1 / (1 + math.exp(-1.0))
    for sc in (stack([near, far]), stack([far, near])):          # index order must not matter
        S = oracle.render(sc, Pair(rx, rx, 1e-3), g)["S"][1]
        assert S == pytest.approx(N1 * 1.0 + (1 - o1) * N2 * 2.0j, rel=1e-9)


# --------------------------------------- T7 azimuth equivariance -----------
def test_azimuth_rotation_shifts_spectrum_one_column():
    g = Grid(n_az=36, n_el=9, fle_L=2)
    b = synth.tiny()
    sc = b.scenes[0].subset(slice(0, 600))
    rx = b.pairs[0].rx.astype(np.float64)
    tx = b.pairs[0].tx.astype(np.float64)
    d = 2 * math.pi / g.n_az
    Rz = np.array([[math.cos(d), -math.sin(d), 0], [math.sin(d), math.cos(d), 0], [0, 0, 1]])
    qz = np.array([math.cos(d / 2), 0, 0, math.sin(d / 2)])

    def qmul(a, b):
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b.T
        return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=1)

    K = g.K
    m_of = np.array([i - int(math.isqrt(i)) ** 2 - int(math.isqrt(i)) for i in range(K)])
    c = sc.coeffs.astype(np.float64)
    cc = (c[..., 0] + 1j * c[..., 1]) * np.exp(-1j * m_of * d)[None, :]
    rot = Scene((sc.means.astype(np.float64) - rx) @ Rz.T + rx, sc.log_scales.astype(np.float64),
                qmul(qz, sc.quats.astype(np.float64)), sc.logits.astype(np.float64),
                np.stack([cc.real, cc.imag], axis=-1))
    sc64 = Scene(*(getattr(sc, f).astype(np.float64) for f in ("means", "log_scales", "quats", "logits", "coeffs")))
    r0 = oracle.render(sc64, Pair(rx, tx, 2.4e9), g)
    r1 = oracle.render(rot, Pair(rx, (tx - rx) @ Rz.T + rx, 2.4e9), g)
    S0 = r0["S_grid"]
    S1 = r1["S_grid"]
    A0 = r0["A_uv"].reshape(g.n_el, g.n_az)
    marg = (r0["marginal"] | np.roll(r1["marginal"].reshape(g.n_el, g.n_az), -1, axis=1).ravel()).reshape(g.n_el, g.n_az)
    shifted = np.roll(S1, -1, axis=1)            # S1[:, u+1] vs S0[:, u], wrapping the seam
    err = np.abs(shifted - S0)
    ok = ~marg
    assert ok.sum() > 0.9 * ok.size
    assert np.all(err[ok] <= 1e-4 * np.maximum(A0[ok], 1e-30))
    assert np.abs(S0).max() > 0


# ------------------------- T9 tiny brute force at 50 digits (paper route) ---
def test_tiny_brute_force_mpmath():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(7)
    g = Grid(n_az=4, n_el=2, fle_L=1, el_lo=0.1, el_hi=1.2)
    n = 7
    rx = np.array([1.0, 1.0, 1.0], np.float32)
    tx = np.array([0.2, 1.7, 0.4], np.float32)
    # place Gaussians around rays so that most rays see several of them
    dirs = oracle.ray_dirs(g).reshape(-1, 3)
    mu = np.array([rx + rng.uniform(1.2, 2.5) * dirs[i % 8] + rng.normal(0, 0.05, 3) for i in range(n)], np.float32)
    sc = Scene(mu, rng.normal(-1.8, 0.3, (n, 3)).astype(np.float32), rng.normal(size=(n, 4)).astype(np.float32),
               rng.normal(0, 1, n).astype(np.float32), rng.normal(0, 0.3, (n, g.K, 2)).astype(np.float32))
    f = 2.4e9
    r = oracle.render(sc, Pair(rx, tx, f), g)
    alpha_u, beta_v = oracle.ray_angles(g)
    lam = mp.mpf(3e8) / mp.mpf(f)
    order = sorted(range(n), key=lambda i: (int(np.float32(((np.float64(mu[i]) - np.float64(rx)) ** 2)[:2].sum()
                                                            + ((np.float64(mu[i][2]) - np.float64(rx[2])) ** 2))
                                                 .view(np.uint32)), i))
    for k in range(g.n_el * g.n_az):
        v_i, u_i = divmod(k, g.n_az)
        vd = [mp.mpf(float(x)) for x in oracle.ray_dirs(g)[v_i, u_i]]
        Y = []
        for l in range(g.fle_L + 1):
            for m in range(-l, l + 1):
                x = mp.sin(mp.mpf(float(beta_v[v_i])))
                Y.append(mp.expj(m * mp.mpf(float(alpha_u[u_i]))) * mp.legenp(l, m, x))
        S = mp.mpc(0)
        rho_prod = mp.mpf(1)
        for i in order:
            qw, qx, qy, qz = [mp.mpf(float(x)) for x in sc.quats[i]]
            nq = mp.sqrt(qw ** 2 + qx ** 2 + qy ** 2 + qz ** 2)
            qw, qx, qy, qz = qw / nq, qx / nq, qy / nq, qz / nq
            Rm = mp.matrix([[1 - 2 * (qy ** 2 + qz ** 2), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)],
                            [2 * (qx * qy + qw * qz), 1 - 2 * (qx ** 2 + qz ** 2), 2 * (qy * qz - qw * qx)],
                            [2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx ** 2 + qy ** 2)]])
            Sd = mp.diag([mp.e ** mp.mpf(float(x)) for x in sc.log_scales[i]])
            Sig = Rm * Sd * Sd.T * Rm.T
            Si = mp.inverse(Sig)
            m_ = mp.matrix([mp.mpf(float(x)) for x in mu[i]])
            lrx = mp.matrix([mp.mpf(float(x)) for x in rx])
            v_ = mp.matrix(vd)
            w = lrx - m_
            A = (v_.T * Si * v_)[0]
            B = (v_.T * Si * w)[0]
            C = (w.T * Si * w)[0]
            disc = B * B - A * (C - 9)
            if disc < 0:
                continue
            d1 = (-B + mp.sqrt(disc)) / A
            d2 = (-B - mp.sqrt(disc)) / A
            tm = (d1 + d2) / 2
            if tm < 1:
                continue
            x_int = lrx + tm * v_
            dx = x_int - m_
            pdf = mp.exp(-(dx.T * Si * dx)[0] / 2) / ((2 * mp.pi) ** mp.mpf(1.5) * mp.sqrt(mp.det(Sig)))
            if rho_prod < mp.mpf(float(np.float32(1e-4))):
                break
            psi = sum(complex(float(sc.coeffs[i, j, 0]), float(sc.coeffs[i, j, 1])) * Y[j] for j in range(g.K))
            dist = mp.norm(m_ - mp.matrix([mp.mpf(float(x)) for x in tx])) + tm
            S += pdf * psi * mp.expj(-2 * mp.pi * dist / lam) * rho_prod
            o = 1 / (1 + mp.e ** (-mp.mpf(float(sc.logits[i]))))
            a = min(o * mp.exp(-(dx.T * Si * dx)[0] / 2), mp.mpf(float(np.float32(0.99))))
            rho_prod *= (1 - a)
        ref = complex(S)
        got = r["S"][k]
        assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref)), (k, got, ref)
    assert (np.abs(r["S"]) > 0).sum() >= 4


# --------------------------------------------- binning definition ----------
def _brute_cell_cover(mu, ls, rx, grid, theta_extra=0.0):
    """Cells whose centre direction lies inside the bounding cap (brute force)."""
    alpha, beta = oracle.ray_angles(grid)
    A, Bt = np.meshgrid(alpha, beta)
    dirs = np.stack([np.cos(Bt) * np.cos(A), np.cos(Bt) * np.sin(A), np.sin(Bt)], -1)
    e = mu.astype(np.float64) - rx.astype(np.float64)
    D = np.linalg.norm(e)
    Rb = 3 * math.exp(float(np.max(ls.astype(np.float64))))
    if D + Rb < grid.r_rx:               # wholly inside the RESS: no ray can count it
        return np.zeros(dirs.shape[:2], bool)
    if D <= Rb:
        return np.ones(dirs.shape[:2], bool)
    th = math.asin(Rb / D) + theta_extra
    cosang = dirs @ (e / D)
    return cosang >= math.cos(th)


def test_cap_rect_contains_every_cap_cell_and_tile_lists_are_conservative():
    b = synth.tiny()
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    for grid in (g, Grid(n_az=72, n_el=18, fle_L=2, tile_w=8, tile_h=4)):
        tu0, ntu, tv0, ntv, marg = oracle.cap_rects(sc.means, sc.log_scales, p.rx, grid)
        assert not marg.any()
        for i in range(0, sc.n, 7):
            cells = _brute_cell_cover(sc.means[i], sc.log_scales[i], p.rx, grid)
            tiles = set(oracle.rect_tiles(int(tu0[i]), int(ntu[i]), int(tv0[i]), int(ntv[i]), grid))
            vv, uu = np.nonzero(cells)
            need = set((vv // grid.tile_h) * grid.n_tiles_az + uu // grid.tile_w)
            assert need <= tiles, i
        # every brute-force hit is in one of its Gaussian's tiles
        lists, keys, _ = oracle.tile_lists(sc.means, sc.log_scales, p.rx, grid)
        members = [set(l.tolist()) for l in lists]
        rays = [(u, v) for v in range(0, grid.n_el, 3) for u in range(0, grid.n_az, 5)]
        for (u, v) in rays:
            sq = oracle.ray_sequence(sc, p, grid, u, v)
            tile = (v // grid.tile_h) * grid.n_tiles_az + u // grid.tile_w
            hits = sq["order"][sq["hit"]]
            assert set(hits.tolist()) <= members[tile], (u, v)


def test_tile_lists_sorted_by_key_then_index():
    b = synth.tiny()
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    lists, keys, _ = oracle.tile_lists(sc.means, sc.log_scales, p.rx, g)
    for l, k in zip(lists, keys):
        pairs = list(zip(k.tolist(), l.tolist()))
        assert pairs == sorted(pairs)
    # key32 order equals the order of the exact distance
    d = np.linalg.norm(sc.means.astype(np.float64) - p.rx.astype(np.float64), axis=1)
    k = oracle.depth_key32(sc.means, p.rx)
    o = np.argsort(k, kind="stable")
    assert np.all(np.diff(d[o]) >= -1e-6)


def test_cap_rect_seam_wrap_and_culls():
    g = Grid(n_az=360, n_el=90, fle_L=0, tile_w=16, tile_h=16)
    rx = np.array([5.0, 5.0, 1.0])
    # a Gaussian straight along +x (azimuth ~0) covers tiles on both sides of the seam
    sc = one_gaussian(np.array([8.0, 5.0, 1.5]), 0.1, np.array([1.0, 0.0]), 1)
    tu0, ntu, tv0, ntv, _ = oracle.cap_rects(sc.means, sc.log_scales, rx, g)
    tiles = oracle.rect_tiles(int(tu0[0]), int(ntu[0]), int(tv0[0]), int(ntv[0]), g)
    cols = sorted(set(t % g.n_tiles_az for t in tiles))
    assert 0 in cols and g.n_tiles_az - 1 in cols
    # below the RX (elevation span is [0, 90) deg) -> culled
    below = one_gaussian(np.array([8.0, 5.0, 0.2]), 0.05, np.array([1.0, 0.0]), 1)
    assert oracle.cap_rects(below.means, below.log_scales, rx, g)[1][0] == 0
    # inside the RESS -> culled; RX inside the bounding sphere -> every tile
    ress = one_gaussian(np.array([5.3, 5.0, 1.2]), 0.05, np.array([1.0, 0.0]), 1)
    assert oracle.cap_rects(ress.means, ress.log_scales, rx, g)[1][0] == 0
    big = one_gaussian(np.array([5.3, 5.0, 1.2]), 0.5, np.array([1.0, 0.0]), 1)
    r = oracle.cap_rects(big.means, big.log_scales, rx, g)
    assert r[1][0] * r[3][0] == g.n_tiles


# --------------------------------------------------------------------------
# Paper footprint binning variant (Sec. 3.3 splatting: Sigma2D = J Sigma J^T,
# r_k = 3 sqrt(lambda_max)); tile 1 x 1 makes the rectangle the ray square.
# --------------------------------------------------------------------------

def _index_map(e, g):
    d_a = 2 * math.pi / g.n_az
    d_b = (g.el_hi - g.el_lo) / g.n_el
    return np.array([math.atan2(e[1], e[0]) / d_a,
                     (math.atan2(e[2], math.sqrt(e[0] ** 2 + e[1] ** 2)) - g.el_lo) / d_b])


def test_footprint_jacobian_matches_finite_differences():
    g = Grid(n_az=360, n_el=90, el_lo=0.0, el_hi=math.pi / 2)
    rng = np.random.default_rng(5)
    for _ in range(20):
        e = rng.normal(size=3) * 3
        J = oracle.footprint_jacobian(e, g)
        h = 1e-6
        fd = np.stack([(_index_map(e + h * ax, g) - _index_map(e - h * ax, g)) / (2 * h) for ax in np.eye(3)], 1)
        np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-6)
        # the radial direction maps to no displacement
        np.testing.assert_allclose(J @ e, 0.0, atol=1e-9)


def _deg_dir(az_deg, el_deg):
    a, b = math.radians(az_deg), math.radians(el_deg)
    return np.array([math.cos(b) * math.cos(a), math.cos(b) * math.sin(a), math.sin(b)])


def _quat_x_to(axis_world, roll=0.0):
    """(w, x, y, z) of a rotation that takes the x axis to ``axis_world``."""
    a = axis_world / np.linalg.norm(axis_world)
    v = np.cross([1.0, 0.0, 0.0], a)
    ang = math.acos(np.clip(a[0], -1.0, 1.0))
    rot = Rotation.from_rotvec(v / np.linalg.norm(v) * ang) * Rotation.from_rotvec([roll, 0.0, 0.0])
    x, y, z, w = rot.as_quat()
    return (w, x, y, z)


def test_footprint_isotropic_and_anisotropic_closed_forms():
    g = Grid(n_az=360, n_el=90, fle_L=0, tile_w=1, tile_h=1)     # 1 degree cells
    rx = np.array([5.0, 4.0, 1.5])
    D, az, el = 5.0, 100.3, 30.4
    e = D * _deg_dir(az, el)
    rho = D * math.cos(math.radians(el))
    d1 = math.radians(1.0)
    # isotropic: lambda_max = s^2 max(1/(rho da)^2, 1/(D db)^2) = (s / (rho da))^2; r_k = 4.5
    s = 4.5 * rho * d1 / 3.0
    sc = one_gaussian(rx + e, s, np.array([1.0, 0.0]), 1)
    tu0, ntu, tv0, ntv, marg = oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, rx, g)
    assert not marg[0]
    assert (tu0[0], ntu[0], tv0[0], ntv[0]) == (96, 9, 26, 9)
    # long axis along the ray: it projects to nothing, same square as the isotropic one
    ls = np.log([[0.4, s, s]])
    q = np.array([_quat_x_to(e, roll=0.7)])
    r = oracle.footprint_rects(sc.means, ls, q, rx, g)
    assert (r[0][0], r[1][0], r[2][0], r[3][0]) == (96, 9, 26, 9)
    # long axis along the azimuth tangent: a = (s_big / (rho da))^2, c = (s / (D db))^2, b = 0
    t_az = np.array([-math.sin(math.radians(az)), math.cos(math.radians(az)), 0.0])
    s_big = 6.5 * rho * d1 / 3.0                                 # r_k = 6.5 -> m = 6
    r = oracle.footprint_rects(sc.means, np.log([[s_big, s, s]]), np.array([_quat_x_to(t_az, roll=0.3)]), rx, g)
    assert (r[0][0], r[1][0], r[2][0], r[3][0]) == (94, 13, 24, 13)
    # the same axis along the elevation tangent: c dominates, r_k = 3 s_big / (D db)
    t_el = np.array([-math.sin(math.radians(el)) * math.cos(math.radians(az)),
                     -math.sin(math.radians(el)) * math.sin(math.radians(az)), math.cos(math.radians(el))])
    s_el = 7.5 * D * d1 / 3.0                                    # r_k = 7.5 -> m = 7
    r = oracle.footprint_rects(sc.means, np.log([[s_el, s, s]]), np.array([_quat_x_to(t_el, roll=1.1)]), rx, g)
    assert (r[0][0], r[1][0], r[2][0], r[3][0]) == (93, 15, 23, 15)


def test_footprint_guards_vertical_and_tiles():
    g = Grid(n_az=360, n_el=90, fle_L=0, tile_w=16, tile_h=16)
    rx = np.array([5.0, 5.0, 1.0])
    one = lambda mu, s: one_gaussian(np.asarray(mu, float), s, np.array([1.0, 0.0]), 1)
    fr = lambda sc: oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, rx, g)
    # straight above the receiver: every column, the top rows
    r = fr(one([5.0, 5.0, 3.0], 0.05))
    assert r[1][0] == g.n_tiles_az and r[2][0] + r[3][0] == -(-90 // 16)
    # inside the RESS -> culled; receiver inside the bounding sphere -> every tile
    assert fr(one([5.3, 5.0, 1.2], 0.05))[1][0] == 0
    r = fr(one([5.3, 5.0, 1.2], 0.5))
    assert r[1][0] * r[3][0] == g.n_tiles
    # at the seam: columns on both sides
    r = fr(one([8.0, 5.0, 1.5], 0.1))
    tiles = oracle.rect_tiles(int(r[0][0]), int(r[1][0]), int(r[2][0]), int(r[3][0]), g)
    cols = sorted(set(t % g.n_tiles_az for t in tiles))
    assert 0 in cols and g.n_tiles_az - 1 in cols


def test_trace_rect_restriction_keeps_conservative_results():
    """Restricting each ray to the exact cap's tiles changes nothing (the cap
    holds every hit); the footprint restriction only removes hits."""
    b = synth.tiny(n=400)
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    full = oracle.render(sc, p, g)
    capped = oracle.render(sc, p, g, rects=oracle.cap_rects(sc.means, sc.log_scales, p.rx, g))
    np.testing.assert_array_equal(full["n_active"], capped["n_active"])
    np.testing.assert_allclose(full["S"], capped["S"], rtol=1e-12, atol=1e-12 * np.abs(full["S"]).max())
    fp = oracle.render(sc, p, g, rects=oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, p.rx, g))
    assert np.all(fp["n_active"] <= full["n_active"] + (fp["T_end"] < g.t_min * 1.01))


def test_rect_allow_matches_rect_tile_enumeration():
    """The per-(ray, Gaussian) restriction mask equals membership of the ray's
    tile in the rectangle's explicit tile list (seam-wrapping ones included)."""
    g = Grid(n_az=72, n_el=18, fle_L=0, tile_w=8, tile_h=4)
    b = synth.tiny(grid=g, n=300)
    sc, p = b.scenes[0], b.pairs[0]
    vv, uu = np.meshgrid(np.arange(g.n_el), np.arange(g.n_az), indexing="ij")
    uv = np.stack([uu.ravel(), vv.ravel()], 1)
    tile_of = (uv[:, 1] // g.tile_h) * g.n_tiles_az + uv[:, 0] // g.tile_w
    for rects in (oracle.cap_rects(sc.means, sc.log_scales, p.rx, g),
                  oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, p.rx, g)):
        allow = oracle.rect_allow(rects, g, uv)
        wraps = 0
        for i in range(sc.n):
            tiles = set(oracle.rect_tiles(int(rects[0][i]), int(rects[1][i]), int(rects[2][i]), int(rects[3][i]), g))
            wraps += int(rects[0][i] + rects[1][i] > g.n_tiles_az)
            np.testing.assert_array_equal(allow[:, i], np.isin(tile_of, list(tiles)))
        assert wraps > 0
