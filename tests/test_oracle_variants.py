"""CPU pins of the oracle's paper-literal variants (no GPU).

  depth_order = 1    hits taken in increasing chord-midpoint parameter t_mid
                     (App. A.3, discretized rendering equation)
  fle_eval = 1       radiance psi_k evaluated once per Gaussian at the
                     direction of its mean (the per-Gaussian alternative to
                     Sec. 3.2's per-ray FLE)
  transmittance = 1  rho_m = exp(-alpha_m dt_m) over the 3-sigma chord
                     (App. A.2 transmittance derivation)

Each is pinned to a 50-digit brute force along the paper's route (both roots,
explicit sort by t_mid, explicit product of rho_m), to closed forms of one or
two Gaussians, and its gradients to FP64 central differences.
"""
import math

import numpy as np
import pytest
import scipy.special
import torch

import oracle
import synth
from synth import Grid, Pair, Scene

VARIANTS = [dict(depth_order=1), dict(fle_eval=1), dict(transmittance=1),
            dict(depth_order=1, fle_eval=1, transmittance=1)]


def grid_with(**kw):
    g = Grid(**{k: v for k, v in kw.items() if k in Grid.__dataclass_fields__})
    return g


def one(mu, s, c, logit=0.0, K=1):
    cc = np.zeros((1, K, 2))
    cc[0, :len(c)] = c
    return Scene(np.array([mu], float), np.full((1, 3), math.log(s)), np.array([[1.0, 0, 0, 0]]),
                 np.array([logit], float), cc)


def stack(scenes):
    return Scene(*(np.concatenate([getattr(s, f) for s in scenes]) for f in
                   ("means", "log_scales", "quats", "logits", "coeffs")))


def axis(g):
    v = oracle.ray_dirs(g)[(g.n_el - 1) // 2, (g.n_az - 1) // 2]
    assert v[0] == -1.0 and v[2] == 0.0 and abs(v[1]) < 1e-15
    return v


def _mp_render(mp, sc, rx, tx, f, g, variant):
    """The paper's route at 50 digits: Sigma from R S S^T R^T, its inverse and
    determinant, both roots of the 3-sigma quadratic, midpoint, density, and
    the explicit product of the transmittances of the earlier hits."""
    n = sc.n
    lam = mp.mpf(3e8) / mp.mpf(f)
    alpha_u, beta_v = oracle.ray_angles(g)
    key = lambda i: (int(np.float32(((np.float64(sc.means[i]) - np.float64(rx)) ** 2)[:2].sum()
                                    + (np.float64(sc.means[i][2]) - np.float64(rx[2])) ** 2).view(np.uint32)), i)
    order = sorted(range(n), key=key)
    lrx = mp.matrix([mp.mpf(float(x)) for x in rx])
    ltx = mp.matrix([mp.mpf(float(x)) for x in tx])

    def basis(alpha, x):
        return [mp.expj(m * alpha) * mp.legenp(l, m, x) for l in range(g.fle_L + 1) for m in range(-l, l + 1)]

    out = []
    for k in range(g.n_el * g.n_az):
        v_i, u_i = divmod(k, g.n_az)
        v_ = mp.matrix([mp.mpf(float(x)) for x in oracle.ray_dirs(g)[v_i, u_i]])
        Yray = basis(mp.mpf(float(alpha_u[u_i])), mp.sin(mp.mpf(float(beta_v[v_i]))))
        hits = []
        for pos, i in enumerate(order):
            qw, qx, qy, qz = [mp.mpf(float(x)) for x in sc.quats[i]]
            nq = mp.sqrt(qw ** 2 + qx ** 2 + qy ** 2 + qz ** 2)
            qw, qx, qy, qz = qw / nq, qx / nq, qy / nq, qz / nq
            Rm = mp.matrix([[1 - 2 * (qy ** 2 + qz ** 2), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)],
                            [2 * (qx * qy + qw * qz), 1 - 2 * (qx ** 2 + qz ** 2), 2 * (qy * qz - qw * qx)],
                            [2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx ** 2 + qy ** 2)]])
            Sd = mp.diag([mp.e ** mp.mpf(float(x)) for x in sc.log_scales[i]])
            Sig = Rm * Sd * Sd.T * Rm.T
            Si = mp.inverse(Sig)
            m_ = mp.matrix([mp.mpf(float(x)) for x in sc.means[i]])
            w = lrx - m_
            A = (v_.T * Si * v_)[0]
            B = (v_.T * Si * w)[0]
            C = (w.T * Si * w)[0]
            disc = B * B - A * (C - 9)
            if disc < 0:
                continue
            t_out = (-B + mp.sqrt(disc)) / A
            t_in = (-B - mp.sqrt(disc)) / A
            tm = (t_in + t_out) / 2
            if tm < 1:
                continue
            dx = lrx + tm * v_ - m_
            Gm = mp.exp(-(dx.T * Si * dx)[0] / 2)
            pdf = Gm / ((2 * mp.pi) ** mp.mpf(1.5) * mp.sqrt(mp.det(Sig)))
            if variant.get("fle_eval"):
                e = m_ - lrx
                Y = basis(mp.atan2(e[1], e[0]), e[2] / mp.norm(e))
            else:
                Y = Yray
            psi = sum(mp.mpc(float(sc.coeffs[i, j, 0]), float(sc.coeffs[i, j, 1])) * Y[j] for j in range(g.K))
            dist = mp.norm(m_ - ltx) + tm
            c_t = pdf * psi * mp.expj(-2 * mp.pi * dist / lam)
            if variant.get("transmittance"):
                rho = mp.exp(-mp.e ** mp.mpf(float(sc.logits[i])) * (t_out - t_in))
            else:
                o = 1 / (1 + mp.e ** (-mp.mpf(float(sc.logits[i]))))
                rho = 1 - min(o * Gm, mp.mpf(float(np.float32(0.99))))
            hits.append((tm, pos, c_t, rho))
        if variant.get("depth_order"):
            hits.sort(key=lambda h: (h[0], h[1]))
        S = mp.mpc(0)
        prod = mp.mpf(1)
        for tm, pos, c_t, rho in hits:
            if prod < mp.mpf(float(np.float32(1e-4))):
                break
            S += prod * c_t
            prod *= rho
        out.append(complex(S))
    return np.array(out)


@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "+".join(v))
def test_variants_match_paper_route_at_50_digits(variant):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(17)
    g = grid_with(n_az=4, n_el=2, fle_L=1, el_lo=0.1, el_hi=1.2, **variant)
    n = 9
    rx = np.array([1.0, 1.0, 1.0], np.float32)
    tx = np.array([0.2, 1.7, 0.4], np.float32)
    dirs = oracle.ray_dirs(g).reshape(-1, 3)
    mu = np.array([rx + rng.uniform(1.2, 2.5) * dirs[i % 8] + rng.normal(0, 0.08, 3) for i in range(n)], np.float32)
    # plus two whose distance order and midpoint order disagree on ray 0 (off-axis nearer centre)
    d0 = dirs[0].astype(np.float64)
    side = np.cross(d0, [0.0, 0.0, 1.0])
    side /= np.linalg.norm(side)
    extra = np.array([rx + math.sqrt(2.0 ** 2 - 0.15 ** 2) * d0 + 0.15 * side, rx + 1.998 * d0], np.float32)
    mu = np.concatenate([mu, extra])
    ls = np.concatenate([rng.normal(-1.6, 0.3, (n, 3)), np.log([[0.06] * 3, [0.05] * 3])]).astype(np.float32)
    n += 2
    sc = Scene(mu, ls, rng.normal(size=(n, 4)).astype(np.float32),
               rng.normal(0, 1, n).astype(np.float32), rng.normal(0, 0.3, (n, g.K, 2)).astype(np.float32))
    r = oracle.render(sc, Pair(rx, tx, 2.4e9), g)
    ref = _mp_render(mp, sc, rx, tx, 2.4e9, g, variant)
    assert (np.abs(ref) > 0).sum() >= 4
    np.testing.assert_allclose(r["S"], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
    # and each variant changes the result of the default reading somewhere
    base = oracle.render(sc, Pair(rx, tx, 2.4e9), grid_with(n_az=4, n_el=2, fle_L=1, el_lo=0.1, el_hi=1.2))
    assert np.abs(base["S"] - r["S"]).max() > 1e-6 * np.abs(ref).max()


# --------------------------------------------------- depth_order = 1 ------
def _two_disagreeing(g):
    """A: centre 2.0 m from the RX, 0.15 m off the axis ray (t_mid = 1.99437...);
    B: on the axis at 1.998 m.  Key order (distance) puts B first, t_mid order A."""
    v = axis(g)
    rx = np.zeros(3)
    sA, sB = 0.06, 0.05
    muA = rx + math.sqrt(2.0 ** 2 - 0.15 ** 2) * v + np.array([0.0, 0.15, 0.0])
    muB = rx + 1.998 * v
    A = one(muA, sA, [(0.9, 0.2)], logit=1.5)
    B = one(muB, sB, [(-0.3, 0.7)], logit=0.5)
    return rx, A, B, muA, muB, sA, sB, v


def test_tmid_order_two_gaussians_closed_form():
    g = grid_with(n_az=3, n_el=1, el_lo=-0.5, el_hi=0.5, fle_L=0, depth_order=1)
    rx, A, B, muA, muB, sA, sB, v = _two_disagreeing(g)
    f = 1e-3                                          # no propagation phase (3DGS reduction)
    N = lambda s: (2 * math.pi) ** -1.5 / s ** 3
    oA, oB = 1 / (1 + math.exp(-1.5)), 1 / (1 + math.exp(-0.5))
    gA = math.exp(-0.5 * (0.15 / sA) ** 2)
    cA = N(sA) * gA * (0.9 + 0.2j)
    cB = N(sB) * (-0.3 + 0.7j)
    tA = float(v @ (muA - rx))
    assert tA < 1.998 and np.linalg.norm(muA - rx) > 1.998
    for sc in (stack([A, B]), stack([B, A])):
        S = oracle.render(sc, Pair(rx, rx, f), g)["S"][1]
        assert S == pytest.approx(cA + (1 - oA * gA) * cB, rel=1e-9)
        g0 = grid_with(n_az=3, n_el=1, el_lo=-0.5, el_hi=0.5, fle_L=0)
        S0 = oracle.render(sc, Pair(rx, rx, f), g0)["S"][1]
        assert S0 == pytest.approx(cB + (1 - oB) * cA, rel=1e-9)


def test_tmid_order_equals_key_order_on_the_axis():
    """Gaussians centred on a ray have t_mid = distance: both orders agree."""
    g0 = grid_with(n_az=3, n_el=1, el_lo=-0.5, el_hi=0.5, fle_L=0)
    g1 = grid_with(n_az=3, n_el=1, el_lo=-0.5, el_hi=0.5, fle_L=0, depth_order=1)
    v = axis(g0)
    rng = np.random.default_rng(2)
    sc = stack([one(np.zeros(3) + d * v, 0.02, [(rng.normal(), rng.normal())], logit=rng.normal())
                for d in rng.uniform(1.5, 4.0, 12)])
    a = oracle.render(sc, Pair(np.zeros(3), np.array([1.0, 2.0, 0.5]), 5e9), g0)["S"][1]
    b = oracle.render(sc, Pair(np.zeros(3), np.array([1.0, 2.0, 0.5]), 5e9), g1)["S"][1]
    assert a == pytest.approx(b, rel=1e-12)


def test_tmid_near_tie_is_flagged_and_both_orders_enumerated():
    g = grid_with(n_az=3, n_el=1, el_lo=-0.5, el_hi=0.5, fle_L=0, depth_order=1)
    v = axis(g)
    rx = np.zeros(3)
    # two Gaussians with t_mid 2.0 and 2.0 + 5e-7 (inside the tie band), off-axis on either side
    A = one(rx + 2.0 * v + np.array([0.0, 0.05, 0.0]), 0.05, [(1.0, 0.0)], logit=1.0)
    B = one(rx + (2.0 + 5e-7) * v + np.array([0.0, 0.0, -0.04]), 0.05, [(0.0, 1.0)], logit=0.0)
    sc = stack([A, B])
    r = oracle.render(sc, Pair(rx, rx, 1e-3), g)
    assert r["marginal"][1]
    vs = oracle.ray_variants(sc, Pair(rx, rx, 1e-3), g, 1, 0)
    sq = oracle.ray_sequence(sc, Pair(rx, rx, 1e-3), g, 1, 0)
    ct = {int(gid): c for gid, c in zip(sq["order"], sq["ct"])}
    al = {int(gid): a for gid, a in zip(sq["order"], sq["alpha"])}
    ab = ct[0] + (1 - al[0]) * ct[1]
    ba = ct[1] + (1 - al[1]) * ct[0]
    scale = abs(ct[0]) + abs(ct[1])
    assert any(abs(x - ab) <= 1e-12 * scale for x in vs) and any(abs(x - ba) <= 1e-12 * scale for x in vs)
    # far apart: not flagged
    B2 = one(rx + 2.01 * v + np.array([0.0, 0.0, -0.04]), 0.05, [(0.0, 1.0)], logit=0.0)
    assert not oracle.render(stack([A, B2]), Pair(rx, rx, 1e-3), g)["marginal"][1]


# ------------------------------------------------------ fle_eval = 1 ------
def test_fle_basis_at_a_direction_closed_forms_and_scipy():
    rng = np.random.default_rng(4)
    e = rng.normal(size=(40, 3))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    Yr, Yi = oracle.fle_basis_dir(6, torch.tensor(e))
    Y = Yr.numpy() + 1j * Yi.numpy()
    w = e[:, 0] + 1j * e[:, 1]
    np.testing.assert_allclose(Y[:, 0], 1.0, atol=1e-15)
    np.testing.assert_allclose(Y[:, 2], e[:, 2], atol=1e-15)               # l=1, m=0
    np.testing.assert_allclose(Y[:, 3], -w, atol=1e-15)                    # l=1, m=1: -sin(b) e^{ja}
    np.testing.assert_allclose(Y[:, 1], 0.5 * np.conj(w), atol=1e-15)      # l=1, m=-1
    np.testing.assert_allclose(Y[:, 8], 3 * w * w, atol=1e-14)             # l=2, m=2: 3 (1-x^2) e^{2ja}
    alpha = np.arctan2(e[:, 1], e[:, 0])
    x = e[:, 2]
    for l in range(7):
        for m in range(-l, l + 1):
            pm = scipy.special.lpmv(abs(m), l, x)
            if m < 0:
                pm = (-1) ** (-m) * math.factorial(l + m) / math.factorial(l - m) * pm
            ref = np.exp(1j * m * alpha) * pm
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, rtol=1e-11, atol=1e-11 * max(1, np.abs(ref).max()))
    # the pole: finite, and only m = 0 survives
    Yr, Yi = oracle.fle_basis_dir(3, torch.tensor([[0.0, 0.0, 1.0]], dtype=torch.float64))
    m_of = [i - int(math.isqrt(i)) ** 2 - int(math.isqrt(i)) for i in range(16)]
    for i in range(16):
        if m_of[i] != 0:
            assert Yr[0, i] == 0 and Yi[0, i] == 0
        else:
            assert Yr[0, i] == pytest.approx(1.0)


def test_fle_per_gaussian_single_gaussian_closed_form():
    """One isotropic Gaussian: S_uv = N e^{-rho^2/2s^2} psi(e_k) e^{-j 2 pi d/lambda}
    with psi(e_k) the same for every ray, from scipy's Legendre functions at the
    mean's azimuth and elevation."""
    g = grid_with(n_az=72, n_el=18, fle_L=2, fle_eval=1)
    rng = np.random.default_rng(8)
    rx = np.array([1.0, 2.0, 1.0])
    tx = np.array([3.0, 0.5, 2.0])
    mu = np.array([2.3, 2.9, 2.1])
    s = 0.12
    c = rng.normal(0, 0.3, (g.K, 2))
    sc = one(mu, s, [tuple(x) for x in c], logit=0.7, K=g.K)
    r = oracle.render(sc, Pair(rx, tx, 2.4e9), g)
    e = (mu - rx) / np.linalg.norm(mu - rx)
    a_k, x_k = math.atan2(e[1], e[0]), e[2]
    psi = 0j
    for l in range(3):
        for m in range(-l, l + 1):
            pm = scipy.special.lpmv(abs(m), l, x_k)
            if m < 0:
                pm = (-1) ** (-m) * math.factorial(l + m) / math.factorial(l - m) * pm
            psi += complex(*c[l * l + l + m]) * np.exp(1j * m * a_k) * pm
    dirs = oracle.ray_dirs(g).reshape(-1, 3)
    w = mu - rx
    nv2 = (dirs * dirs).sum(1)
    rho = np.linalg.norm(np.cross(dirs, w), axis=1) / np.sqrt(nv2)
    tpar = dirs @ w / nv2
    N = (2 * math.pi) ** -1.5 / s ** 3
    val = N * np.exp(-rho ** 2 / (2 * s * s)) * psi * np.exp(-2j * math.pi * (np.linalg.norm(mu - tx) + tpar) / 0.125)
    hit = (rho <= 3 * s) & (tpar >= 1.0)
    assert hit.sum() >= 4
    ok = np.abs(rho / s - 3) > 1e-6
    np.testing.assert_allclose(r["S"][ok], np.where(hit, val, 0)[ok], rtol=1e-9, atol=1e-9 * np.abs(val).max())


# --------------------------------------------------- transmittance = 1 ----
def test_chord_transmittance_two_gaussians_closed_form():
    """Sphere of radius 3s at perpendicular distance rho: chord 2 sqrt(9 s^2 - rho^2),
    so the far Gaussian is weighted by exp(-e^{a} 2 sqrt(9 s^2 - rho^2))."""
    g = grid_with(n_az=3, n_el=1, el_lo=-0.5, el_hi=0.5, fle_L=0, transmittance=1)
    v = axis(g)
    rx = np.zeros(3)
    s1, s2, rho1 = 0.05, 0.04, 0.07
    a1 = 0.8
    near = one(rx + 2.0 * v + np.array([0.0, rho1, 0.0]), s1, [(1.0, 0.5)], logit=a1)
    far = one(rx + 3.0 * v, s2, [(-0.4, 0.9)], logit=-2.0)
    N = lambda s: (2 * math.pi) ** -1.5 / s ** 3
    c1 = N(s1) * math.exp(-0.5 * (rho1 / s1) ** 2) * (1.0 + 0.5j)
    c2 = N(s2) * (-0.4 + 0.9j)
    chord = 2 * math.sqrt(9 * s1 * s1 - rho1 * rho1)
    for sc in (stack([near, far]), stack([far, near])):
        r = oracle.render(sc, Pair(rx, rx, 1e-3), g)
        assert r["S"][1] == pytest.approx(c1 + math.exp(-math.exp(a1) * chord) * c2, rel=1e-9)
        assert r["T_end"][1] == pytest.approx(math.exp(-math.exp(a1) * chord - math.exp(-2.0) * 6 * s2), rel=1e-9)


def test_chord_transmittance_vanishes_at_the_three_sigma_edge():
    g = grid_with(n_az=3, n_el=1, el_lo=-0.5, el_hi=0.5, fle_L=0, transmittance=1)
    v = axis(g)
    s = 0.05
    sc = one(2.0 * v + np.array([0.0, 3 * s * (1 - 1e-10), 0.0]), s, [(1.0, 0.0)], logit=3.0)
    r = oracle.render(sc, Pair(np.zeros(3), np.zeros(3), 1e-3), g)
    assert r["n_active"][1] == 1
    assert 1.0 - r["T_end"][1] < 1e-3


# -------------------------------------------------------- gradients -------
@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "+".join(v))
def test_variant_gradients_match_central_differences(variant):
    b = synth.tiny()
    g = grid_with(n_az=16, n_el=5, fle_L=2, **variant)
    sc = b.scenes[0].subset(slice(0, 300))
    sc = Scene(*(getattr(sc, f).astype(np.float64) for f in ("means", "log_scales", "quats", "logits", "coeffs")))
    p = b.pairs[0]
    G = synth.cotangent((g.n_el * g.n_az,), seed=4).astype(np.float64)
    grads = oracle.vjp(sc, p, g, G)
    base = oracle.render(sc, p, g)

    def loss(s2):
        r = oracle.render(s2, p, g)
        return float((G[:, 0] * r["S"].real + G[:, 1] * r["S"].imag).sum()), r["active_sig"], r["n_active"]

    contrib = set()
    for k in range(0, g.n_el * g.n_az, 3):
        vv, uu = divmod(k, g.n_az)
        sq = oracle.ray_sequence(sc, p, g, uu, vv)
        contrib |= set(sq["order"][sq["active"]].tolist())
    contrib = sorted(contrib)
    rng = np.random.default_rng(12)
    fields = ["means", "log_scales", "quats", "logits", "coeffs"]
    checked = 0
    for trial in range(40):
        gi = int(rng.choice(contrib))
        name = fields[trial % 5]
        arr = getattr(sc, name)
        idx = (gi,) + tuple(int(rng.integers(0, s_)) for s_ in arr.shape[1:])
        h = 1e-6 * max(1.0, abs(float(arr[idx])))
        vals, sigs = [], []
        for sgn in (1, -1):
            a2 = arr.copy()
            a2[idx] += sgn * h
            L, sig, na = loss(Scene(**{**sc.__dict__, name: a2}))
            vals.append(L)
            sigs.append((sig, na))
        if not (np.array_equal(sigs[0][0], sigs[1][0]) and np.array_equal(sigs[0][1], sigs[1][1])
                and np.array_equal(sigs[0][0], base["active_sig"])):
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        ad = float(grads[name][idx])
        scale = max(abs(fd), 1e-3 * np.abs(grads[name]).max())
        assert abs(ad - fd) <= 2e-5 * scale + 1e-7, (name, idx, ad, fd)
        checked += 1
    assert checked >= 25
