"""CPU pins of the oracle's several-correct-results machinery (reading R28)
and of the paper footprint's rule for a radius too large for the grid.

Every GPU parity test excuses a ray whose error exceeds the tolerance only if
``trace`` flags it marginal and one of ``ray_variants``' outcomes matches.  A
slip here would silently widen what counts as matching, so each piece is
pinned on hand-built rays whose decisions sit at a known distance from their
thresholds (App. D.3: the 3-sigma test B^2 - A(C - 9) >= 0 and the midpoint
t >= r_rx; Sec. 3.4: the ray stops once its transmittance is below t_min),
against the single-Gaussian closed form (point-line distance) and the
geometric series of identical Gaussians on one axis.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import Grid, Pair, Scene

BANDS = oracle.Bands()


def one(mu, s, c00, K=1, logit=0.0):
    c = np.zeros((1, K, 2))
    c[0, 0] = c00
    return Scene(np.array([mu], float), np.full((1, 3), math.log(s)), np.array([[1.0, 0, 0, 0]]),
                 np.array([logit], float), c)


def stack(scenes):
    return Scene(*(np.concatenate([getattr(s, f) for s in scenes]) for f in
                   ("means", "log_scales", "quats", "logits", "coeffs")))


def axis_setup():
    """Grid whose ray (u=1, v=0) points exactly along -x (|v| = 1 in FP64)."""
    g = Grid(n_az=3, n_el=1, el_lo=-0.5, el_hi=0.5, fle_L=0, tile_w=16, tile_h=16)
    v = oracle.ray_dirs(g)[0, 1]
    assert v[0] == -1.0 and v[2] == 0.0 and abs(v[1]) < 1e-15
    return g, v


def closed_form(mu, s, c00, rx, tx, f, v):
    """S of one isotropic Gaussian on ray v (T = 1): N e^{-rho^2/2s^2} c00 e^{-j 2 pi d / lambda}."""
    w = np.asarray(mu) - rx
    tpar = float(v @ w)
    rho2 = float(w @ w) - tpar * tpar
    lam = oracle.C0 / f
    N = (2 * math.pi) ** -1.5 / s ** 3
    d = np.linalg.norm(np.asarray(mu) - tx) + tpar
    return N * math.exp(-rho2 / (2 * s * s)) * complex(*c00) * np.exp(-2j * math.pi * d / lam)


def variants_contain(vs, S, scale, rel=1e-12):
    return any(abs(x - S) <= rel * max(scale, 1e-300) for x in vs)


RX = np.zeros(3)
TX = np.array([0.4, -1.3, 0.7])
F = 2.4e9
S_ISO = 0.05
C00 = (0.6, -0.3)


def gaussian_at_q(q, depth=2.0):
    """Isotropic Gaussian beside the axis ray with Mahalanobis^2 q at the chord midpoint."""
    _, v = axis_setup()
    rho = S_ISO * math.sqrt(q)
    return RX + depth * v + np.array([0.0, rho, 0.0])


@pytest.mark.parametrize("dq", [-2e-5, 2e-5])
def test_three_sigma_edge_is_flagged_and_both_branches_enumerated(dq):
    g, v = axis_setup()
    mu = gaussian_at_q(9.0 + dq)
    sc = one(mu, S_ISO, C00)
    r = oracle.render(sc, Pair(RX, TX, F), g)
    ref = closed_form(mu, S_ISO, C00, RX, TX, F, v)
    assert r["marginal"][1]
    # the oracle's own branch is the exact one: a hit iff Q <= 9
    assert (r["n_active"][1] == 1) == (dq < 0)
    vs = oracle.ray_variants(sc, Pair(RX, TX, F), g, 1, 0)
    assert len(vs) == 2 * 3                       # one open decision x three termination thresholds
    assert variants_contain(vs, 0.0, abs(ref))    # not hit
    assert variants_contain(vs, ref, abs(ref), rel=1e-9)    # hit, by the closed form
    assert variants_contain(vs, r["S"][1], abs(ref))


@pytest.mark.parametrize("dt", [-5e-7, 5e-7])
def test_ress_edge_is_flagged_and_both_branches_enumerated(dt):
    g, v = axis_setup()
    r_rx = float(np.float32(g.r_rx))
    mu = RX + (r_rx + dt) * v + np.array([0.0, 0.0, S_ISO])      # Q = 1, midpoint r_rx + dt
    sc = one(mu, S_ISO, C00)
    r = oracle.render(sc, Pair(RX, TX, F), g)
    ref = closed_form(mu, S_ISO, C00, RX, TX, F, v)
    assert r["marginal"][1]
    assert (r["n_active"][1] == 1) == (dt > 0)
    vs = oracle.ray_variants(sc, Pair(RX, TX, F), g, 1, 0)
    assert len(vs) == 6
    assert variants_contain(vs, 0.0, abs(ref))
    assert variants_contain(vs, ref, abs(ref), rel=1e-9)


def test_decisions_outside_the_bands_are_not_flagged():
    g, v = axis_setup()
    cases = [gaussian_at_q(9.0 - 10 * BANDS.q), gaussian_at_q(9.0 + 10 * BANDS.q), gaussian_at_q(4.0),
             RX + (1.0 + 1e-3) * v, RX + (1.0 - 1e-3) * v]
    for mu in cases:
        sc = one(mu, S_ISO, C00)
        r = oracle.render(sc, Pair(RX, TX, F), g)
        assert not r["marginal"].any(), mu
        vs = oracle.ray_variants(sc, Pair(RX, TX, F), g, 1, 0)
        assert len(vs) == 3
        scale = max(r["A_uv"][1], 1e-300)
        assert all(abs(x - r["S"][1]) <= 1e-12 * scale for x in vs)


def _stack_at_termination(rel):
    """Five identical Gaussians on the axis; T before the fifth = t_min (1 + rel)."""
    g, v = axis_setup()
    t_min = float(np.float32(g.t_min))
    keep = (t_min * (1 + rel)) ** 0.25          # (1 - o)^4 = t_min (1 + rel)
    o = 1.0 - keep
    logit = math.log(o / (1 - o))
    sc = stack([one(RX + (2.0 + 0.2 * i) * v, 0.01, (0.8, 0.1), logit=logit) for i in range(5)])
    return g, v, sc, o


@pytest.mark.parametrize("rel", [-1e-5, 1e-5])
def test_termination_edge_enumerates_the_three_thresholds(rel):
    g, v, sc, o = _stack_at_termination(rel)
    r = oracle.render(sc, Pair(RX, RX, F), g)
    assert r["marginal"][1]
    sq = oracle.ray_sequence(sc, Pair(RX, RX, F), g, 1, 0)
    assert sq["T"][4] == pytest.approx(float(np.float32(g.t_min)) * (1 + rel), rel=1e-9)
    # trace takes the fifth Gaussian iff T_5 >= t_min
    assert r["n_active"][1] == (5 if rel > 0 else 4)
    vs = oracle.ray_variants(sc, Pair(RX, RX, F), g, 1, 0)
    assert len(vs) == 3                          # no open hit decision, three thresholds
    ct = sq["ct"]
    T = sq["T"]
    with5 = sum(T[i] * ct[i] for i in range(5))
    with4 = sum(T[i] * ct[i] for i in range(4))
    scale = r["A_uv"][1]
    # low threshold and t_min itself keep or drop the fifth as trace does; the high one drops it
    assert abs(vs[0] - with5) <= 1e-12 * scale
    assert abs(vs[2] - with4) <= 1e-12 * scale
    assert abs(vs[1] - r["S"][1]) <= 1e-12 * scale
    assert abs(with5 - with4) > 1e-6 * scale


def test_clear_termination_is_not_flagged():
    g, v, sc, o = _stack_at_termination(0.05)
    r = oracle.render(sc, Pair(RX, RX, F), g)
    assert not r["marginal"][1]


def test_too_many_open_decisions_return_none():
    g, v = axis_setup()
    n = 9
    sc = stack([one(gaussian_at_q(9.0 - 1e-5, depth=2.0 + 0.3 * i), S_ISO, C00) for i in range(n)])
    vs8 = oracle.ray_variants(sc.subset(slice(0, 8)), Pair(RX, TX, F), g, 1, 0)
    assert vs8 is not None and len(vs8) == 3 * 2 ** 8
    assert oracle.ray_variants(sc, Pair(RX, TX, F), g, 1, 0) is None


def test_flagged_rays_of_a_random_room_contain_trace_result():
    """On a seeded room (2,000 Gaussians, 144 x 36 rays) every flagged ray's
    variant set holds trace's own S, and no clean ray has a variant that differs."""
    g = Grid(n_az=144, n_el=36, fle_L=2)
    b = synth.tiny(grid=g)
    sc, p = b.scenes[0], b.pairs[0]
    r = oracle.render(sc, p, g)
    flagged = np.nonzero(r["marginal"])[0]
    assert 1 <= flagged.size <= 0.03 * r["marginal"].size
    uv = r["rays_uv"]
    spread = []
    for i in flagged:
        vs = oracle.ray_variants(sc, p, g, int(uv[i][0]), int(uv[i][1]))
        assert vs is not None
        assert variants_contain(vs, r["S"][i], r["A_uv"][i])
        spread.append(max(abs(x - r["S"][i]) for x in vs) / r["A_uv"][i])
    assert max(spread) > 1e-4                    # the open decisions change the result
    rng = np.random.default_rng(3)
    for i in rng.choice(np.nonzero(~r["marginal"])[0], 12, replace=False):
        vs = oracle.ray_variants(sc, p, g, int(uv[i][0]), int(uv[i][1]))
        assert all(abs(x - r["S"][i]) <= 1e-12 * max(r["A_uv"][i], 1e-300) for x in vs)


# ----------------------------- paper footprint: radius beyond the grid -----
def test_footprint_radius_beyond_grid_covers_every_column():
    """Sec. 3.3 footprint near the receiver's vertical: the azimuth row of J
    grows as 1/(rho d_alpha), so r_k = 3 sqrt(lambda_max) exceeds the grid;
    the circle's bounding square then covers every column (2m + 1 >= n_az),
    and a radius of 1e9 cells or more is capped at 1e9 without changing the
    square (reading R25')."""
    g = Grid(n_az=360, n_el=90, fle_L=0, tile_w=8, tile_h=8)
    rx = np.array([0.0, 0.0, 0.5])
    s = 0.08
    dalpha = 2 * math.pi / g.n_az
    for rho, huge in ((1e-9, True), (2e-3, False)):
        mu = rx + np.array([rho, 0.0, 2.0])
        r_k = 3 * s / (rho * dalpha)              # isotropic: the azimuth row dominates
        assert (r_k >= 1e9) == huge and 2 * r_k + 1 >= g.n_az
        sc = one(mu, s, (1.0, 0.0))
        tu0, ntu, tv0, ntv, marg = oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, rx, g)
        assert ntu[0] == g.n_tiles_az and tu0[0] == 0
        # rows: v_k +- m clipped -- every row when m reaches past both ends
        assert tv0[0] == 0 and ntv[0] == -(-g.n_el // g.tile_h)
    # a radius just inside the grid does not cover every column
    rho = 3 * s / (0.45 * g.n_az * dalpha)
    sc = one(rx + np.array([rho, 0.0, 2.0]), s, (1.0, 0.0))
    _, ntu, _, _, _ = oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, rx, g)
    assert ntu[0] < g.n_tiles_az
