"""Batched execution: uneven multi-scene batches against the oracle (forward and
gradients), hipGraph replays against eager launches, and the tile autotuner."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth import Batch, Grid
from gpu_common import GTOL, compare_rays, gpu_problem, say
from paper_2502_01826_amd import Problem
from paper_2502_01826_amd.batch import GraphStep, autotune

pytestmark = pytest.mark.gpu

NAMES = ["means", "log_scales", "quats", "logits", "coeffs"]


def _uneven(grid, seed=0):
    """Three scenes of uneven size, two to four pairs each, carriers 2.4/5/5.8 GHz."""
    rng = np.random.default_rng([55, seed])
    room = (6.0, 5.0, 3.0)
    scenes, pairs = [], []
    for s, (n, m) in enumerate([(3000, 2), (12000, 4), (700, 3)]):
        scenes.append(synth.draw_scene(rng, n, room, grid.K))
        for _ in range(m):
            pairs.append(synth.draw_pair(rng, room, float(rng.choice([2.4e9, 5.0e9, 5.8e9])), scene=s))
    return Batch(scenes, pairs, grid)


def _params(b):
    cat, offs = b.concat()
    return dict(means=cat.means, log_scales=cat.log_scales, quats=cat.quats, logits=cat.logits,
                coeffs=cat.coeffs), offs


def test_uneven_batch_forward_and_gradients_match_oracle():
    g = Grid(n_az=60, n_el=16, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    b = _uneven(g)
    prm, offs = _params(b)
    P = len(b.pairs)
    say("uneven batch: scenes 3000/12000/700, pairs", P)
    prob = Problem(prm, b.pairs, g, scene_offsets=offs)
    sig, ssum, rssi = prob.forward()
    S = torch.view_as_complex(sig).cpu().numpy().astype(np.complex128)
    # cotangent on 24 sampled non-marginal rays of every pair
    rng = np.random.default_rng(8)
    Gt = np.zeros((P, g.n_el, g.n_az, 2))
    per_pair = []
    for k, pr in enumerate(b.pairs):
        sc = b.scenes[pr.scene]
        ref = oracle.render(sc, pr, g)
        compare_rays(S[k].ravel(), ref, sc, pr, g)
        ok = np.nonzero(~ref["marginal"])[0]
        pick = rng.choice(ok, size=24, replace=False)
        uv = np.stack([pick % g.n_az, pick // g.n_az], 1)
        Gs = synth.cotangent((len(uv),), seed=20 + k).astype(np.float64)
        Gt[k, uv[:, 1], uv[:, 0]] = Gs
        per_pair.append((uv, Gs))
    gt = torch.from_numpy(Gt.astype(np.float32)).cuda()
    out = prob.render_bwd(sig, gt)
    torch.cuda.synchronize()
    gg = {n: o.cpu().numpy().astype(np.float64) for n, o in zip(NAMES, out)}
    for s, sc in enumerate(b.scenes):
        lo, hi = offs[s], offs[s + 1]
        ref = scale = None
        for k, pr in enumerate(b.pairs):
            if pr.scene != s:
                continue
            uv, Gs = per_pair[k]
            r, rs = oracle.vjp_abs(sc, pr, g, Gs, rays_uv=uv)
            ref = r if ref is None else {n: ref[n] + r[n] for n in NAMES}
            scale = rs if scale is None else {n: scale[n] + rs[n] for n in NAMES}
        for n in NAMES:
            num = np.linalg.norm(gg[n][lo:hi] - ref[n])
            den = np.linalg.norm(ref[n])
            say(f"  scene {s} grad {n}: rel {num / max(den, 1e-30):.2e}")
            assert num <= GTOL * den, (s, n)
            # every entry against its summed per-group magnitude (vjp_abs)
            err = np.abs(gg[n][lo:hi] - ref[n])
            assert np.all(err <= GTOL * scale[n] + 1e-7 * np.abs(ref[n]).max(initial=0.0)), (s, n)


def test_graph_replays_match_eager():
    """Every replay of the captured project/bin_sort/render_fwd/render_bwd
    sequence equals the eager launches, with eager work between replays."""
    g = Grid(n_az=60, n_el=16, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    b = _uneven(g, seed=1)
    prm, offs = _params(b)
    P = len(b.pairs)
    gt = torch.from_numpy(synth.cotangent((P, g.n_el, g.n_az), seed=31)).cuda()
    gs = torch.from_numpy(synth.cotangent((P,), seed=32)).cuda()
    eager = Problem(prm, b.pairs, g, scene_offsets=offs)
    sig_e, ssum_e, rssi_e = eager.forward()
    grads_e = eager.render_bwd(sig_e, gt, gs)
    torch.cuda.synchronize()
    step = GraphStep(Problem(prm, b.pairs, g, scene_offsets=offs), grad=True, grad_signal=gt, grad_sum=gs)
    for rep in range(3):
        say("graph replay", rep)
        junk = torch.randn(1 << 20, device="cuda")       # unrelated eager work between replays
        step.replay()
        junk.mul_(2.0)
        torch.cuda.synchronize()
        assert torch.equal(step.signal, sig_e) and torch.equal(step.signal_sum, ssum_e)
        assert torch.equal(step.rssi, rssi_e)
        for n, a, e in zip(NAMES, step.grads, grads_e):
            num = torch.linalg.norm((a - e).double()).item()
            den = torch.linalg.norm(e.double()).item()
            assert num <= 1e-5 * max(den, 1e-30), (rep, n, num, den)


def test_autotune_returns_a_timed_candidate():
    g = Grid(n_az=72, n_el=18, fle_L=2, lanes_per_ray=0)
    b = synth.tiny(n=3000, grid=g)
    sc, pr = b.scenes[0], b.pairs[0]
    prm = dict(means=sc.means, log_scales=sc.log_scales, quats=sc.quats, logits=sc.logits, coeffs=sc.coeffs)
    cands = ((8, 8, 0), (16, 16, 0))
    res = autotune(lambda gg: Problem(prm, [pr], gg), g, candidates=cands, iters=2)
    say("autotune", res.seconds)
    assert res.best in cands and set(res.seconds) == set(cands)
    assert all(v > 0 for v in res.seconds.values())
    tw, th, lanes = res.best
    g2 = Grid(n_az=72, n_el=18, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=lanes)
    S = torch.view_as_complex(Problem(prm, [pr], g2).forward()[0]).cpu().numpy().astype(np.complex128)
    compare_rays(S[0].ravel(), oracle.render(sc, pr, g2), sc, pr, g2)


def test_uneven_batch_footprint_binning_matches_oracle():
    """Paper-footprint binning (grid.footprint = 1) over three scenes of uneven
    size and nine pairs: every record's rectangle per pair, and sampled rays of
    every pair against the oracle render restricted to the same tiles."""
    from gpu_common import TOL, gpu_lists
    g = Grid(n_az=72, n_el=18, fle_L=2, tile_w=8, tile_h=8, footprint=1)
    b = _uneven(g, seed=3)
    say("uneven batch, paper footprint:", len(b.scenes), "scenes,", len(b.pairs), "pairs")
    prob = gpu_problem(b)
    sig, _, _ = prob.forward()
    torch.cuda.synchronize()
    S = torch.view_as_complex(sig).cpu().numpy().astype(np.complex128)
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    rng = np.random.default_rng(9)
    for k, p in enumerate(b.pairs):
        sc = b.scenes[p.scene]
        rects = oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, p.rx, g)
        marg = rects[4]
        got = L["rec_rect"][L["base"][k]:L["base"][k] + sc.n]
        np.testing.assert_array_equal(got[~marg], np.stack(rects[:4], 1)[~marg])
        uv = np.stack([rng.integers(0, g.n_az, 24), rng.integers(0, g.n_el, 24)], 1)
        ref = oracle.trace(sc, p, g, uv, rects=rects)
        ok = ~ref["marginal"]
        if marg.any():
            ok &= ~oracle.rect_allow(rects, g, uv)[:, marg].any(1)
        err = np.abs(S[k][uv[:, 1], uv[:, 0]] - ref["S"])
        assert np.all(err[ok] <= TOL * np.maximum(ref["A_uv"][ok], 1e-30)), (k, float(err[ok].max()))
