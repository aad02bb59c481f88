"""GPU parity of the adjoint (a7-a8) against the oracle's FP64 gradients, through the C ABI."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from synth import Batch, Grid, Pair
from gpu_common import GTOL, compare_rays, gpu_forward, gpu_problem, params_of, say
from paper_2502_01826_amd import GSRFRender, Problem

pytestmark = pytest.mark.gpu

NAMES = ["means", "log_scales", "quats", "logits", "coeffs"]


def _gpu_grads(prob, S_sig, G, gsum=None):
    sig = torch.view_as_real(torch.from_numpy(S_sig.astype(np.complex64))).to("cuda").contiguous()
    gt = torch.from_numpy(G.astype(np.float32)).to("cuda").contiguous()
    gs = None if gsum is None else torch.from_numpy(np.asarray(gsum, np.float32)).to("cuda")
    out = prob.render_bwd(sig, gt, gs)
    torch.cuda.synchronize()
    return {n: o.cpu().numpy().astype(np.float64) for n, o in zip(NAMES, out)}


def _compare(gg, gr, tol=GTOL, scale=None):
    """Per tensor: ||g_gpu - g_ref|| <= tol ||g_ref||.  With ``scale`` (the
    oracle's vjp_abs magnitudes) also every entry:
    |g_gpu - g_ref| <= tol * scale + 1e-7 max|g_ref| -- scale is the sum of the
    per-group magnitudes the entry sums, the gradient's analogue of A_uv."""
    for n in NAMES:
        num = np.linalg.norm(gg[n] - gr[n])
        den = np.linalg.norm(gr[n])
        msg = f"  grad {n}: rel {num / max(den, 1e-30):.2e}  |ref| {den:.3e}"
        if scale is not None:
            err = np.abs(gg[n] - gr[n])
            lim = tol * scale[n] + 1e-7 * np.abs(gr[n]).max(initial=0.0)
            worst = float((err / np.maximum(scale[n], 1e-300))[scale[n] > 0].max(initial=0.0))
            bad = np.argwhere(err > lim)
            msg += f"  entrywise max err/scale {worst:.2e} over {int((scale[n] > 0).sum())} entries"
            assert len(bad) == 0, (n, len(bad), [(tuple(i), gg[n][tuple(i)], gr[n][tuple(i)], scale[n][tuple(i)])
                                                 for i in bad[:5]])
        say(msg)
        assert num <= tol * den, n


@pytest.mark.parametrize("tw,th,G", [(16, 16, 1), (8, 8, 4), (16, 8, 2), (8, 8, 0), (16, 8, 0), (16, 16, 0),
                                     (8, 4, 0), (4, 8, 0)])
def test_tiny_gradients_match_oracle(tw, th, G):
    b = synth.tiny(grid=Grid(n_az=36, n_el=9, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=G))
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    prob = gpu_problem(b)
    sig, ssum, _ = prob.forward()
    torch.cuda.synchronize()
    ref = oracle.render(sc, p, g)
    R = g.n_az * g.n_el
    G = synth.cotangent((R,), seed=1).astype(np.float64)
    G[ref["marginal"]] = 0.0            # rays at FP32-marginal decisions carry no cotangent
    gsum = np.array([0.25, -0.4])
    Gr = G.copy()
    Gr[~ref["marginal"]] += gsum[None, :]
    # GPU: per-ray cotangent G plus the S_hat cotangent gsum on every ray; the
    # marginal rays get -gsum so that their total cotangent is zero as well
    Gg = G.copy()
    Gg[ref["marginal"]] = -gsum[None, :]
    gr, scale = oracle.vjp_abs(sc, p, g, Gr)
    gg = _gpu_grads(prob, torch.view_as_complex(sig).cpu().numpy()[0].ravel(), Gg.reshape(1, g.n_el, g.n_az, 2),
                    gsum.reshape(1, 2))
    say("tiny gradients", int(ref["marginal"].sum()), "marginal rays")
    _compare(gg, gr, scale=scale)


@pytest.mark.parametrize("tw,th", [(64, 1), (128, 1)])
def test_single_row_tile_gradients(tw, th):
    """Adjoint after a forward that took the few-tile path with one-row tiles."""
    g = Grid(n_az=290, n_el=5, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=0)
    b = synth.tiny(grid=g, n=1200)
    sc, p = b.scenes[0], b.pairs[0]
    prob = gpu_problem(b)
    sig, _, _ = prob.forward()
    ref = oracle.render(sc, p, g)
    Gc = synth.cotangent((g.n_az * g.n_el,), seed=9).astype(np.float64)
    Gc[ref["marginal"]] = 0.0
    say("single-row tile gradients", tw, th)
    gg = _gpu_grads(prob, torch.view_as_complex(sig).cpu().numpy()[0].ravel(), Gc.reshape(1, g.n_el, g.n_az, 2))
    gr, scale = oracle.vjp_abs(sc, p, g, Gc)
    _compare(gg, gr, scale=scale)


@pytest.mark.parametrize("L,G,th", [(0, 0, 8), (1, 4, 8), (3, 0, 8), (6, 0, 8), (6, 1, 8), (0, 0, 4), (6, 0, 4)])
def test_gradients_across_fle_degrees(L, G, th):
    """Adjoint at every FLE degree the kernels instantiate (K = 1 .. 49)."""
    g = Grid(n_az=24, n_el=8, fle_L=L, tile_w=8, tile_h=th, lanes_per_ray=G)
    rng = np.random.default_rng([101, L])
    sc = synth.draw_scene(rng, 800, (4.0, 4.0, 3.0), g.K)
    p = Pair(np.array([2.0, 2.1, 1.0], np.float32), np.array([0.5, 3.0, 2.0], np.float32), 5.8e9)
    prob = gpu_problem(Batch([sc], [p], g))
    sig, _, _ = prob.forward()
    ref = oracle.render(sc, p, g)
    Gc = synth.cotangent((g.n_az * g.n_el,), seed=5).astype(np.float64)
    Gc[ref["marginal"]] = 0.0
    say("fle degree gradients", L, "lanes", G)
    gg = _gpu_grads(prob, torch.view_as_complex(sig).cpu().numpy()[0].ravel(), Gc.reshape(1, g.n_el, g.n_az, 2))
    gr, scale = oracle.vjp_abs(sc, p, g, Gc)
    _compare(gg, gr, scale=scale)


def test_gradients_against_central_differences():
    """GPU gradients on a 400-Gaussian scene against FP64 central differences of the oracle."""
    b = synth.tiny(n=400)
    g = Grid(n_az=24, n_el=6, fle_L=2, tile_w=8, tile_h=8)
    b = Batch(b.scenes, b.pairs, g)
    sc = b.scenes[0]
    sc = synth.Scene(sc.means, sc.log_scales, sc.quats, sc.logits, np.ascontiguousarray(sc.coeffs[:, :g.K]))
    b = Batch([sc], b.pairs, g)
    p = b.pairs[0]
    prob = gpu_problem(b)
    sig, _, _ = prob.forward()
    base = oracle.render(sc, p, g)
    G = synth.cotangent((g.n_az * g.n_el,), seed=2).astype(np.float64)
    G[base["marginal"]] = 0.0
    gg = _gpu_grads(prob, torch.view_as_complex(sig).cpu().numpy()[0].ravel(), G.reshape(1, g.n_el, g.n_az, 2))
    rng = np.random.default_rng(3)
    contrib = np.unique(np.concatenate([oracle.ray_sequence(sc, p, g, u, v)["order"][
        oracle.ray_sequence(sc, p, g, u, v)["active"]] for v in range(0, g.n_el, 2) for u in range(0, g.n_az, 3)]))
    checked = 0
    sc64 = synth.Scene(*(getattr(sc, f).astype(np.float64) for f in NAMES[:4]), sc.coeffs.astype(np.float64))
    for trial in range(40):
        gi = int(rng.choice(contrib))
        name = NAMES[trial % 5]
        arr = getattr(sc64, name)
        idx = (gi,) + tuple(int(rng.integers(0, s)) for s in arr.shape[1:])
        h = 1e-6 * max(1.0, abs(float(arr[idx])))
        vals, sigs = [], []
        for sgn in (1, -1):
            a2 = arr.copy()
            a2[idx] += sgn * h
            r = oracle.render(synth.Scene(**{**sc64.__dict__, name: a2}), p, g)
            vals.append(float((G[:, 0] * r["S"].real + G[:, 1] * r["S"].imag).sum()))
            sigs.append(r["active_sig"])
        if not (np.array_equal(sigs[0], sigs[1]) and np.array_equal(sigs[0], base["active_sig"])):
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        scale = max(abs(fd), 1e-2 * np.abs(gg[name]).max())
        assert abs(gg[name][idx] - fd) <= GTOL * scale + 1e-6, (name, idx, gg[name][idx], fd)
        checked += 1
    assert checked >= 25


def test_autograd_function_l2_step():
    """torch.autograd through GSRFRender: L2 loss on the spectrum vs a perturbed
    target (rays at FP32-marginal decisions are masked out of the loss)."""
    b = synth.tiny(n=600)
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    target = oracle.render(synth.Scene(sc.means + 0.01, sc.log_scales, sc.quats, sc.logits, sc.coeffs), p, g)
    tgt = torch.tensor(np.stack([target["S"].real, target["S"].imag], -1).reshape(1, g.n_el, g.n_az, 2),
                       dtype=torch.float32, device="cuda")
    ref = oracle.render(sc, p, g)
    ok = ~ref["marginal"]
    mask = torch.tensor(ok.reshape(1, g.n_el, g.n_az, 1), dtype=torch.float32, device="cuda")
    prob = gpu_problem(b)
    ps = [torch.tensor(getattr(sc, n), device="cuda", requires_grad=True) for n in NAMES]
    sig, ssum = GSRFRender.apply(prob, *ps)
    loss = (mask * (sig - tgt) ** 2).sum()
    loss.backward()
    S = torch.view_as_complex(sig.detach()).cpu().numpy()[0].ravel().astype(np.complex128)
    Gr = 2 * np.stack([S.real - target["S"].real, S.imag - target["S"].imag], -1) * ok[:, None]
    gr, scale = oracle.vjp_abs(sc, p, g, Gr)
    _compare({n: t.grad.cpu().numpy().astype(np.float64) for n, t in zip(NAMES, ps)}, gr, tol=2e-3, scale=scale)


@pytest.mark.parametrize("tw,th,G", [(16, 16, 1), (8, 8, 4), (8, 8, 0), (16, 16, 0), (8, 4, 0)])
def test_paper_scale_gradients_on_sampled_rays(tw, th, G):
    """200k Gaussians, 360x90: cotangent on 48 sampled rays only, compared with
    the oracle's gradient of the same rays."""
    b = synth.paper_scale(grid=Grid(n_az=360, n_el=90, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=G))
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    prob = gpu_problem(b)
    sig, _, _ = prob.forward()
    rng = np.random.default_rng(9)
    uv = np.stack([rng.integers(0, g.n_az, 48), rng.integers(0, g.n_el, 48)], 1)
    uv = np.unique(uv, axis=0)
    ref = oracle.trace(sc, p, g, uv)
    keep = ~ref["marginal"]
    uv = uv[keep]
    Gs = synth.cotangent((len(uv),), seed=4).astype(np.float64)
    G = np.zeros((1, g.n_el, g.n_az, 2))
    G[0, uv[:, 1], uv[:, 0]] = Gs
    say("paper-scale gradients on", len(uv), "rays")
    gg = _gpu_grads(prob, torch.view_as_complex(sig).cpu().numpy()[0].ravel(), G)
    gr, scale = oracle.vjp_abs(sc, p, g, Gs, rays_uv=uv)
    _compare(gg, gr, scale=scale)


def test_many_tile_launch_gradients_match_oracle():
    """10 pairs x 540 tiles: the forward renders each tile with one workgroup
    and the adjoint stages full batches (the launch shape of large batches);
    cotangent on 16 sampled rays per pair, gradients summed over the pairs."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    b = synth.batched(n=20_000, n_pairs=10, grid=g)
    sc = b.scenes[0]
    prob = gpu_problem(b)
    assert len(b.pairs) * g.n_tiles > 2048
    sig, _, _ = prob.forward()
    S = torch.view_as_complex(sig).cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(21)
    G = np.zeros((len(b.pairs), g.n_el, g.n_az, 2))
    ref = scale = None
    for k, p in enumerate(b.pairs):
        uv = np.unique(np.stack([rng.integers(0, g.n_az, 16), rng.integers(0, g.n_el, 16)], 1), axis=0)
        tr = oracle.trace(sc, p, g, uv)
        compare_rays(S[k][uv[:, 1], uv[:, 0]], tr, sc, p, g, max_marginal_frac=0.25)   # 16-ray sample
        uv = uv[~tr["marginal"]]
        Gs = synth.cotangent((len(uv),), seed=40 + k).astype(np.float64)
        G[k, uv[:, 1], uv[:, 0]] = Gs
        r, rs = oracle.vjp_abs(sc, p, g, Gs, rays_uv=uv)
        ref = r if ref is None else {n: ref[n] + r[n] for n in NAMES}
        scale = rs if scale is None else {n: scale[n] + rs[n] for n in NAMES}
    say("many-tile launch: 10 pairs x 540 tiles")
    gt = torch.from_numpy(G.astype(np.float32)).cuda()
    out = prob.render_bwd(sig, gt)
    torch.cuda.synchronize()
    _compare({n: o.cpu().numpy().astype(np.float64) for n, o in zip(NAMES, out)}, ref, scale=scale)


@pytest.mark.parametrize("tw,th,G", [(8, 8, 0), (16, 8, 0), (8, 8, 4)])
def test_paper_footprint_gradients_match_oracle(tw, th, G):
    """The adjoint over the paper-footprint binning (grid.footprint = 1) against
    the oracle's gradients of the render restricted to the same tiles."""
    g = Grid(n_az=36, n_el=9, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=G, footprint=1)
    b = synth.tiny(grid=g)
    sc, p = b.scenes[0], b.pairs[0]
    say("footprint gradients", tw, th, "lanes", G)
    rects = oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, p.rx, g)
    assert not rects[4].any()
    prob = gpu_problem(b)
    sig, _, _ = prob.forward()
    torch.cuda.synchronize()
    ref = oracle.render(sc, p, g, rects=rects)
    R = g.n_az * g.n_el
    G = synth.cotangent((R,), seed=2).astype(np.float64)
    G[ref["marginal"]] = 0.0
    gr, scale = oracle.vjp_abs(sc, p, g, G, rects=rects)
    gg = _gpu_grads(prob, torch.view_as_complex(sig).cpu().numpy()[0].ravel(), G.reshape(1, g.n_el, g.n_az, 2))
    _compare(gg, gr, scale=scale)


GOLD_FD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_scale_fd.json")


def test_paper_scale_gradients_full_cotangent_and_central_differences():
    """The differentiated step at full size (200k Gaussians, 360x90 rays, 5 GHz,
    8x8 tiles, two-phase traversal: the launch the benchmark times) with a
    cotangent on every ray the oracle does not flag as marginal.  For 500
    seeded Gaussians that contribute: every attribute's gradient entry by entry
    against the oracle's (within 1e-3 of its vjp_abs scale), and its
    directional derivative along a seeded direction against the oracle's FP64
    central difference; per attribute, the full gradient's norm against the
    oracle's.  Reference values: tests/golden/make_paper_scale_fd.py (oracle
    only)."""
    with open(GOLD_FD) as fh:
        d = json.load(fh)
    gd = d["grid"]
    g = Grid(n_az=gd["n_az"], n_el=gd["n_el"], fle_L=gd["fle_L"], tile_w=gd["tile_w"], tile_h=gd["tile_h"],
             lanes_per_ray=0)
    b = synth.paper_scale(grid=g)
    say("paper scale, full cotangent:", len(d["gaussians"]), "Gaussians with stored differences")
    prob = gpu_problem(b)
    sig, _, _ = prob.forward()
    G = synth.cotangent((g.n_az * g.n_el,), seed=d["cotangent_seed"]).astype(np.float64)
    G[np.asarray(d["marginal_rays"], dtype=np.int64)] = 0.0
    gg = _gpu_grads(prob, torch.view_as_complex(sig).cpu().numpy()[0].ravel(), G.reshape(1, g.n_el, g.n_az, 2))
    for n in NAMES:
        ref = d["grad_norm"][n]
        got = float(np.linalg.norm(gg[n]))
        say(f"  |grad {n}|: gpu {got:.6e} oracle {ref:.6e}")
        assert abs(got - ref) <= GTOL * ref, n
    n_fd = n_ent = 0
    worst = {n: 0.0 for n in NAMES}
    for rec in d["gaussians"]:
        i = rec["index"]
        for n in NAMES:
            e = rec[n]
            gi = gg[n][i].reshape(-1)
            gr, sc = np.asarray(e["grad"]), np.asarray(e["scale"])
            floor = 1e-7 * d["grad_norm"][n]
            err = np.abs(gi - gr)
            assert np.all(err <= GTOL * sc + floor), (i, n, gi, gr, sc)
            worst[n] = max(worst[n], float((err / np.maximum(sc, 1e-300)).max()))
            n_ent += gi.size
            if e["fd"] is not None:
                v = np.asarray(e["v"])
                lim = GTOL * float(np.abs(v) @ sc) + floor
                assert abs(float(gi @ v) - e["fd"]) <= lim, (i, n, float(gi @ v), e["fd"], lim)
                n_fd += 1
    say("  entries", n_ent, "worst err/scale", {n: f"{w:.1e}" for n, w in worst.items()}, "differences", n_fd)
    assert n_fd >= 0.9 * len(NAMES) * len(d["gaussians"])


def _multi_reference(sc, pairs_scene, g, n_freq, step, Gm, gsum_m, ray_chunk=8):
    """sum over carriers of the oracle's gradient at each carrier's frequency,
    with the summed vjp_abs scale."""
    ref = scale = None
    for k, p in pairs_scene:
        for c in range(n_freq):
            pc = Pair(p.rx, p.tx, p.freq_hz + c * step)
            gs = None if gsum_m is None else gsum_m[k, c]
            r, s = oracle.vjp_abs(sc, pc, g, Gm[k, c].reshape(-1, 2), g_sum=gs, ray_chunk=ray_chunk)
            ref = r if ref is None else {n: ref[n] + r[n] for n in NAMES}
            scale = s if scale is None else {n: scale[n] + s[n] for n in NAMES}
    return ref, scale


@pytest.mark.parametrize("n_freq,step,tw,th", [(20, 10e6, 8, 8), (5, 312.5e3, 16, 8), (1, 0.0, 8, 4)])
def test_multi_carrier_gradients_match_oracle_sum(n_freq, step, tw, th):
    """gsrf_render_bwd_multi against the sum over carriers of the oracle's
    gradient at each carrier frequency (20 carriers: two chunks of 16 and 4,
    10 MHz apart so that the phases differ by whole turns across the room; an
    OFDM block's 312.5 kHz spacing; one carrier), per tensor and per entry,
    with dL/dS_hat per carrier."""
    g = Grid(n_az=24, n_el=8, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=0)
    rng = np.random.default_rng([103, n_freq])
    sc = synth.draw_scene(rng, 800, (4.0, 4.0, 3.0), g.K)
    p = Pair(np.array([2.0, 2.1, 1.0], np.float32), np.array([0.5, 3.0, 2.0], np.float32), 2.4e9)
    prob = gpu_problem(Batch([sc], [p], g))
    prob.forward()
    torch.cuda.synchronize()
    marg = oracle.render(sc, p, g)["marginal"]        # hit decisions do not depend on the carrier
    R = g.n_az * g.n_el
    Gm = synth.cotangent((1, n_freq, R), seed=31).astype(np.float64)
    Gm[:, :, marg] = 0.0
    gsum = synth.cotangent((1, n_freq), seed=32).astype(np.float64) * 0.1
    Gdev = Gm.copy()
    Gdev[:, :, marg] = -gsum[:, :, None, :]           # marginal rays: total cotangent zero as well
    Gref = Gm.copy()
    Gref[:, :, ~marg] += gsum[:, :, None, :]
    say("multi-carrier gradients:", n_freq, "carriers", step, "Hz apart, tile", tw, th, int(marg.sum()), "marginal")
    out = prob.render_bwd_multi(n_freq, step, torch.from_numpy(Gdev.reshape(1, n_freq, g.n_el, g.n_az, 2)
                                                               .astype(np.float32)).cuda().contiguous(),
                                torch.from_numpy(gsum.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    gg = {n: o.cpu().numpy().astype(np.float64) for n, o in zip(NAMES, out)}
    ref, scale = _multi_reference(sc, [(0, p)], g, n_freq, step, Gref, None)
    _compare(gg, ref, scale=scale)


def test_multi_carrier_adjoint_of_one_carrier_equals_the_adjoint():
    """One carrier through gsrf_render_bwd_multi and gsrf_render_bwd on the
    same forward: the same gradient to rounding (entry by entry)."""
    b = synth.tiny(n=1200)
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    prob = gpu_problem(b)
    sig, _, _ = prob.forward()
    G = torch.from_numpy(synth.cotangent((1, g.n_el, g.n_az), seed=41)).cuda()
    one = prob.render_bwd(sig, G, None)
    multi = prob.render_bwd_multi(1, 0.0, G.reshape(1, 1, g.n_el, g.n_az, 2).contiguous())
    torch.cuda.synchronize()
    for n, a, m in zip(NAMES, one, multi):
        a, m = a.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(a - m) <= 1e-5 * np.abs(a).max() + 1e-6 * np.abs(a)), n


def test_multi_carrier_gradients_in_a_multi_scene_batch():
    """Three scenes, two pairs each at 2.4 / 5 / 5.8 GHz, 4 carriers 1 MHz
    apart; cotangent on 12 sampled rays per pair and carrier."""
    g = Grid(n_az=36, n_el=9, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    rng = np.random.default_rng(77)
    scenes = [synth.draw_scene(rng, n, (4.0, 4.0, 3.0), g.K) for n in (900, 1500, 400)]
    pairs = []
    for s, f in zip(range(3), (2.4e9, 5.0e9, 5.8e9)):
        for _ in range(2):
            pairs.append(Pair(rng.uniform([0.5, 0.5, 0.3], [3.5, 3.5, 2.7]).astype(np.float32),
                              rng.uniform([0.5, 0.5, 0.3], [3.5, 3.5, 2.7]).astype(np.float32), f, scene=s))
    b = Batch(scenes, pairs, g)
    prob = gpu_problem(b)
    prob.forward()
    torch.cuda.synchronize()
    n_freq, step, P, R = 4, 1e6, len(pairs), g.n_az * g.n_el
    Gm = np.zeros((P, n_freq, R, 2))
    for k, pr in enumerate(pairs):
        marg = oracle.render(scenes[pr.scene], pr, g)["marginal"]
        pick = rng.choice(np.nonzero(~marg)[0], size=12, replace=False)
        Gm[k][:, pick] = synth.cotangent((n_freq, 12), seed=50 + k)
    say("multi-carrier gradients, 3 scenes x 2 pairs, 4 carriers")
    out = prob.render_bwd_multi(n_freq, step, torch.from_numpy(Gm.reshape(P, n_freq, g.n_el, g.n_az, 2)
                                                               .astype(np.float32)).cuda().contiguous())
    torch.cuda.synchronize()
    gg = {n: o.cpu().numpy().astype(np.float64) for n, o in zip(NAMES, out)}
    cat, offs = b.concat()
    for s, sc in enumerate(scenes):
        lo, hi = offs[s], offs[s + 1]
        ref, scale = _multi_reference(sc, [(k, pr) for k, pr in enumerate(pairs) if pr.scene == s], g, n_freq, step,
                                      Gm, None)
        _compare({n: gg[n][lo:hi] for n in NAMES}, ref, scale=scale)


@pytest.mark.parametrize("tw,th", [(8, 8), (16, 8)])
def test_workspace_contents_do_not_matter(tw, th):
    """The workspace filled with 0xFF bytes before the step gives the same
    signal (bit for bit) and gradients (to the rounding of the accumulators'
    atomic adds, whose order varies from run to run) as a zeroed one.  At paper
    scale the forward stops most tiles once all their rays have terminated,
    leaving the rest of the list's hit masks unwritten; the adjoints (one
    carrier and several) must not read them."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=0)
    b = synth.paper_scale(grid=g)
    prob = gpu_problem(b)
    P = 1
    G = torch.from_numpy(synth.cotangent((P, g.n_el, g.n_az), seed=51)).cuda()
    Gm = torch.from_numpy(synth.cotangent((P, 3, g.n_el, g.n_az), seed=52)).cuda()
    runs = []
    for fill in (0, 255):
        prob.ws.fill_(fill)
        sig, ssum, _ = prob.forward()
        one = prob.render_bwd(sig, G, None)
        multi = prob.render_bwd_multi(3, 312.5e3, Gm)
        torch.cuda.synchronize()
        runs.append([t.clone() for t in (sig, ssum, *one, *multi)])
    say("workspace fill: 0 and 0xFF, tile", tw, th)
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    for a, c in zip(runs[0][2:], runs[1][2:]):
        a, c = a.cpu().numpy().astype(np.float64), c.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(a - c) <= 1e-5 * np.abs(a).max() + 1e-5 * np.abs(a))
