"""Writes paper_scale_fd.json: FP64 oracle gradients and central differences of
the differentiated step at the paper's scale (200k Gaussians in a 10 x 8 x 3 m
room, one TX/RX pair, 360 x 90 rays at 1 degree, 5 GHz, FLE L = 2), for 500
seeded Gaussians that contribute to the received signal.  Calls only the
oracle and the seeded input generator; nothing here comes from the GPU path.

    python tests/golden/make_paper_scale_fd.py [--gaussians 500]

The functional is L = sum_r Re(conj(G_r) S_r) (App. D: the gradient of any
loss reaches the render through such a cotangent G = dL/dRe S + j dL/dIm S),
with G a seeded CN(0, 1) draw on every ray and zero on the rays where the
oracle flags an FP32-marginal decision (several results are correct there).
Stored per sampled Gaussian and attribute (mean, log-scale, quaternion,
opacity logit, coefficients): the oracle's gradient, its per-entry scale
(``oracle.vjp_abs`` over groups of 64 rays), a seeded unit direction v in that
attribute's space and the FP64 central difference (L(theta + h v) -
L(theta - h v)) / 2h over the rays of its binning cap that it hits (no other
ray changes with it), rendered against every Gaussian whose cap covers one of
those rays' tiles (the cap is conservative, so those rays see exactly the
full scene); differences whose
+-h renders change any hit or termination decision, or the Gaussian's place
in the depth order, are dropped.  Also
stored: the marginal rays and the full gradient's norm per attribute.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from synth import Grid  # noqa: E402

NAMES = ["means", "log_scales", "quats", "logits", "coeffs"]
COTANGENT_SEED = 31
PICK_SEED = 33
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_scale_fd.json")


def grid():
    return Grid(n_az=360, n_el=90, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gaussians", type=int, default=500)
    args = ap.parse_args()
    t0 = time.time()
    b = synth.paper_scale(grid=grid())
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    R = g.n_az * g.n_el
    sc64 = synth.Scene(*(getattr(sc, f).astype(np.float64) for f in NAMES))
    base = oracle.render(sc, p, g)
    marg = np.nonzero(base["marginal"])[0]
    print(f"oracle render: {time.time() - t0:.0f}s, {len(marg)} marginal rays", flush=True)
    G = synth.cotangent((R,), seed=COTANGENT_SEED).astype(np.float64)
    G[marg] = 0.0
    grads, scales = oracle.vjp_abs(sc, p, g, G, ray_chunk=64)
    print(f"oracle gradient: {time.time() - t0:.0f}s", flush=True)
    contrib = np.nonzero(np.any(np.abs(grads["coeffs"].reshape(sc.n, -1)) > 0, axis=1))[0]
    rng = np.random.default_rng(PICK_SEED)
    pick = np.sort(rng.choice(contrib, size=min(args.gaussians, len(contrib)), replace=False))

    tu0, ntu, tv0, ntv, _ = oracle.cap_rects(sc.means, sc.log_scales, p.rx, g)
    nta, tw, th = g.n_tiles_az, g.tile_w, g.tile_h
    Gr = G.reshape(g.n_el, g.n_az, 2)
    out = []
    for n_done, i in enumerate(pick):
        # rays of Gaussian i's rectangle that i itself hits (i alone: every hit
        # is active); only these change when i's parameters move
        tus = (tu0[i] + np.arange(ntu[i])) % nta
        tvs = tv0[i] + np.arange(ntv[i])
        us = np.concatenate([np.arange(t * tw, min((t + 1) * tw, g.n_az)) for t in tus])
        vs = np.concatenate([np.arange(t * th, min((t + 1) * th, g.n_el)) for t in tvs])
        uu, vv = np.meshgrid(us, vs)
        uv = np.stack([uu.ravel(), vv.ravel()], 1)
        alone = oracle.trace(sc64.subset(np.array([i])), p, g, uv)
        uv = uv[alone["n_active"] > 0]
        Gs = Gr[uv[:, 1], uv[:, 0]]
        # Gaussians whose rectangle holds a tile of those rays (index order kept)
        hit_tiles = np.unique((uv[:, 1] // th) * nta + uv[:, 0] // tw)
        near_m = np.zeros(sc.n, bool)
        for t in hit_tiles:
            tv, tu = divmod(int(t), nta)
            near_m |= (ntu * ntv > 0) & (tv >= tv0) & (tv < tv0 + ntv) & (((tu - tu0) % nta) < ntu)
        near = np.nonzero(near_m)[0]
        sub = sc64.subset(near)
        j = int(np.searchsorted(near, i))
        assert near[j] == i
        ref_sig = oracle.trace(sub, p, g, uv)["active_sig"]
        rank0 = int(np.nonzero(oracle.depth_order(sub.means, p.rx) == j)[0][0])
        rec = dict(index=int(i), n_rays=int(len(uv)), n_near=int(len(near)))
        for a, nm in enumerate(NAMES):
            arr = getattr(sub, nm)
            theta = arr[j].reshape(-1)
            v = np.random.default_rng([PICK_SEED, int(i), a]).normal(size=theta.shape)
            v /= np.linalg.norm(v)
            h = 1e-6 * max(1.0, float(np.linalg.norm(theta)))
            vals, sigs, ranks = [], [], []
            for sgn in (1, -1):
                a2 = arr.copy()
                a2[j] = (theta + sgn * h * v).reshape(arr[j].shape)
                r = oracle.trace(synth.Scene(**{**sub.__dict__, nm: a2}), p, g, uv)
                vals.append(float((Gs[:, 0] * r["S"].real + Gs[:, 1] * r["S"].imag).sum()))
                sigs.append(r["active_sig"])
                if nm == "means":   # the depth order: i's place among the (key, index) pairs
                    ranks.append(int(np.nonzero(oracle.depth_order(a2, p.rx) == j)[0][0]))
            ok = bool(np.array_equal(sigs[0], ref_sig) and np.array_equal(sigs[1], ref_sig))
            if nm == "means":
                ok = ok and ranks[0] == ranks[1] == rank0
            rec[nm] = dict(v=v.tolist(), fd=(vals[0] - vals[1]) / (2 * h) if ok else None,
                           grad=grads[nm][i].reshape(-1).tolist(), scale=scales[nm][i].reshape(-1).tolist())
        out.append(rec)
        if n_done % 25 == 0:
            print(f"  {n_done}/{len(pick)} Gaussians, {time.time() - t0:.0f}s ({len(uv)} rays, "
                  f"{len(near)} Gaussians near)", flush=True)
    doc = dict(
        what="oracle gradients and central differences, 200k Gaussians, 360x90 rays, 5 GHz, one pair",
        source="tests/golden/make_paper_scale_fd.py (FP64 oracle only)",
        passage="App. D (gradients of the rendering); Sec. 3.4 (rendering); App. A (discretized rendering)",
        grid=dict(n_az=g.n_az, n_el=g.n_el, fle_L=g.fle_L, tile_w=g.tile_w, tile_h=g.tile_h),
        cotangent_seed=COTANGENT_SEED, pick_seed=PICK_SEED, marginal_rays=marg.tolist(),
        grad_norm={nm: float(np.linalg.norm(grads[nm])) for nm in NAMES},
        n_contributing=int(len(contrib)), gaussians=out)
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1024:.0f} KiB) in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
