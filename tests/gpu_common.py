"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI,
read its workspace, and compare with the FP64 oracle under the tolerance and
marginal-decision rules (per ray |S_gpu - S_ref| <= 1e-4 * A_uv, with
A_uv = sum_i T_i |c~_i|; at FP32-marginal decisions any admissible variant)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
import synth
from paper_2502_01826_amd import Problem

TOL = 1e-4        # forward, relative to the condition scale A_uv
GTOL = 1e-3       # gradients, norm-wise per parameter tensor


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def params_of(scene) -> dict:
    return dict(means=scene.means, log_scales=scene.log_scales, quats=scene.quats, logits=scene.logits,
                coeffs=scene.coeffs)


def gpu_problem(batch: synth.Batch, grid=None, cap=None) -> Problem:
    cat, offs = batch.concat()
    return Problem(params_of(cat), batch.pairs, grid or batch.grid, scene_offsets=offs, splat_capacity=cap)


def gpu_forward(prob: Problem):
    sig, ssum, rssi = prob.forward()
    torch.cuda.synchronize()
    S = torch.view_as_complex(sig).cpu().numpy().astype(np.complex128)
    return S, torch.view_as_complex(ssum).cpu().numpy().astype(np.complex128), rssi.cpu().numpy()


def u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def gpu_lists(prob: Problem):
    """Sorted (khi, klo, val), tile ranges and per-record keys read back from the workspace."""
    torch.cuda.synchronize()
    lay = prob.layout()
    cnt = prob.view(lay.counters, torch.int64, 4).cpu().numpy()
    n = int(cnt[0])
    PT = prob.n_pairs * lay.n_tiles
    klo = u32(prob.view(lay.sorted_klo, torch.int32, n))
    val = u32(prob.view(lay.sorted_val, torch.int32, n))
    ts = u32(prob.view(lay.tile_start, torch.int32, PT)).astype(np.int64)
    te = u32(prob.view(lay.tile_end, torch.int32, PT)).astype(np.int64)
    base = prob.view(lay.rec_base, torch.int64, prob.n_pairs + 1).cpu().numpy()
    rkey = u32(prob.view(lay.rec_key, torch.int32, int(lay.n_records)))
    rrect = prob.view(lay.rec_rect, torch.int16, int(lay.n_records) * 4).cpu().numpy().view(np.uint16)
    return dict(n=n, overflow=int(cnt[1]), klo=klo, val=val, ts=ts, te=te, T=lay.n_tiles, base=base,
                rec_key=rkey, rec_rect=rrect.reshape(-1, 4).astype(np.int64))


def lists_from_rects(L: dict, nta: int, gauss_base):
    """Every tile's expected sorted list, built on the host from the records'
    rectangles and keys: each record (pair k, Gaussian j) lands in the tiles of
    its rectangle (columns modulo nta); within a tile the entries are ordered by
    (key, Gaussian index).  Returns (tile of each entry, key, Gaussian index),
    tile-major.  gauss_base[k] is pair k's first Gaussian index."""
    base, T = L["base"], L["T"]
    R = int(base[-1])
    rect = L["rec_rect"][:R]
    cnt = rect[:, 1] * rect[:, 3]
    rec = np.repeat(np.arange(R, dtype=np.int64), cnt)
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(rec.size, dtype=np.int64) - first
    ntu = rect[rec, 1]
    row, col = local // ntu, local % ntu
    pair = np.searchsorted(base, rec, side="right") - 1
    tile = pair * T + (rect[rec, 2] + row) * nta + (rect[rec, 0] + col) % nta
    key = L["rec_key"][rec].astype(np.int64)
    gid = np.asarray(gauss_base, np.int64)[pair] + (rec - base[pair])
    order = np.lexsort((gid, key, tile))
    return tile[order], key[order], gid[order]


def assert_lists_complete(L: dict, nta: int, gauss_base):
    """Every tile list (all tiles of all pairs) equals the host expansion of
    the records' rectangles, entry for entry and in (key, Gaussian) order."""
    tile, key, gid = lists_from_rects(L, nta, gauss_base)
    PT = L["ts"].size
    lens = L["te"] - L["ts"]
    np.testing.assert_array_equal(lens, np.bincount(tile, minlength=PT))
    idx = np.repeat(L["ts"], lens) + (np.arange(int(lens.sum()), dtype=np.int64) -
                                      np.repeat(np.cumsum(lens) - lens, lens))
    np.testing.assert_array_equal(L["klo"][idx].astype(np.int64), key)
    np.testing.assert_array_equal(L["val"][idx].astype(np.int64), gid)
    return lens


def compare_rays(S_gpu, res, scene, pair, grid, tol=TOL, max_marginal_frac=0.03):
    """Per-ray check of GPU values against an oracle ``trace`` result.

    Rays whose error exceeds tol * A_uv must be flagged marginal by the oracle
    and must match one of the oracle's admissible variants.
    """
    S_ref, A = res["S"], res["A_uv"]
    uv = res["rays_uv"]
    err = np.abs(S_gpu - S_ref)
    bad = err > tol * np.maximum(A, 1e-30)
    marg = res["marginal"]
    assert marg.mean() <= max_marginal_frac, f"too many marginal rays: {marg.mean():.4f}"
    unexplained = []
    for i in np.nonzero(bad)[0]:
        if not marg[i]:
            unexplained.append((tuple(uv[i]), S_gpu[i], S_ref[i], A[i]))
            continue
        vs = oracle.ray_variants(scene, pair, grid, int(uv[i][0]), int(uv[i][1]))
        if vs is None:   # more than eight open decisions on one ray: not enumerated, so not excused
            unexplained.append((tuple(uv[i]), S_gpu[i], S_ref[i], A[i]))
            continue
        if not any(abs(S_gpu[i] - v) <= 2 * tol * max(A[i], abs(v), 1e-30) for v in vs):
            unexplained.append((tuple(uv[i]), S_gpu[i], S_ref[i], A[i]))
    assert not unexplained, f"{len(unexplained)} rays off: {unexplained[:5]}"
    ok = ~marg
    num = np.linalg.norm((S_gpu - S_ref)[ok])
    den = np.linalg.norm(S_ref[ok])
    assert num <= tol * max(den, 1e-30), (num, den)
    return dict(max_rel=float((err / np.maximum(A, 1e-30))[ok].max(initial=0.0)), n_bad=int(bad.sum()),
                n_marg=int(marg.sum()))


def oracle_tile_members(scene, pair, grid, tiles):
    """Oracle lists for selected tiles (vectorised rectangle membership)."""
    tu0, ntu, tv0, ntv, marg = oracle.cap_rects(scene.means, scene.log_scales, pair.rx, grid)
    key = oracle.depth_key32(scene.means, pair.rx)
    nta = grid.n_tiles_az
    out = {}
    idx = np.arange(scene.n)
    for t in tiles:
        tv, tu = divmod(int(t), nta)
        inside = (ntu * ntv > 0) & (tv >= tv0) & (tv < tv0 + ntv) & (((tu - tu0) % nta) < ntu)
        g = idx[inside]
        o = np.lexsort((g, key[g]))
        out[int(t)] = (g[o], key[g][o])
    return out, marg
