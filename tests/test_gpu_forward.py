"""GPU parity of the forward path (a1-a6) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from synth import Batch, Grid, Pair, Scene
from gpu_common import (TOL, assert_lists_complete, compare_rays, gpu_forward, gpu_lists, gpu_problem,
                        oracle_tile_members, params_of, say)

pytestmark = pytest.mark.gpu


def _scene_f32(s):
    return Scene(*(np.ascontiguousarray(getattr(s, f), dtype=np.float32)
                   for f in ("means", "log_scales", "quats", "logits", "coeffs")))


def test_tiny_forward_matches_oracle_and_lists_are_bit_exact():
    b = synth.tiny()
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    say("tiny: 2000 gaussians, 36x9 rays, tiles", g.tile_w, g.tile_h)
    prob = gpu_problem(b)
    S, Ssum, rssi = gpu_forward(prob)
    ref = oracle.render(sc, p, g)
    st = compare_rays(S[0].ravel(), ref, sc, p, g)
    say("tiny forward", st)
    A = ref["A_uv"]
    assert abs(Ssum[0] - ref["S_sum"]) <= TOL * A.sum() + np.abs(S[0].ravel() - ref["S"])[ref["marginal"]].sum()
    assert rssi[0] == pytest.approx(oracle.rssi_dbm(ref["S_sum"]), abs=1e-3)
    # depth keys of every record and the tile lists, bit for bit
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    np.testing.assert_array_equal(L["rec_key"], oracle.depth_key32(sc.means, p.rx).astype(np.uint32))
    tu0, ntu, tv0, ntv, marg = oracle.cap_rects(sc.means, sc.log_scales, p.rx, g)
    np.testing.assert_array_equal(L["rec_rect"][~marg], np.stack([tu0, ntu, tv0, ntv], 1)[~marg])
    lists, keys, _ = oracle.tile_lists(sc.means, sc.log_scales, p.rx, g)
    assert L["n"] == sum(len(x) for x in lists)
    assert L["ts"][0] == 0 and np.all(L["ts"][1:] == L["te"][:-1]) and L["te"][-1] == L["n"]
    for t in range(L["T"]):
        a, e = L["ts"][t], L["te"][t]
        np.testing.assert_array_equal(L["val"][a:e], lists[t].astype(np.uint32))
        np.testing.assert_array_equal(L["klo"][a:e], keys[t].astype(np.uint32))


@pytest.mark.parametrize("tw,th,G", [(8, 8, 0), (8, 4, 0), (16, 8, 2)])
def test_render_stats_counts_match_oracle(tw, th, G):
    """The traversal counters: rays and processed hits against the oracle (hits
    of rays with a marginal decision may differ by the flipped decisions), and
    the orderings every traversal obeys."""
    g = Grid(n_az=37, n_el=11, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=G)
    b = synth.tiny(grid=g, n=1500)
    sc, p = b.scenes[0], b.pairs[0]
    say("render_stats", tw, th, "lanes", G)
    prob = gpu_problem(b)
    prob.forward()
    st = prob.render_stats()
    torch.cuda.synchronize()
    ref = oracle.render(sc, p, g)
    say("  counts", st)
    assert st["rays"] == g.n_az * g.n_el
    n_act = ref["n_active"].astype(np.int64)
    # a flipped hit or termination decision moves a marginal ray's count by one
    slack = 8 * int(ref["marginal"].sum())
    assert abs(st["hits"] - int(n_act.sum())) <= slack
    assert st["hits"] <= st["tests"] <= st["tile_tests"]
    assert st["staged"] > 0
    if G == 0:
        assert st["walk_slots"] % 64 == 0 and st["hits"] <= st["walk_slots"]
    else:
        assert st["walk_slots"] == 0


@pytest.mark.parametrize("n_pairs", [1, 12])
def test_capacity_overflow_renders_nothing_then_recovers(n_pairs):
    """A splat capacity below the count: gsrf_splat_count reports it, bin_sort
    emits nothing and every tile range is empty (zero signal, overflow flag
    set); with the capacity grown the same problem matches the oracle.  One
    pair of 36x9 rays takes the one-launch tile scan; 12 pairs of 360x90 rays
    (6480 tiles) the three-launch scan and the two-kernel sort."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0) if n_pairs > 1 else \
        Grid(n_az=36, n_el=9, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    b = synth.batched(n=3000, n_pairs=n_pairs, grid=g) if n_pairs > 1 else synth.tiny(grid=g)
    say("capacity overflow, pairs", n_pairs)
    prob = gpu_problem(b, cap=64)
    prob.project()
    n, ok = prob.splat_count()
    assert not ok and n > 64
    prob.bin_sort()
    sig, ssum, _ = prob.render_fwd()
    torch.cuda.synchronize()
    assert torch.count_nonzero(sig).item() == 0 and torch.count_nonzero(ssum).item() == 0
    L = gpu_lists(prob)
    assert L["overflow"] == n and np.all(L["ts"] == 0) and np.all(L["te"] == 0)
    prob.cap = n
    prob._alloc()
    S, _, _ = gpu_forward(prob)
    sc, p = b.scenes[0], b.pairs[0]
    if n_pairs == 1:
        compare_rays(S[0].ravel(), oracle.render(sc, p, g), sc, p, g)
    else:
        uv = np.stack([np.arange(0, 360, 15), np.arange(0, 90, 90 // 24)[:24]], 1)
        compare_rays(S[0][uv[:, 1], uv[:, 0]], oracle.trace(sc, p, g, uv), sc, p, g)


def test_multi_carrier_forward_matches_oracle_per_carrier():
    """40 carriers 40 MHz apart (two traversals: 32 carriers, then 8 in a
    16-carrier one) on the tiny room:
    every checked carrier against the oracle rendered at that frequency, the
    per-carrier sums against the rays, carrier 0 against the one-carrier
    forward, and a repeated call bit for bit."""
    g = Grid(n_az=37, n_el=11, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    b = synth.tiny(grid=g, n=1500)
    sc, p = b.scenes[0], b.pairs[0]
    prob = gpu_problem(b)
    sig1, _, _ = prob.forward()
    F, df = 40, 40e6
    say("multi-carrier: 40 carriers, 40 MHz apart")
    sig, ssum = prob.render_fwd_multi(F, df)
    sig2, ssum2 = prob.render_fwd_multi(F, df)
    torch.cuda.synchronize()
    assert torch.equal(sig, sig2) and torch.equal(ssum, ssum2)
    S = torch.view_as_complex(sig).cpu().numpy().astype(np.complex128)        # [1, F, n_el, n_az]
    Ssum = torch.view_as_complex(ssum).cpu().numpy().astype(np.complex128)    # [1, F]
    for c in (0, 1, 15, 16, 31, 32, 39):
        pc = Pair(p.rx, p.tx, p.freq_hz + c * df, p.scene)
        ref = oracle.render(sc, pc, g)
        compare_rays(S[0, c].ravel(), ref, sc, pc, g)
        assert abs(Ssum[0, c] - S[0, c].sum()) <= 1e-5 * np.abs(S[0, c]).sum() + 1e-30
    S1 = torch.view_as_complex(sig1).cpu().numpy().astype(np.complex128)[0]
    A = oracle.render(sc, p, g)["A_uv"].reshape(g.n_el, g.n_az)
    assert np.all(np.abs(S[0, 0] - S1) <= 1e-5 * np.maximum(A, 1e-30))


def test_multi_carrier_forward_in_a_many_tile_launch():
    """12 pairs of 360x90 rays (6480 tiles: one workgroup per tile), 3 carriers
    5 MHz apart (one 16-carrier traversal), sampled rays of three pairs against
    the oracle."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    b = synth.batched(n=5000, n_pairs=12, grid=g)
    sc = b.scenes[0]
    prob = gpu_problem(b)
    prob.forward()
    F, df = 3, 5e6
    sig, _ = prob.render_fwd_multi(F, df)
    torch.cuda.synchronize()
    S = torch.view_as_complex(sig).cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(5)
    for k in (0, 5, 11):
        p = b.pairs[k]
        uv = np.unique(np.stack([rng.integers(0, 360, 32), rng.integers(0, 90, 32)], 1), axis=0)
        for c in range(F):
            pc = Pair(p.rx, p.tx, p.freq_hz + c * df, p.scene)
            compare_rays(S[k, c][uv[:, 1], uv[:, 0]], oracle.trace(sc, pc, g, uv), sc, pc, g, max_marginal_frac=0.1)


def test_forward_is_deterministic():
    b = synth.tiny()
    prob = gpu_problem(b)
    S1, s1, _ = gpu_forward(prob)
    S2, s2, _ = gpu_forward(prob)
    assert np.array_equal(S1.view(np.float64), S2.view(np.float64)) and np.array_equal(s1, s2)


@pytest.mark.parametrize("tw,th,G", [(8, 8, 1), (16, 8, 2), (32, 8, 1), (16, 16, 1), (8, 8, 4), (16, 16, 4),
                                     (16, 8, 4), (8, 8, 2), (8, 8, 0), (16, 8, 0), (16, 16, 0), (32, 8, 0),
                                     (8, 4, 0), (4, 8, 0)])
def test_ragged_tiles_and_seam(tw, th, G):
    # 37 x 11 rays do not divide by any tile shape: ragged last column and row
    g = Grid(n_az=37, n_el=11, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=G)
    b = synth.tiny(grid=g, n=1500)
    sc, p = b.scenes[0], b.pairs[0]
    say("ragged", tw, th, "lanes", G)
    S, Ssum, _ = gpu_forward(gpu_problem(b))
    ref = oracle.render(sc, p, g)
    compare_rays(S[0].ravel(), ref, sc, p, g)


@pytest.mark.parametrize("tw,th", [(64, 1), (128, 1), (32, 2), (256, 1)])
def test_single_row_tiles_in_a_few_tile_launch(tw, th):
    """Tiles of one or two rows in a launch with few tiles (the forward's
    two-workgroups-per-tile path): every ray rendered, no row left unwritten."""
    g = Grid(n_az=290, n_el=5, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=0)
    b = synth.tiny(grid=g, n=1200)
    sc, p = b.scenes[0], b.pairs[0]
    say("single-row tiles", tw, th)
    prob = gpu_problem(b)
    sig = torch.full((1, g.n_el, g.n_az, 2), float("nan"), device="cuda")
    ssum = torch.empty((1, 2), device="cuda")
    prob.prepare()
    prob.render_fwd(sig, ssum, None)
    torch.cuda.synchronize()
    S = torch.view_as_complex(sig).cpu().numpy().astype(np.complex128)
    assert np.isfinite(S).all()
    ref = oracle.render(sc, p, g)
    compare_rays(S[0].ravel(), ref, sc, p, g)
    assert abs(complex(*ssum[0].cpu().numpy()) - ref["S_sum"]) <= 1e-4 * ref["A_uv"].sum()


@pytest.mark.parametrize("L,G,th", [(0, 1, 8), (1, 2, 8), (3, 4, 8), (4, 1, 8), (6, 4, 8), (5, 2, 8), (0, 0, 8),
                                    (1, 0, 8), (3, 0, 8), (6, 0, 8), (2, 0, 4), (6, 0, 4)])
def test_fle_degrees(L, G, th):
    g = Grid(n_az=24, n_el=8, fle_L=L, tile_w=8, tile_h=th, lanes_per_ray=G)
    rng = np.random.default_rng([100, L])
    sc = synth.draw_scene(rng, 800, (4.0, 4.0, 3.0), g.K)
    p = Pair(np.array([2.0, 2.1, 1.0], np.float32), np.array([0.5, 3.0, 2.0], np.float32), 5.8e9)
    say("fle degree", L)
    S, _, _ = gpu_forward(gpu_problem(Batch([sc], [p], g)))
    compare_rays(S[0].ravel(), oracle.render(sc, p, g), sc, p, g)


def test_empty_scene_and_empty_lists():
    g = Grid(n_az=36, n_el=9, fle_L=2)
    empty = Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros((0, 4), np.float32),
                  np.zeros((0,), np.float32), np.zeros((0, g.K, 2), np.float32))
    p = Pair(np.array([1, 1, 1], np.float32), np.array([2, 2, 2], np.float32), 2.4e9)
    S, Ssum, rssi = gpu_forward(gpu_problem(Batch([empty], [p, p], g)))
    assert np.all(S == 0) and np.all(Ssum == 0) and np.all(np.isneginf(rssi))
    # every Gaussian below the RX: all culled, exact zeros
    b = synth.tiny(n=300)
    sc = b.scenes[0]
    low = Scene(sc.means * np.array([1, 1, 0.0], np.float32) + np.array([0, 0, 0.1], np.float32), sc.log_scales - 1.0,
                sc.quats, sc.logits, sc.coeffs)
    S, Ssum, _ = gpu_forward(gpu_problem(Batch([low], b.pairs, b.grid)))
    assert np.all(S == 0)


def test_worked_example_on_gpu():
    """Two nearly transparent Gaussians on one ray at path lengths 3 m and
    3.0625 m (TX at the RX, 2.4 GHz) cancel: |S| <= 1e-4 A_uv in FP32."""
    g = Grid(n_az=36, n_el=9, fle_L=0, tile_w=8, tile_h=8)
    u, v = 7, 4
    d = oracle.ray_dirs(g)[v, u]
    rx = np.array([1.0, 1.5, 0.5])
    mu = np.array([rx + 1.5 * d, rx + 1.53125 * d], np.float32)
    c = np.zeros((2, 1, 2), np.float32)
    c[:, 0, 0] = 0.7
    sc = Scene(mu, np.full((2, 3), math.log(0.004), np.float32), np.tile(np.float32([1, 0, 0, 0]), (2, 1)),
               np.full(2, -30.0, np.float32), c)
    p = Pair(rx.astype(np.float32), rx.astype(np.float32), 2.4e9)
    S, _, _ = gpu_forward(gpu_problem(Batch([sc], [p], g)))
    ref = oracle.trace(sc, p, g, [(u, v)])
    assert ref["n_active"][0] == 2
    A = ref["A_uv"][0]
    assert abs(S[0, v, u]) <= 1e-4 * A
    one = Scene(*(getattr(sc, f)[:1] for f in ("means", "log_scales", "quats", "logits", "coeffs")))
    S1, _, _ = gpu_forward(gpu_problem(Batch([one], [p], g)))
    assert abs(S1[0, v, u]) == pytest.approx(A / 2, rel=1e-4)


def test_multi_scene_multi_pair_batch():
    g = Grid(n_az=48, n_el=12, fle_L=2, tile_w=8, tile_h=8)
    rng = np.random.default_rng(77)
    room = (6.0, 5.0, 3.0)
    scenes = [synth.draw_scene(rng, n, room, g.K) for n in (700, 0, 1500)]
    pairs = []
    for s, f in [(0, 2.4e9), (2, 5.0e9), (1, 5.8e9), (2, 2.4e9), (0, 5.8e9)]:
        pr = synth.draw_pair(rng, room, f, scene=s)
        pairs.append(pr)
    b = Batch(scenes, pairs, g)
    say("batch: scenes 700/0/1500, 5 pairs")
    S, Ssum, rssi = gpu_forward(gpu_problem(b))
    for k, pr in enumerate(pairs):
        sc = scenes[pr.scene]
        ref = oracle.render(sc, pr, g)
        compare_rays(S[k].ravel(), ref, sc, pr, g)
        assert abs(Ssum[k] - S[k].sum()) <= 1e-5 * np.abs(S[k]).sum() + 1e-30


@pytest.mark.parametrize("tw,th,G", [(16, 16, 1), (8, 8, 4), (16, 8, 2), (8, 8, 0), (16, 16, 0), (8, 4, 0)])
def test_paper_scale_sampled_rays_and_tiles(tw, th, G):
    """200k Gaussians, 360x90 rays, 5 GHz, at the launch configurations the
    benchmark times: sampled rays against the oracle, every record's rectangle
    and every tile list bit exact, and S_hat equal to the sum of the spectrum."""
    b = synth.paper_scale(grid=Grid(n_az=360, n_el=90, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=G))
    sc, p, g = b.scenes[0], b.pairs[0], b.grid
    say("paper scale: 200k gaussians, 360x90, tile", tw, th, "lanes", G)
    prob = gpu_problem(b)
    S, Ssum, rssi = gpu_forward(prob)
    rng = np.random.default_rng(5)
    uv = np.stack([rng.integers(0, g.n_az, 160), rng.integers(0, g.n_el, 160)], 1)
    ref = oracle.trace(sc, p, g, uv)
    st = compare_rays(S[0][uv[:, 1], uv[:, 0]], ref, sc, p, g)
    say("paper scale forward", st)
    assert abs(Ssum[0] - S[0].sum()) <= 1e-5 * np.abs(S[0]).sum()
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    np.testing.assert_array_equal(L["rec_key"], oracle.depth_key32(sc.means, p.rx).astype(np.uint32))
    # every record's cap rectangle (the FP32 screen or its FP64 fallback) and
    # every tile list, bit for bit, except Gaussians at a marginal decision
    tu0, ntu, tv0, ntv, cm = oracle.cap_rects(sc.means, sc.log_scales, p.rx, g)
    np.testing.assert_array_equal(L["rec_rect"][~cm], np.stack([tu0, ntu, tv0, ntv], 1)[~cm])
    say("paper scale: records", sc.n, "marginal rectangles", int(cm.sum()))
    tiles = np.arange(L["T"])
    ref_l, marg = oracle_tile_members(sc, p, g, tiles)
    bad = set(np.nonzero(marg)[0].tolist())
    for t in tiles:
        a, e = L["ts"][t], L["te"][t]
        gv, kv = L["val"][a:e].astype(np.int64), L["klo"][a:e].astype(np.int64)
        rg, rk = ref_l[int(t)]
        keep_g = np.array([x not in bad for x in gv], bool)
        keep_r = np.array([x not in bad for x in rg], bool)
        np.testing.assert_array_equal(gv[keep_g], rg[keep_r])
        np.testing.assert_array_equal(kv[keep_g], rk[keep_r])


def test_long_tile_lists_are_merged_exactly():
    """500k Gaussians with 16x16 tiles: the longest lists (tens of thousands of
    entries) exceed one LDS chunk, so sorted runs are merged in global memory;
    those lists and sampled rays must still match the oracle exactly."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=16, tile_h=16, lanes_per_ray=1)
    b = synth.batched(n=500_000, n_pairs=1, grid=g)
    sc, p = b.scenes[0], b.pairs[0]
    say("500k gaussians, 16x16 tiles")
    prob = gpu_problem(b)
    S, _, _ = gpu_forward(prob)
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    lens = L["te"] - L["ts"]
    say("longest lists", np.sort(lens)[-5:])
    assert lens.max() > 16384
    rng = np.random.default_rng(8)
    tiles = np.concatenate([np.argsort(lens)[-6:], rng.choice(L["T"], 4, replace=False)])
    ref_l, marg = oracle_tile_members(sc, p, g, tiles)
    bad = set(np.nonzero(marg)[0].tolist())
    for t in tiles:
        a, e = L["ts"][t], L["te"][t]
        gv, kv = L["val"][a:e].astype(np.int64), L["klo"][a:e].astype(np.int64)
        rg, rk = ref_l[int(t)]
        keep_g = np.array([x not in bad for x in gv], bool)
        keep_r = np.array([x not in bad for x in rg], bool)
        np.testing.assert_array_equal(gv[keep_g], rg[keep_r])
        np.testing.assert_array_equal(kv[keep_g], rk[keep_r])
    uv = np.stack([rng.integers(0, g.n_az, 64), rng.integers(0, g.n_el, 64)], 1)
    compare_rays(S[0][uv[:, 1], uv[:, 0]], oracle.trace(sc, p, g, uv), sc, p, g)


def test_large_batch_wide_workgroups_match_oracle():
    """500k Gaussians x 9 pairs = 4.5 M records: project and emit run with
    1024-record workgroups; every record's key and rectangle and sampled tile
    lists of three pairs stay bit exact and sampled rays match the oracle."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=16, tile_h=8, lanes_per_ray=0)
    b = synth.batched(n=500_000, n_pairs=9, grid=g)
    sc = b.scenes[0]
    say("500k gaussians x 9 pairs, 16x8 tiles")
    prob = gpu_problem(b)
    assert prob.layout().n_records == 9 * 500_000
    S, Ssum, _ = gpu_forward(prob)
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    rng = np.random.default_rng(17)
    T = L["T"]
    # every list of every pair is ordered by (key, Gaussian index)
    comp = (L["klo"].astype(np.uint64) << np.uint64(32)) | L["val"].astype(np.uint64)
    step_ok = comp[1:] > comp[:-1]
    first = np.zeros(len(comp), bool)
    first[L["ts"][L["te"] > L["ts"]]] = True
    assert np.all(step_ok | first[1:])
    say("longest list", int((L["te"] - L["ts"]).max()))
    # every list of every pair against the host expansion of the records'
    # rectangles (all bucket-length tiers of the sort: up to 2048, 3840, the
    # 2-per-CU chunk, 16384 entries and beyond)
    lens = assert_lists_complete(L, g.n_az // g.tile_w + (g.n_az % g.tile_w > 0), [0] * 9)
    say("list lengths per tier", [int(((lens > a) & (lens <= b_)).sum()) for a, b_ in
                                  [(0, 2048), (2048, 3840), (3840, 7936), (7936, 16384), (16384, 1 << 30)]])
    assert (lens > 16384).any() and ((lens > 2048) & (lens <= 3840)).any()
    for k in range(9):     # every record's key and cap rectangle, bit for bit
        p = b.pairs[k]
        np.testing.assert_array_equal(L["rec_key"][k * sc.n:(k + 1) * sc.n],
                                      oracle.depth_key32(sc.means, p.rx).astype(np.uint32))
        tu0, ntu, tv0, ntv, cm = oracle.cap_rects(sc.means, sc.log_scales, p.rx, g)
        np.testing.assert_array_equal(L["rec_rect"][k * sc.n:(k + 1) * sc.n][~cm],
                                      np.stack([tu0, ntu, tv0, ntv], 1)[~cm])
    for k in (0, 4, 8):
        p = b.pairs[k]
        lens = L["te"][k * T:(k + 1) * T] - L["ts"][k * T:(k + 1) * T]
        # six random tiles and the two longest (sorted by the long-bucket kernel)
        tiles = np.unique(np.concatenate([rng.choice(T, 6, replace=False), np.argsort(lens)[-2:]]))
        ref_l, marg = oracle_tile_members(sc, p, g, tiles)
        bad = set(np.nonzero(marg)[0].tolist())
        for t in tiles:
            a, e = L["ts"][k * T + t], L["te"][k * T + t]
            gv, kv = L["val"][a:e].astype(np.int64), L["klo"][a:e].astype(np.int64)
            rg, rk = ref_l[int(t)]
            keep_g = np.array([x not in bad for x in gv], bool)
            keep_r = np.array([x not in bad for x in rg], bool)
            np.testing.assert_array_equal(gv[keep_g], rg[keep_r])
            np.testing.assert_array_equal(kv[keep_g], rk[keep_r])
        uv = np.stack([rng.integers(0, g.n_az, 24), rng.integers(0, g.n_el, 24)], 1)
        compare_rays(S[k][uv[:, 1], uv[:, 0]], oracle.trace(sc, p, g, uv), sc, p, g)


@pytest.mark.parametrize("tw,th,G", [(8, 8, 0), (16, 8, 0), (8, 8, 2)])
def test_paper_footprint_binning_matches_oracle(tw, th, G):
    """Binning by the paper's footprint (grid.footprint = 1): every record's
    rectangle bit for bit (outside FP64-marginal floors), the tile lists, and
    the render restricted to those tiles against the oracle, ray by ray."""
    g = Grid(n_az=72, n_el=18, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=G, footprint=1)
    b = synth.tiny(grid=g, n=2000)
    sc, p = b.scenes[0], b.pairs[0]
    say("paper footprint", tw, th, "lanes", G)
    prob = gpu_problem(b)
    S, Ssum, _ = gpu_forward(prob)
    rects = oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, p.rx, g)
    marg = rects[4]
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    np.testing.assert_array_equal(L["rec_rect"][~marg], np.stack(rects[:4], 1)[~marg])
    if not marg.any():
        assert L["n"] == int((rects[1] * rects[3]).sum())
    ref = oracle.render(sc, p, g, rects=rects)
    # rays in a tile of a Gaussian whose rectangle is marginal are not compared
    skip = np.zeros(ref["S"].shape[0], bool)
    if marg.any():
        allow = oracle.rect_allow(rects, g, ref["rays_uv"])
        skip = allow[:, marg].any(1)
    ok = ~skip & ~ref["marginal"]
    err = np.abs(S[0].ravel() - ref["S"])
    assert np.all(err[ok] <= TOL * np.maximum(ref["A_uv"][ok], 1e-30)), float(err[ok].max())
    # a real variant: some hit of the exact binning is dropped here
    exact = oracle.render(sc, p, Grid(n_az=72, n_el=18, fle_L=2, tile_w=tw, tile_h=th))
    assert (ref["n_active"] < exact["n_active"]).any()


def test_paper_footprint_at_paper_scale():
    """200k Gaussians, 360x90 rays, 8x8 tiles (the benchmark's launch
    configuration) with the paper footprint: every record's rectangle against
    the oracle, sampled rays against the oracle render restricted to the same
    tiles, and S_hat equal to the sum of the spectrum."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=8, tile_h=8, footprint=1)
    b = synth.paper_scale(grid=g)
    sc, p = b.scenes[0], b.pairs[0]
    say("paper footprint at paper scale")
    prob = gpu_problem(b)
    S, Ssum, _ = gpu_forward(prob)
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    rects = oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, p.rx, g)
    marg = rects[4]
    np.testing.assert_array_equal(L["rec_rect"][~marg], np.stack(rects[:4], 1)[~marg])
    rng = np.random.default_rng(7)
    uv = np.stack([rng.integers(0, g.n_az, 160), rng.integers(0, g.n_el, 160)], 1)
    ref = oracle.trace(sc, p, g, uv, rects=rects)
    ok = ~ref["marginal"]
    if marg.any():
        ok &= ~oracle.rect_allow(rects, g, uv)[:, marg].any(1)
    err = np.abs(S[0][uv[:, 1], uv[:, 0]] - ref["S"])
    say("paper footprint at paper scale:", int(ok.sum()), "rays compared,", int(marg.sum()), "marginal records")
    assert ok.sum() >= 150
    assert np.all(err[ok] <= TOL * np.maximum(ref["A_uv"][ok], 1e-30)), float(err[ok].max())
    assert abs(Ssum[0] - S[0].sum()) <= 1e-5 * np.abs(S[0]).sum()


def test_paper_footprint_multi_carrier_forward():
    """The multi-carrier traversal over the paper-footprint lists: checked
    carriers against the oracle restricted to the same tiles at that frequency."""
    g = Grid(n_az=37, n_el=11, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0, footprint=1)
    b = synth.tiny(grid=g, n=1500)
    sc, p = b.scenes[0], b.pairs[0]
    say("paper footprint, multi-carrier: 20 carriers, 40 MHz apart")
    prob = gpu_problem(b)
    prob.forward()
    rects = oracle.footprint_rects(sc.means, sc.log_scales, sc.quats, p.rx, g)
    assert not rects[4].any()
    F, df = 20, 40e6
    sig, _ = prob.render_fwd_multi(F, df)
    torch.cuda.synchronize()
    S = torch.view_as_complex(sig).cpu().numpy().astype(np.complex128)
    for c in (0, 7, 19):
        pc = Pair(p.rx, p.tx, p.freq_hz + c * df, p.scene)
        ref = oracle.render(sc, pc, g, rects=rects)
        ok = ~ref["marginal"]
        err = np.abs(S[0, c].ravel() - ref["S"])
        assert np.all(err[ok] <= TOL * np.maximum(ref["A_uv"][ok], 1e-30)), (c, float(err[ok].max()))


@pytest.mark.gpu
def test_every_record_on_the_fp64_rectangle_matches_oracle():
    """100k Gaussians 80-87 degrees above the receiver: cos(beta_c) < 0.2 and
    the cap below the pole, so the FP32 screen decides none of them and every
    record takes the FP64 evaluation (all 256 lanes of each projection
    workgroup).  Every rectangle bit for bit against the oracle, every tile
    list complete, and sampled rays near the zenith against the oracle."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    rng = np.random.default_rng(23)
    n = 100_000
    rx = np.array([5.0, 4.0, 0.5], np.float32)
    el = np.radians(rng.uniform(80.0, 87.0, n))
    az = rng.uniform(0.0, 2 * np.pi, n)
    d = rng.uniform(1.5, 2.5, n)
    means = rx.astype(np.float64) + np.stack([d * np.cos(el) * np.cos(az), d * np.cos(el) * np.sin(az),
                                              d * np.sin(el)], 1)
    base = synth.draw_scene(rng, n, (1.0, 1.0, 1.0), g.K)
    sc = Scene(means.astype(np.float32), np.log(rng.uniform(0.004, 0.008, (n, 3))).astype(np.float32),
                     base.quats, base.logits, base.coeffs)
    p = Pair(rx, np.array([2.0, 2.0, 1.5], np.float32), 5e9)
    b = Batch([sc], [p], g)
    # premise: not full (beta_c + theta below the pole) and cos(beta_c) < 0.2 for every record
    e = sc.means.astype(np.float64) - rx
    D = np.linalg.norm(e, axis=1)
    Rb = 3.0 * np.exp(sc.log_scales.astype(np.float64).max(1))
    bc = np.arctan2(e[:, 2], np.hypot(e[:, 0], e[:, 1]))
    assert np.all(bc + np.arcsin(Rb / D) + 1e-4 < np.pi / 2) and np.all(np.cos(bc) < 0.2) and np.all(D > 1.2)
    say("FP64 rectangles: 100k records near the pole")
    prob = gpu_problem(b)
    S, _, _ = gpu_forward(prob)
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    tu0, ntu, tv0, ntv, cm = oracle.cap_rects(sc.means, sc.log_scales, p.rx, g)
    assert (ntu * ntv > 0).sum() > 90_000
    np.testing.assert_array_equal(L["rec_rect"][~cm], np.stack([tu0, ntu, tv0, ntv], 1)[~cm])
    say("records", n, "marginal", int(cm.sum()))
    lens = assert_lists_complete(L, g.n_tiles_az, [0])
    say("splats", int(lens.sum()))
    uv = np.stack([rng.integers(0, g.n_az, 40), rng.integers(80, g.n_el, 40)], 1)
    compare_rays(S[0][uv[:, 1], uv[:, 0]], oracle.trace(sc, p, g, uv), sc, p, g)


def test_large_uneven_batch_binning_is_complete():
    """Three scenes (1,000,000, 333,333 and 40,001 Gaussians, sizes not multiples
    of the workgroups' 1024 records) and 7 pairs: 4.7 M records, so project takes
    four 256-record chunks per workgroup (one FP64 rectangle pass for the four)
    and emit 1024 records per workgroup, across scene boundaries.  Every record's
    key and rectangle against the oracle and every tile list of every pair
    against the host expansion of the rectangles."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    rng = np.random.default_rng(31)
    room = (10.0, 8.0, 3.0)
    scenes = [synth.draw_scene(rng, n, room, g.K) for n in (1_000_000, 333_333, 40_001)]
    pairs = [synth.draw_pair(rng, room, 5e9, scene=s) for s in (0, 0, 0, 0, 1, 1, 2)]
    b = Batch(scenes, pairs, g)
    say("large uneven batch: 3 scenes, 7 pairs")
    prob = gpu_problem(b)
    n_rec = sum(scenes[p.scene].n for p in pairs)
    assert prob.layout().n_records == n_rec and n_rec >= (1 << 22)
    S, _, _ = gpu_forward(prob)
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    offs = np.cumsum([0] + [s.n for s in scenes])
    for k, p in enumerate(pairs):
        sc = scenes[p.scene]
        a, e = int(L["base"][k]), int(L["base"][k + 1])
        np.testing.assert_array_equal(L["rec_key"][a:e], oracle.depth_key32(sc.means, p.rx).astype(np.uint32))
        tu0, ntu, tv0, ntv, cm = oracle.cap_rects(sc.means, sc.log_scales, p.rx, g)
        np.testing.assert_array_equal(L["rec_rect"][a:e][~cm], np.stack([tu0, ntu, tv0, ntv], 1)[~cm])
    lens = assert_lists_complete(L, g.n_tiles_az, [int(offs[p.scene]) for p in pairs])
    say("splats", int(lens.sum()), "longest list", int(lens.max()))
    p = pairs[4]
    uv = np.stack([rng.integers(0, g.n_az, 24), rng.integers(0, g.n_el, 24)], 1)
    compare_rays(S[4][uv[:, 1], uv[:, 0]], oracle.trace(scenes[p.scene], p, g, uv), scenes[p.scene], p, g)


@pytest.mark.parametrize("n_gauss,n_pairs", [(200_000, 8), (500_000, 9)])
def test_tiered_sort_ignores_workspace_contents(n_gauss, n_pairs):
    """More than 2048 (pair, tile) units: the sort runs in tiers by bucket length,
    the long buckets taken from a queue whose counts and pop counters live in the
    workspace.  A workspace filled with 0xFF bytes before the forward gives the
    same tile ranges, sorted lists and signal, bit for bit, as a zeroed one.
    200k x 8: 256-record projection and emit workgroups, buckets up to about
    7,500 entries (the 16-entry tier's classes stay empty); 500k x 9: 4.5 M
    records, so four-chunk projection and staged 1024-record emit, and buckets
    past the 16384 entries that the longest tier keeps in LDS."""
    g = Grid(n_az=360, n_el=90, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    rng = np.random.default_rng([41, n_pairs])
    room = (10.0, 8.0, 3.0)
    sc = synth.draw_scene(rng, n_gauss, room, g.K)
    b = Batch([sc], [synth.draw_pair(rng, room, 5e9) for _ in range(n_pairs)], g)
    say("tiered sort, workspace fill 0 and 0xFF:", n_gauss, "gaussians,", n_pairs, "pairs")
    prob = gpu_problem(b)
    assert n_pairs * g.n_tiles > 2048
    runs = []
    for fill in (0, 255):
        prob.ws.fill_(fill)
        sig, ssum, _ = prob.forward()
        L = gpu_lists(prob)
        runs.append((sig.clone(), ssum.clone(), L))
    (s0, m0, L0), (s1, m1, L1) = runs
    assert L0["overflow"] == 0 and L0["n"] == L1["n"]
    lengths = L0["te"] - L0["ts"]
    assert lengths.max() > 3840   # the long-bucket tiers are exercised
    if n_gauss >= 500_000:
        assert lengths.max() > 16384
    for key in ("ts", "te", "klo", "val", "rec_key", "rec_rect"):
        np.testing.assert_array_equal(L0[key], L1[key], err_msg=key)
    assert torch.equal(s0, s1) and torch.equal(m0, m1)


def test_large_batch_on_a_fine_grid_is_complete():
    """720 x 180 rays in 8x8 tiles (2070 tiles per pair, past the 1536 that the
    staged 1024-record emit holds in LDS, so emit takes its direct path) and
    4.2 M records (one 600,000-Gaussian scene, 7 pairs).  Every record's key and
    rectangle against the oracle, every tile list of every pair against the
    host expansion of the rectangles, and sampled rays against the oracle."""
    g = Grid(n_az=720, n_el=180, fle_L=2, tile_w=8, tile_h=8, lanes_per_ray=0)
    assert g.n_tiles > 1536
    rng = np.random.default_rng(43)
    room = (10.0, 8.0, 3.0)
    sc = synth.draw_scene(rng, 600_000, room, g.K)
    pairs = [synth.draw_pair(rng, room, 5e9) for _ in range(7)]
    b = Batch([sc], pairs, g)
    say("fine grid batch: 720x180 rays, 600k gaussians, 7 pairs")
    prob = gpu_problem(b)
    assert prob.layout().n_records == 7 * sc.n >= (1 << 22)
    S, _, _ = gpu_forward(prob)
    L = gpu_lists(prob)
    assert L["overflow"] == 0
    for k, p in enumerate(pairs):
        a, e = int(L["base"][k]), int(L["base"][k + 1])
        np.testing.assert_array_equal(L["rec_key"][a:e], oracle.depth_key32(sc.means, p.rx).astype(np.uint32))
        tu0, ntu, tv0, ntv, cm = oracle.cap_rects(sc.means, sc.log_scales, p.rx, g)
        np.testing.assert_array_equal(L["rec_rect"][a:e][~cm], np.stack([tu0, ntu, tv0, ntv], 1)[~cm])
    lens = assert_lists_complete(L, g.n_tiles_az, [0] * len(pairs))
    say("splats", int(lens.sum()), "longest list", int(lens.max()))
    p = pairs[3]
    uv = np.stack([rng.integers(0, g.n_az, 16), rng.integers(0, g.n_el, 16)], 1)
    compare_rays(S[3][uv[:, 1], uv[:, 0]], oracle.trace(sc, p, g, uv), sc, p, g)
