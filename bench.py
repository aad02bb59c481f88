#!/usr/bin/env python
"""Throughput of the GSRF hot path on one MI355X.

A step is one pass of the whole path over one TX/RX pair of a 200k-Gaussian
synthetic room at 360x90 rays and 5 GHz: activation + splatting
(gsrf_project), binning + per-tile sort (gsrf_bin_sort), complex rendering +
RSSI (gsrf_render_fwd) and the adjoint + chain rule (gsrf_render_bwd) with a
seeded upstream gradient.  Inputs are resident in HBM before timing starts.
The headline rate replays the step captured once as a hipGraph (the way a
training loop over a fixed-shape problem runs it: the same kernels, launched
without host round trips); the rate of eager launches is reported beside it.

Prints one JSON line (rank 0).  Extra fields report the forward-only rate,
the two batched workloads -- 256 pairs over one 500k-Gaussian room (forward)
and 16 scenes of 20k-1M Gaussians with 8-64 pairs each (forward + adjoint) --
each as hipGraph replays with an autotuned tile shape, the multi-carrier
forward (26 carriers of one OFDM block per pass), a whole training iteration
(render, spectrum loss, adjoint, SGD update), the roofline of the
dominant kernel of each workload and the FP64 oracle timed on the host's
cores.  ``--workloads`` restricts the run (profiling).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "received spectra/s (360×90 rays, 200k Gaussians) fwd & fwd+bwd; batched vs plain"
PEAK_FP32_VALU = 157.3e12   # FLOP/s: 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
PEAK_HBM = 8.0e12           # B/s


# Algorithmic work per unit of the tiled method (the scope table's measurement
# model): a tile test (a ray of a tile against a list entry up to the tile's
# termination) costs 20 FP32 operations (6 FMA for A, 3 FMA for B, rcp, Q, t,
# two compares), a processed hit 70 (exp, p, alpha, local phase, sincos, psi
# as 9 complex MACs, complex scale and accumulate, T), and the adjoint three
# times the forward.  These are the counts `frac` is taken against.
ALG_TEST, ALG_HIT, ALG_BWD_FACTOR = 20.0, 70.0, 3.0


def alg_flops(st: dict) -> dict:
    fwd = st["tile_tests"] * ALG_TEST + st["hits"] * ALG_HIT
    return {"render_fwd": fwd, "render_bwd": ALG_BWD_FACTOR * fwd}


def flops_impl(K: int) -> dict:
    """FP32 operations (FMA = 2) the kernels execute per hit test and per
    processed hit, for comparison with the algorithmic counts.

    test: eps (6) + M v (15) + A (5) + b (5) + M eps (15) + c (5) + 1/A, b/A (2)
          + Q (3) + t (2) + two compares (2) = 60 (forward only: the adjoint
          reuses the forward's hit masks and makes no tests)
    hit, forward: exp(-Q/2) (2) + alpha, p (3) + phase (2) + sincos (30)
          + psi (8K) + psi e^{-j phase} (6) + c~ (2) + S, T update (7) = 52 + 8K
    hit, adjoint: the forward's hit terms (52 + 8K) + prefix and remainder (6)
          + dL/dp, dL/dphase, dL/dalpha (13) + dL/dG, dL/dQ, dL/dt (7)
          + p_perp, M p_perp (18) + dL/dM (30) + dL/dmu (9) + dL/dN, dL/do (2)
          + dL/dpsi (8) + dL/dc (6K) + T (2) + one add per accumulator for the
          reduction over rays (12 + 2K) = 159 + 16K
    """
    return dict(test=60.0, hit_fwd=52.0 + 8 * K, hit_bwd=52.0 + 8 * K + 107.0 + 8 * K)


def impl_flops(st: dict, K: int) -> dict:
    f = flops_impl(K)
    return {"render_fwd": st["tests"] * f["test"] + st["hits"] * f["hit_fwd"],
            "render_bwd": st["hits"] * f["hit_bwd"]}


def flops_multi(n_freq: int, tile_tests: int, hits: int) -> float:
    """Algorithmic FP32 FLOPs of the multi-carrier forward: the single-carrier
    forward's (tile tests x 20 + processed hits x 70) once, plus per hit and
    extra carrier the phase term and the complex accumulate (10)."""
    return tile_tests * ALG_TEST + hits * (ALG_HIT + 10.0 * (n_freq - 1))


def kernel_roofline(kernel: str, st: dict, K: int, t_kernel: float) -> dict:
    """Roofline object of one render kernel: algorithmic FLOPs per launch over
    its measured duration, against the FP32 VALU peak."""
    fl = alg_flops(st)[kernel]
    ach = fl / t_kernel
    return {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP32_VALU, "traffic": None, "kernel": kernel, "kernel_ms": t_kernel * 1e3,
            "flop_per_launch": fl,
            "flop_model": f"tile tests x {ALG_TEST:g} + processed hits x {ALG_HIT:g}"
                          + (f", x {ALG_BWD_FACTOR:g} for the adjoint" if kernel == "render_bwd" else ""),
            "flop_model_impl": impl_flops(st, K)[kernel]}


def pipeline_roofline(st: dict, n_gauss: int, visible: int, splats: int, rays: int, t_step: float,
                      bwd: bool) -> dict:
    """Whole-path roofline time t_roof = max(F / VALU peak, B / HBM peak) over
    the measured step time, with F the algorithmic FLOPs of the render
    kernel(s) and B the algorithmic bytes: the scene read once (116 B per
    Gaussian), 16 B per visible (pair, Gaussian) record, two passes of 12 B per
    splat, 8 B per output ray, and for the adjoint 29 floats per staged
    (tile, Gaussian) entry."""
    af = alg_flops(st)
    F = af["render_fwd"] + (af["render_bwd"] if bwd else 0.0)
    B = 116.0 * n_gauss + 16.0 * visible + 24.0 * splats + 8.0 * rays + (116.0 * st["staged"] if bwd else 0.0)
    t_roof = max(F / PEAK_FP32_VALU, B / PEAK_HBM)
    return {"flop": F, "bytes": B, "t_roof_ms": t_roof * 1e3, "t_measured_ms": t_step * 1e3,
            "frac": t_roof / t_step, "bound": "alu" if F / PEAK_FP32_VALU >= B / PEAK_HBM else "hbm"}


def visible_records(prob) -> int:
    """(pair, Gaussian) records whose tile rectangle is not empty."""
    import torch
    lay = prob.layout()
    r = prob.view(lay.rec_rect, torch.int16, int(lay.n_records) * 4).view(-1, 4).to(torch.int32) & 0xFFFF
    return int(((r[:, 1] * r[:, 3]) > 0).sum())


def host_cpu() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import psutil
        phys = psutil.cpu_count(logical=False)
    except Exception:
        phys = None
    return {"cpu_model": model, "physical_cores": phys, "logical_cpus": os.cpu_count()}


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "render_traffic.json")


def measured_traffic(kernel: str, config: str):
    """HBM bytes per launch of `kernel` at `config` from the committed PMC record
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel's readings), or None when
    there is no record or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_2502_01826_amd.profiling import sources_hash
    if rec.get("sources_sha256") != sources_hash():
        return None
    ent = rec.get("kernels", {}).get(kernel, {}).get(config)
    return None if ent is None else float(ent["bytes_per_launch"])


def cpu_baseline(scene, pair, grid, min_seconds: float = 8.0) -> dict:
    """The FP64 oracle (forward + autograd gradient) on a sample of rays of the
    same pair, scaled to a full spectrum."""
    import numpy as np
    import torch

    import oracle
    import synth

    rng = np.random.default_rng(123)
    n_rays = grid.n_az * grid.n_el
    sample = 256
    while True:
        uv = np.stack([rng.integers(0, grid.n_az, sample), rng.integers(0, grid.n_el, sample)], 1)
        G = synth.cotangent((sample,), seed=7)
        t0 = time.perf_counter()
        oracle.vjp(scene, pair, grid, G, rays_uv=uv)
        dt = time.perf_counter() - t0
        if dt >= min_seconds or sample >= n_rays:
            break
        sample = min(n_rays, sample * 2)
    per_spectrum = dt * n_rays / sample
    return {"value": 1.0 / per_spectrum, "unit": "spectra/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"FP64 forward + autograd gradient of {sample} of {n_rays} rays of one pair "
                      f"({dt:.1f} s), scaled by {n_rays / sample:.1f}",
            "threads_used": torch.get_num_threads(), **host_cpu()}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batched", choices=("full", "small", "none"), default="full",
                    help="batched workloads: full (256 pairs x 500k; 16 uneven scenes), small, or none")
    ap.add_argument("--workloads", default="plain,fwd_500k,uneven,multi,train",
                    help="comma list of plain, fwd_500k, uneven, multi, train (profiling runs pick one)")
    ap.add_argument("--carriers", type=int, default=26, help="multi-carrier workload: carriers per pair")
    ap.add_argument("--carrier-step", type=float, default=312.5e3, help="multi-carrier workload: spacing in Hz")
    ap.add_argument("--batched-pairs", type=int, default=256)
    ap.add_argument("--batched-iters", type=int, default=50)
    ap.add_argument("--batched-warmup", type=int, default=10)
    ap.add_argument("--gaussians", type=int, default=200_000)
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched workloads: use --tile instead of autotuning (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", default="8x8", help="tile_w x tile_h (64, 128 or 256 rays)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="render traversal: 0 two-phase, or 1, 2, 4 lanes per ray (direct)")
    ap.add_argument("--footprint", choices=("cap", "paper"), default="cap",
                    help="splat binning: exact bounding cap, or the paper's 3 sqrt(lambda_max) footprint")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} (WORLD_SIZE={world}) is not supported; "
              "the pair batch would shard across GPUs with no exchange in the forward pass", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_2502_01826_amd import Problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tw, th = (int(x) for x in args.tile.split("x"))
    grid = synth.Grid(n_az=360, n_el=90, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=args.lanes,
                      footprint=int(args.footprint == "paper"))
    batch = synth.paper_scale(n=args.gaussians, grid=grid)
    scene, pair = batch.scenes[0], batch.pairs[0]
    params = dict(means=scene.means, log_scales=scene.log_scales, quats=scene.quats, logits=scene.logits,
                  coeffs=scene.coeffs)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    def make(pairs):
        prob = Problem(params, pairs, grid)
        prob.forward()                    # sizes the splat buffers once (host sync here only)
        prob.auto_capacity = False
        P = len(pairs)
        bufs = dict(
            sig=torch.empty((P, grid.n_el, grid.n_az, 2), dtype=torch.float32, device=dev),
            ssum=torch.empty((P, 2), dtype=torch.float32, device=dev),
            rssi=torch.empty((P,), dtype=torch.float32, device=dev),
            G=torch.from_numpy(synth.cotangent((P, grid.n_el, grid.n_az), seed=11)).to(dev),
            gsum=torch.from_numpy(synth.cotangent((P,), seed=12)).to(dev),
        )
        G_ = prob.n_gauss
        e = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
        bufs["grads"] = (e(G_, 3), e(G_, 3), e(G_, 4), e(G_), e(G_, grid.K, 2))
        return prob, bufs

    from paper_2502_01826_amd import _lib

    def new_event():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)                  # creates the underlying hipEvent_t
        return e

    def run(prob, bufs, steps, bwd, ev=None):
        for i in range(steps):
            if ev is not None and "s0" in ev:
                ev["s0"][i].record(stream)
            if ev is not None:
                # the library records these around its render kernels only
                _lib.lib().gsrf_set_kernel_events(ev["f0"][i].cuda_event, ev["f1"][i].cuda_event,
                                                  ev["b0"][i].cuda_event, ev["b1"][i].cuda_event)
            prob.project()
            prob.bin_sort()
            prob.render_fwd(bufs["sig"], bufs["ssum"], bufs["rssi"])
            if bwd:
                prob.render_bwd(bufs["sig"], bufs["G"], bufs["gsum"], out=bufs["grads"])
            if ev is not None and "s1" in ev:
                ev["s1"][i].record(stream)
        _lib.lib().gsrf_set_kernel_events(None, None, None, None)

    def timed(prob, bufs, steps, warmup, bwd, ev=None):
        run(prob, bufs, warmup, bwd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(prob, bufs, steps, bwd, ev)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def roofline(prob, bufs, bwd, pairs_timed=1):
        """Eager instrumented pass: render kernel times (HIP events around the
        kernels on their stream) and the algorithmic FLOPs of the traversal."""
        ev1 = {k: [new_event()] for k in ("f0", "f1", "b0", "b1")}
        run(prob, bufs, 1, bwd, ev1)
        torch.cuda.synchronize()
        t_f = ev1["f0"][0].elapsed_time(ev1["f1"][0]) * 1e-3
        t_b = ev1["b0"][0].elapsed_time(ev1["b1"][0]) * 1e-3 if bwd else 0.0
        st = prob.render_stats()
        dom, tk = ("render_bwd", t_b) if (bwd and t_b >= t_f) else ("render_fwd", t_f)
        roof = kernel_roofline(dom, st, grid.K, tk)
        roof["counts"] = st
        roof["other_kernel"] = (kernel_roofline("render_fwd" if dom == "render_bwd" else "render_bwd", st, grid.K,
                                                t_f if dom == "render_bwd" else t_b) if bwd else None)
        return roof

    def run_batched(b, grad, label):
        from paper_2502_01826_amd.batch import GraphStep, TuneCache, TuneResult, autotune
        cat, offs = b.concat()
        prm = dict(means=cat.means, log_scales=cat.log_scales, quats=cat.quats, logits=cat.logits,
                   coeffs=cat.coeffs)
        P = len(b.pairs)

        def build(g):
            return Problem(prm, b.pairs, g, scene_offsets=offs)

        def make_grad(prob):
            return (torch.from_numpy(synth.cotangent((P, grid.n_el, grid.n_az), seed=13)).to(dev),
                    torch.from_numpy(synth.cotangent((P,), seed=14)).to(dev))

        if args.no_autotune:
            tune = TuneResult(best=(grid.tile_w, grid.tile_h, grid.lanes_per_ray))
        else:
            tune = autotune(build, grid, grad=grad, make_grad=make_grad, iters=2,
                            cache=TuneCache(TuneCache.default_path()), size=(int(cat.means.shape[0]), P))
        tw, th, lanes = tune.best
        g = synth.Grid(n_az=360, n_el=90, fle_L=2, tile_w=tw, tile_h=th, lanes_per_ray=lanes,
                       footprint=grid.footprint)
        prob = build(g)
        gs, gsum = make_grad(prob) if grad else (None, None)
        step = GraphStep(prob, grad, gs, gsum)
        st = step.time_stats(iters=args.batched_iters, warmup=args.batched_warmup)
        t = st["median"]
        bufs = dict(sig=step.signal, ssum=step.signal_sum, rssi=step.rssi, G=gs, gsum=gsum, grads=step.grads)
        roof = roofline(prob, bufs, grad)
        # HBM bytes per launch from the committed PMC record, keyed by tile, lanes and Gaussians x pairs
        cfg = f"{tw}x{th}/{lanes}/{int(cat.means.shape[0])}x{P}"
        roof["traffic"] = measured_traffic(roof["kernel"], cfg) if grid.footprint == 0 else None
        if roof["other_kernel"] is not None:
            roof["other_kernel"]["traffic"] = (measured_traffic(roof["other_kernel"]["kernel"], cfg)
                                               if grid.footprint == 0 else None)
        n_splats, ok = prob.splat_count()
        if not ok:
            raise RuntimeError(f"{label}: {n_splats} splats exceed the capacity fixed before capture")
        roof["counts"]["splats"] = n_splats
        vis = visible_records(prob)
        pipe = pipeline_roofline(roof["counts"], int(cat.means.shape[0]), vis, n_splats,
                                 P * grid.n_az * grid.n_el, t, grad)
        del step, prob
        torch.cuda.empty_cache()
        return {"workload": label, "pairs": P, "gaussians": int(cat.means.shape[0]),
                "spectra_per_s": P / t, "ms_per_replay": t * 1e3,
                "ms_per_replay_p10_p90": [st["p10"] * 1e3, st["p90"] * 1e3],
                "timing": f"median of {st['n']} hipGraph replays after {args.batched_warmup} warm-up replays, HIP "
                "events around each replay (project+bin_sort+render_fwd" + ("+render_bwd" if grad else "") +
                " for all pairs)",
                "tile": f"{tw}x{th}", "lanes_per_ray": lanes,
                "autotune_ms": {f"{a}x{b_}/{c}": v * 1e3 for (a, b_, c), v in tune.seconds.items()},
                "autotune_cached": tune.cached,
                "splats_within_capacity": True, "visible_records": vis,
                "roofline": roof, "pipeline_roofline": pipe}

    def run_plain():
        prob, bufs = make([pair])
        ev = {k: [new_event() for _ in range(args.steps)] for k in ("f0", "f1", "b0", "b1", "s0", "s1")}
        torch.cuda.synchronize()
        t_eager = timed(prob, bufs, args.steps, args.warmup, True, ev)
        t_fwd_k = sum(a.elapsed_time(b) for a, b in zip(ev["f0"], ev["f1"])) / args.steps * 1e-3
        t_bwd_k = sum(a.elapsed_time(b) for a, b in zip(ev["b0"], ev["b1"])) / args.steps * 1e-3
        steps_ms = sorted(a.elapsed_time(b) for a, b in zip(ev["s0"], ev["s1"]))
        q = lambda f: steps_ms[min(len(steps_ms) - 1, int(round(f * (len(steps_ms) - 1))))]
        eager.update(ms_per_step=t_eager * 1e3, spectra_per_s=1.0 / t_eager,
                     step_ms_events={"median": q(0.5), "p10": q(0.1), "p90": q(0.9)})
        # the same step captured once and replayed: W untimed replays, then K
        # back-to-back replays bracketed by synchronisation
        from paper_2502_01826_amd.batch import GraphStep
        gstep = GraphStep(prob, grad=True, grad_signal=bufs["G"], grad_sum=bufs["gsum"])
        for _ in range(args.warmup):
            gstep.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            gstep.replay()
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t0) / args.steps
        gst = gstep.time_stats(iters=args.steps, warmup=1)
        step_stats.update(median=gst["median"] * 1e3, p10=gst["p10"] * 1e3, p90=gst["p90"] * 1e3)
        del gstep
        t_fwd_only = timed(prob, bufs, args.steps, 1, False)
        stats = prob.render_stats()
        n_splats, ok = prob.splat_count()
        if not ok:
            raise RuntimeError(f"plain step: {n_splats} splats exceed the capacity fixed before timing")
        K = grid.K
        dom, tk = ("render_bwd", t_bwd_k) if t_bwd_k >= t_fwd_k else ("render_fwd", t_fwd_k)
        roof = kernel_roofline(dom, stats, K, tk)
        roof["traffic"] = (measured_traffic(dom, f"{args.tile}/{args.lanes}/{args.gaussians}")
                           if args.footprint == "cap" else None)
        roof["timing"] = ("HIP events recorded by the library immediately around the render kernel on its "
                          "stream, averaged over the timed steps")
        roof["counts"] = {**stats, "splats": n_splats}
        roof["other_kernel"] = kernel_roofline("render_fwd" if dom == "render_bwd" else "render_bwd", stats, K,
                                               t_fwd_k if dom == "render_bwd" else t_bwd_k)
        vis = visible_records(prob)
        roof["pipeline"] = {
            "graph_replay": pipeline_roofline(stats, prob.n_gauss, vis, n_splats, grid.n_az * grid.n_el, t_step, True),
            "plain_eager": pipeline_roofline(stats, prob.n_gauss, vis, n_splats, grid.n_az * grid.n_el, t_eager,
                                             True)}
        del prob, bufs
        torch.cuda.empty_cache()
        return t_step, t_fwd_only, t_fwd_k, t_bwd_k, roof

    def run_multi():
        """One pair, n carriers per render: project + bin_sort + render_fwd_multi
        per pass (eager), against the single-carrier forward kernel of the same
        pair repeated once per carrier."""
        from paper_2502_01826_amd.render import multi_chunks
        nf, df = args.carriers, args.carrier_step
        prob, bufs = make([pair])
        msig = torch.empty((1, nf, grid.n_el, grid.n_az, 2), dtype=torch.float32, device=dev)
        msum = torch.empty((1, nf, 2), dtype=torch.float32, device=dev)
        steps = args.steps
        ev = {k: [new_event() for _ in range(steps)] for k in ("f0", "f1")}

        def passes(n, with_ev):
            for i in range(n):
                if with_ev:
                    _lib.lib().gsrf_set_kernel_events(ev["f0"][i].cuda_event, ev["f1"][i].cuda_event, None, None)
                prob.project()
                prob.bin_sort()
                prob.render_fwd_multi(nf, df, msig, msum)
            _lib.lib().gsrf_set_kernel_events(None, None, None, None)

        passes(args.warmup, False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        passes(steps, True)
        torch.cuda.synchronize()
        t_pass = (time.perf_counter() - t0) / steps
        t_mk = sum(a.elapsed_time(b) for a, b in zip(ev["f0"], ev["f1"])) / steps * 1e-3
        # the single-carrier forward kernel of the same pair, same instrumentation
        ev1 = {k: [new_event() for _ in range(steps)] for k in ("f0", "f1", "b0", "b1")}
        run(prob, bufs, 1, False)
        torch.cuda.synchronize()
        run(prob, bufs, steps, False, ev1)
        torch.cuda.synchronize()
        t_1k = sum(a.elapsed_time(b) for a, b in zip(ev1["f0"], ev1["f1"])) / steps * 1e-3
        # the several-carrier adjoint (after the one-carrier forward that records the hit
        # masks), against the one-carrier adjoint kernel of the same pair
        Gm = torch.from_numpy(synth.cotangent((1, nf, grid.n_el, grid.n_az), seed=15)).to(dev)
        Gms = torch.from_numpy(synth.cotangent((1, nf), seed=16)).to(dev)
        ev2 = {k: [new_event() for _ in range(steps)] for k in ("b0", "b1")}
        prob.render_bwd_multi(nf, df, Gm, Gms, out=bufs["grads"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            _lib.lib().gsrf_set_kernel_events(None, None, ev2["b0"][i].cuda_event, ev2["b1"][i].cuda_event)
            prob.render_bwd_multi(nf, df, Gm, Gms, out=bufs["grads"])
        _lib.lib().gsrf_set_kernel_events(None, None, None, None)
        torch.cuda.synchronize()
        t_bwd_call = (time.perf_counter() - t0) / steps
        t_mb = sum(a.elapsed_time(b) for a, b in zip(ev2["b0"], ev2["b1"])) / steps * 1e-3
        run(prob, bufs, 1, True)
        torch.cuda.synchronize()
        run(prob, bufs, steps, True, ev1)
        torch.cuda.synchronize()
        t_1b = sum(a.elapsed_time(b) for a, b in zip(ev1["b0"], ev1["b1"])) / steps * 1e-3
        st = prob.render_stats()
        n_splats, ok = prob.splat_count()
        if not ok:
            raise RuntimeError(f"multi-carrier: {n_splats} splats exceed the capacity fixed before timing")
        fl = flops_multi(nf, st["tile_tests"], st["hits"])
        ach = fl / t_mk
        del prob, bufs, msig, msum, Gm, Gms
        torch.cuda.empty_cache()
        adjoint = {"kernel_ms": t_mb * 1e3, "call_ms": t_bwd_call * 1e3,
                   "carrier_gradients_per_s": nf / t_bwd_call,
                   "single_carrier_adjoint_kernel_ms": t_1b * 1e3,
                   "speedup_vs_per_carrier_adjoints": nf * t_1b / t_mb,
                   "timing": f"{steps} eager gsrf_render_bwd_multi calls (total and adjoint passes per 16 carriers, "
                             "chain rule) after one warm-up call; kernel_ms: HIP events recorded by the library "
                             "around the traversals"}
        return {"workload": f"multi-carrier forward: {nf} carriers {df / 1e3:g} kHz apart (one OFDM block) on the "
                            "plain pair, 200k Gaussians, 360x90 rays",
                "carriers": nf, "carrier_step_hz": df,
                "carrier_spectra_per_s": nf / t_pass, "ms_per_pass": t_pass * 1e3,
                "timing": f"{steps} eager passes (project+bin_sort+render_fwd_multi) after {args.warmup} warm-up "
                          "passes, wall clock between synchronisations",
                "carriers_per_traversal": multi_chunks(nf),
                "kernel_ms": t_mk * 1e3, "single_carrier_kernel_ms": t_1k * 1e3,
                "speedup_vs_per_carrier_kernels": nf * t_1k / t_mk,
                "adjoint": adjoint,
                "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                             "unit": "TFLOP/s", "frac": ach / PEAK_FP32_VALU,
                             "traffic": (measured_traffic("render_fwd_multi", f"{args.tile}/{args.lanes}/{args.gaussians}")
                                         if args.footprint == "cap" else None),
                             "kernel": "render_fwd_multi traversals", "flop_per_launch": fl,
                             "timing": "HIP events recorded by the library around the carrier-chunk traversals",
                             "counts": st}}

    def run_train():
        """One training iteration per step on the plain pair: project, bin_sort,
        render_fwd, the antenna-array loss against a target spectrum (the power
        spectrum of a perturbed copy of the room), render_bwd with the loss's
        gradient, the mean-gradient statistics and the SGD update of every
        attribute.  Eager launches (the mean learning rate changes every
        iteration).  Then one density-control pass on the statistics."""
        from paper_2502_01826_amd import train as tr
        prob, bufs = make([pair])
        _, pert = synth.training_step(n=args.gaussians, grid=grid)
        tprob = Problem(dict(means=pert.means, log_scales=pert.log_scales, quats=pert.quats, logits=pert.logits,
                             coeffs=pert.coeffs), [pair], grid)
        tsig, _, _ = tprob.forward()
        target = (tsig ** 2).sum(-1)
        pscale = 1.0 / float(target.max())           # spectra compared as images normalised to a peak of 1
        target = (target * pscale).contiguous()
        del tprob, tsig
        lam1, lam2 = 0.2, 0.1
        loss_fn = tr.SpectrumLoss(1, grid.n_el, grid.n_az, lam1, lam2, power_scale=pscale)
        lossb = torch.empty((1, 4), dtype=torch.float32, device=dev)
        gsig = torch.empty_like(bufs["sig"])
        params = (prob.means, prob.log_scales, prob.quats, prob.logits, prob.coeffs)
        gstats = tr.GradStats(prob.n_gauss)
        steps = args.steps
        ev = {k: [new_event() for _ in range(steps)] for k in ("l0", "l1", "o0", "o1")}
        first_loss = []

        def iterate(n, it0, with_ev):
            for i in range(n):
                prob.project()
                prob.bin_sort()
                prob.render_fwd(bufs["sig"], bufs["ssum"], bufs["rssi"])
                if with_ev:
                    ev["l0"][i].record(stream)
                loss_fn(bufs["sig"], target, loss=lossb, grad_signal=gsig)
                if with_ev:
                    ev["l1"][i].record(stream)
                prob.render_bwd(bufs["sig"], gsig, None, out=bufs["grads"])
                if with_ev:
                    ev["o0"][i].record(stream)
                gstats.accumulate(bufs["grads"][0])
                tr.sgd_step(params, bufs["grads"], it0 + i, fle_L=grid.fle_L)
                if with_ev:
                    ev["o1"][i].record(stream)

        iterate(1, 0, False)
        torch.cuda.synchronize()
        first_loss.append(float(lossb[0, 0]))
        iterate(args.warmup, 1, False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iterate(steps, 1 + args.warmup, True)
        torch.cuda.synchronize()
        t_it = (time.perf_counter() - t0) / steps
        t_loss = sum(a.elapsed_time(b) for a, b in zip(ev["l0"], ev["l1"])) / steps * 1e-3
        t_sgd = sum(a.elapsed_time(b) for a, b in zip(ev["o0"], ev["o1"])) / steps * 1e-3
        n_splats, ok = prob.splat_count()
        G_, K = prob.n_gauss, grid.K
        sgd_bytes = G_ * (11 + 2 * K) * 4 * 3          # read w and g, write w
        # one density-control pass on the window's statistics (every 100 iterations in the paper)
        z = torch.from_numpy(np.random.default_rng(5).normal(0, 1, (G_, 2, 3)).astype(np.float32)).to(dev)
        dp = tr.DensityParams(clone_step=tr.LearningRates().mean_init)
        d_ev = [(new_event(), new_event()) for _ in range(5)]
        for a_, b_ in d_ev:
            a_.record(stream)
            _, _, dcounts = tr.density_control(params, gstats, z, grid.fle_L, dp, read_counts=False)
            b_.record(stream)
        torch.cuda.synchronize()
        t_dc = sorted(a_.elapsed_time(b_) for a_, b_ in d_ev)[2] * 1e-3
        n_out, n_clone, n_split, n_pruned = (int(v) for v in dcounts.cpu())
        row = (11 + 2 * K + 4) * 4                      # attributes + statistics per Gaussian
        dc_bytes = G_ * (row + 24) + n_out * row         # read every Gaussian and its draws, write the survivors
        out = {"workload": "training iteration on the plain pair (200k Gaussians, 360x90 rays): project+bin_sort+"
                           "render_fwd+loss_spectrum+render_bwd+grad_stats+sgd_step, loss (1-l1-l2) L1 + l1 SSIM + "
                           "l2 Fourier "
                           f"with l1={lam1}, l2={lam2} against the spectrum of a perturbed room",
               "iterations_per_s": 1.0 / t_it, "ms_per_iteration": t_it * 1e3,
               "timing": f"{steps} eager iterations after {1 + args.warmup} untimed ones, wall clock between "
                         "synchronisations",
               "loss_first_last": [first_loss[0], float(lossb[0, 0])],
               "kernel_ms": {"loss_spectrum": t_loss * 1e3, "sgd_step": t_sgd * 1e3},
               "sgd_roofline": {"bound": "hbm", "achieved": sgd_bytes / t_sgd / 1e9, "peak": PEAK_HBM / 1e9,
                                "unit": "GB/s", "frac": sgd_bytes / t_sgd / PEAK_HBM, "traffic": None,
                                "bytes_per_launch": sgd_bytes,
                                "timing": "HIP events around the call on its stream (includes one launch gap)"},
               "splats_within_capacity": bool(ok),
               "density_control": {"ms": t_dc * 1e3, "gaussians_in": G_, "gaussians_out": n_out, "clones": n_clone,
                                   "splits": n_split, "pruned": n_pruned,
                                   "statistics": f"mean gradients accumulated over the {1 + args.warmup + steps} "
                                                 "iterations above",
                                   "timing": "median of 5 calls, HIP events around the call (count, scan and apply "
                                             "kernels plus the binding's allocations)",
                                   "roofline": {"bound": "hbm", "achieved": dc_bytes / t_dc / 1e9,
                                                "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                                "frac": dc_bytes / t_dc / PEAK_HBM, "traffic": None,
                                                "bytes_per_launch": dc_bytes}}}
        del prob, bufs, target, gsig
        torch.cuda.empty_cache()
        return out

    step_stats = {}
    eager = {}
    work = set(args.workloads.split(","))
    # ---- plain: one pair per launch sequence (the headline step) -------------
    t_step = t_fwd_only = t_fwd_k = t_bwd_k = None
    roof = None
    if "plain" in work:
        t_step, t_fwd_only, t_fwd_k, t_bwd_k, roof = run_plain()

    # ---- batched: all pairs of a batch in one hipGraph replay -----------------
    batched = None
    if args.batched != "none":
        batched = {}
        small = args.batched == "small"
        if "fwd_500k" in work:
            b4 = synth.batched(n=100_000 if small else 500_000, n_pairs=16 if small else args.batched_pairs)
            batched["fwd_500k"] = run_batched(b4, grad=False, label="batched forward: {} pairs over one {}-Gaussian "
                                              "room, 360x90 rays, 5 GHz".format(len(b4.pairs), b4.scenes[0].n))
            del b4
        if "uneven" in work:
            b5 = synth.batched_uneven(n_scenes=4 if small else 16, n_hi=100_000 if small else 1_000_000,
                                      pairs_hi=8 if small else 64)
            batched["uneven_fwd_bwd"] = run_batched(
                b5, grad=True, label="batched uneven fwd+bwd: {} scenes ({}-{} Gaussians), {} pairs, carriers "
                "2.4/5/5.8 GHz, 360x90 rays".format(len(b5.scenes), min(s_.n for s_ in b5.scenes),
                                                    max(s_.n for s_ in b5.scenes), len(b5.pairs)))
            del b5

    multi = run_multi() if "multi" in work else None
    train = run_train() if "train" in work else None

    cpu = None
    if not args.no_cpu_baseline and "plain" in work:
        cpu = cpu_baseline(scene, pair, grid)

    out = {
        "metric": METRIC,
        "value": None if t_step is None else 1.0 / t_step,
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None if t_step is None else t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-scale differentiated step: 200k Gaussians in a 10x8x3 m room, one TX/RX "
                               "pair, 360x90 rays, 5 GHz, FLE L=2; project+bin_sort+render_fwd+render_bwd",
                   "gaussians": args.gaussians, "rays": "360x90", "pairs": 1, "tile": args.tile,
                   "lanes_per_ray": args.lanes, "footprint": args.footprint},
        "step_timing": "hipGraph replays of the captured step (project, bin_sort, render_fwd, render_bwd)",
        "step_ms_events": step_stats or None,
        "eager": eager or None,
        "plain": None if not eager else {"spectra_per_s": eager["spectra_per_s"], "ms_per_step": eager["ms_per_step"],
                                         "timing": "eager launches of project, bin_sort, render_fwd, render_bwd "
                                                   "for one pair on one stream, wall clock between "
                                                   "synchronisations (the plain per-pair launch)"},
        "fwd_only": None if t_fwd_only is None else {"spectra_per_s": 1.0 / t_fwd_only, "ms": t_fwd_only * 1e3},
        "kernels_ms": None if t_fwd_k is None else {"render_fwd": t_fwd_k * 1e3, "render_bwd": t_bwd_k * 1e3},
        "batched": batched,
        "multi_carrier": multi,
        "train_step": train,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
