"""Batched execution: a whole batch of (pair, scene) work items as one
hipGraph replay, and a tile-shape autotuner that picks the launch
configuration by timing replays on the actual workload.

A batch is one ``Problem`` holding every scene (CSR-concatenated) and every
TX/RX pair; project, bin_sort, render_fwd and (optionally) render_bwd each
cover all pairs in one launch sequence, and the sequence is captured once
into a graph.  The splat capacity is fixed before capture (one eager pass
measures it), so a replay never synchronises with the host; a caller whose
inputs change between replays checks ``Problem.splat_count()`` afterwards.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass, field

import torch

from .render import GridSpec, Problem

# Launch configurations the tuner tries: (tile_w, tile_h, lanes_per_ray).
DEFAULT_CANDIDATES = ((8, 4, 0), (8, 8, 0), (16, 8, 0), (16, 16, 0), (32, 8, 0))


class GraphStep:
    """project -> bin_sort -> render_fwd [-> render_bwd] of a Problem, captured in a graph.

    Outputs live in preallocated tensors (``signal``, ``signal_sum``, ``rssi``,
    ``grads``) that every replay overwrites.
    """

    def __init__(self, prob: Problem, grad: bool = False, grad_signal=None, grad_sum=None):
        self.prob, self.grad = prob, grad
        dev, g, P = prob.device, prob.grid, prob.n_pairs
        prob.prepare()                       # sizes the splat buffers (one host sync)
        prob.auto_capacity = False
        self.signal = torch.empty((P, g.n_el, g.n_az, 2), dtype=torch.float32, device=dev)
        self.signal_sum = torch.empty((P, 2), dtype=torch.float32, device=dev)
        self.rssi = torch.empty((P,), dtype=torch.float32, device=dev)
        self.grads = None
        if grad:
            G, K = prob.n_gauss, g.K
            e = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
            self.grads = (e(G, 3), e(G, 3), e(G, 4), e(G), e(G, K, 2))
            self.grad_signal = grad_signal if grad_signal is not None else torch.zeros_like(self.signal)
            self.grad_sum = grad_sum
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):        # one eager pass off the default stream before capture
            self._launch()
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._launch()

    def _launch(self):
        p = self.prob
        p.project()
        p.bin_sort()
        p.render_fwd(self.signal, self.signal_sum, self.rssi)
        if self.grad:
            p.render_bwd(self.signal, self.grad_signal, self.grad_sum, out=self.grads)

    def replay(self):
        self.graph.replay()

    def time(self, iters: int = 5, warmup: int = 1) -> float:
        """Median seconds per replay (HIP events around each replay)."""
        return self.time_stats(iters, warmup)["median"]

    def time_stats(self, iters: int = 50, warmup: int = 10) -> dict:
        """Per-replay seconds from HIP events recorded on the replay stream
        around each replay: median, p10, p90 over `iters` replays after
        `warmup` untimed ones."""
        for _ in range(warmup):
            self.replay()
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(iters)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            self.replay()
            b.record(stream)
        torch.cuda.synchronize()
        ts = sorted(a.elapsed_time(b) * 1e-3 for a, b in ev)
        q = lambda f: ts[min(len(ts) - 1, int(round(f * (len(ts) - 1))))]
        return {"median": q(0.5), "p10": q(0.1), "p90": q(0.9), "n": len(ts)}


@dataclass
class TuneResult:
    best: tuple
    seconds: dict = field(default_factory=dict)     # candidate -> median seconds per replay
    cached: bool = False                            # taken from a TuneCache without timing


def tune_key(grid, n_gauss: int, n_pairs: int, grad: bool, candidates, arch: str | None = None) -> str:
    """Cache key of a tuning result: the device's architecture, the batch's
    size class (powers of two of the Gaussian and pair counts), the ray grid,
    the FLE degree, the binning and paper-literal switches, whether the
    adjoint is included, and the candidate set."""
    g = GridSpec.of(grid)
    if arch is None:
        props = torch.cuda.get_device_properties(torch.cuda.current_device())
        arch = getattr(props, "gcnArchName", props.name)
    bucket = lambda x: int(round(math.log2(max(1, x))))
    cand = ";".join(f"{a}x{b}/{c}" for a, b, c in candidates)
    return (f"{arch}|G2^{bucket(n_gauss)}|P2^{bucket(n_pairs)}|{g.n_az}x{g.n_el}|L{g.fle_L}|"
            f"fp{g.footprint}|v{g.depth_order}{g.fle_eval}{g.transmittance}|{'bwd' if grad else 'fwd'}|{cand}")


class TuneCache:
    """Tuning results by ``tune_key``, kept in memory and, when a path is
    given, in a JSON file (read at construction, rewritten on every put)."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.entries = {}
        if path and os.path.exists(path):
            try:
                with open(path) as fh:
                    self.entries = json.load(fh)
            except (OSError, ValueError):
                self.entries = {}

    @staticmethod
    def default_path() -> str:
        return os.environ.get("GSRF_TUNE_CACHE",
                              os.path.join(os.path.expanduser("~"), ".cache", "gsrf", "tune.json"))

    def get(self, key: str):
        e = self.entries.get(key)
        if e is None:
            return None
        return TuneResult(best=tuple(e["best"]),
                          seconds={tuple(int(x) for x in k.split(",")): v for k, v in e["seconds"].items()},
                          cached=True)

    def put(self, key: str, res: TuneResult):
        self.entries[key] = {"best": list(res.best),
                             "seconds": {",".join(str(x) for x in k): v for k, v in res.seconds.items()}}
        if self.path:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(self.entries, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def autotune(build, grid, candidates=DEFAULT_CANDIDATES, grad: bool = False, iters: int = 3,
             make_grad=None, cache: TuneCache | None = None, size: tuple | None = None) -> TuneResult:
    """Time one graph replay per launch configuration and return the fastest.

    ``build(grid)`` returns a fresh Problem for a grid; ``make_grad(prob)``
    returns (grad_signal, grad_sum) when ``grad``.  Each candidate's problem is
    released before the next is built, so peak memory is one batch.  With a
    ``cache`` and ``size`` = (Gaussians, pairs), a result stored under the
    batch's ``tune_key`` is returned without timing, and a new one is stored.
    """
    key = tune_key(grid, size[0], size[1], grad, candidates) if (cache is not None and size) else None
    if key is not None:
        hit = cache.get(key)
        if hit is not None:
            return hit
    res = TuneResult(best=None)
    base = GridSpec.of(grid)
    for tw, th, lanes in candidates:
        g = GridSpec(**{**base.__dict__, "tile_w": tw, "tile_h": th, "lanes_per_ray": lanes})
        prob = build(g)
        gs, gsum = make_grad(prob) if (grad and make_grad) else (None, None)
        step = GraphStep(prob, grad, gs, gsum)
        res.seconds[(tw, th, lanes)] = step.time(iters=iters)
        del step, prob
        torch.cuda.empty_cache()
    res.best = min(res.seconds, key=res.seconds.get)
    if key is not None:
        cache.put(key, res)
    return res
