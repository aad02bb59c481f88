"""Seeded synthetic inputs for the GSRF hot path.

This module is shared by the tests, the benchmark and the smoke run. It only
draws random numbers and packs them: it holds none of the rendering
arithmetic, so the FP64 oracle and the HIP path can both consume its output
without sharing any of the method's code.

Every draw is made in FP64 with ``numpy.random.default_rng([cfg_id, stream])``
in a fixed order (means, log-scales, quaternions, opacity logits, FLE
coefficients, then pairs with RX before TX) and cast to FP32, so both sides
see identical FP32 inputs.

The distributions follow the synthetic-room recipe used throughout:
means uniform in an axis-aligned room, log-scales ~ N(-2.5, 0.3) per axis,
quaternions normalised N(0, I4), opacity logits ~ N(0, 1), complex
coefficients ~ CN(0, 0.1) (real and imaginary parts each N(0, 0.05)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GHZ = 1.0e9


@dataclass
class Grid:
    """Receiver ray grid and render constants (mirrors the C ``gsrf_grid``)."""

    n_az: int = 360
    n_el: int = 90
    el_lo: float = 0.0
    el_hi: float = math.pi / 2
    fle_L: int = 2
    r_rx: float = 1.0
    t_min: float = 1.0e-4
    alpha_max: float = 0.99
    tile_w: int = 16
    tile_h: int = 16
    lanes_per_ray: int = 0
    footprint: int = 0          # 0: exact bounding cap, 1: the paper's 3 sqrt(lambda_max) footprint
    depth_order: int = 0        # 0: per-Gaussian distance key, 1: per-ray chord-midpoint order
    fle_eval: int = 0           # 0: radiance at the ray's direction, 1: at the Gaussian's direction
    transmittance: int = 0      # 0: 1 - o G(x_mid), 1: chord form exp(-alpha dt)

    @property
    def K(self) -> int:
        return (self.fle_L + 1) ** 2

    @property
    def n_tiles_az(self) -> int:
        return -(-self.n_az // self.tile_w)

    @property
    def n_tiles_el(self) -> int:
        return -(-self.n_el // self.tile_h)

    @property
    def n_tiles(self) -> int:
        return self.n_tiles_az * self.n_tiles_el

    def with_tiles(self, tile_w: int, tile_h: int) -> "Grid":
        g = Grid(**self.__dict__)
        g.tile_w, g.tile_h = tile_w, tile_h
        return g


@dataclass
class Scene:
    """One scene's Gaussian parameters, FP32 numpy arrays."""

    means: np.ndarray        # [N,3]
    log_scales: np.ndarray   # [N,3]
    quats: np.ndarray        # [N,4] (w,x,y,z), unit length as drawn
    logits: np.ndarray       # [N]
    coeffs: np.ndarray       # [N,K,2] (re, im)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx], self.log_scales[idx], self.quats[idx],
                     self.logits[idx], self.coeffs[idx])


@dataclass
class Pair:
    rx: np.ndarray   # [3] FP32
    tx: np.ndarray   # [3] FP32
    freq_hz: float
    scene: int = 0


@dataclass
class Batch:
    """Several scenes (concatenated) and the TX/RX pairs that query them."""

    scenes: list
    pairs: list
    grid: Grid = field(default_factory=Grid)

    def concat(self) -> tuple[Scene, np.ndarray]:
        offs = np.zeros(len(self.scenes) + 1, dtype=np.int64)
        for i, s in enumerate(self.scenes):
            offs[i + 1] = offs[i] + s.n
        cat = Scene(*(np.concatenate([getattr(s, f) for s in self.scenes], axis=0)
                      for f in ("means", "log_scales", "quats", "logits", "coeffs")))
        return cat, offs


def draw_scene(rng: np.random.Generator, n: int, room, K: int) -> Scene:
    room = np.asarray(room, dtype=np.float64)
    means = rng.uniform(0.0, 1.0, size=(n, 3)) * room
    log_scales = rng.normal(-2.5, 0.3, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.normal(0.0, 1.0, size=(n,))
    coeffs = rng.normal(0.0, math.sqrt(0.05), size=(n, K, 2))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f32(means), f32(log_scales), f32(q), f32(logits), f32(coeffs))


def draw_pair(rng: np.random.Generator, room, freq_hz: float, scene: int = 0) -> Pair:
    room = np.asarray(room, dtype=np.float64)
    rx = rng.uniform(0.0, 1.0, size=3) * room
    tx = rng.uniform(0.0, 1.0, size=3) * room
    return Pair(rx.astype(np.float32), tx.astype(np.float32), float(freq_hz), scene)


# --------------------------------------------------------------------------
# The five workloads, cfg ids 1..5 in this order: tiny parity case,
# paper-scale forward, differentiated step, batched forward, batched uneven
# forward+backward.
# --------------------------------------------------------------------------

def tiny(seed_stream: int = 0, n: int = 2000, grid: Grid | None = None) -> Batch:
    """2,000 Gaussians in a 4x4x3 m room, TX (1,1,1.5), RX (3,2,1.2), 2.4 GHz, 36x9 rays."""
    grid = grid or Grid(n_az=36, n_el=9, fle_L=2)
    rng = np.random.default_rng([1, seed_stream])
    sc = draw_scene(rng, n, (4.0, 4.0, 3.0), grid.K)
    p = Pair(np.array([3.0, 2.0, 1.2], np.float32), np.array([1.0, 1.0, 1.5], np.float32), 2.4 * GHZ)
    return Batch([sc], [p], grid)


def paper_scale(seed_stream: int = 0, n: int = 200_000, grid: Grid | None = None) -> Batch:
    """200k Gaussians in a 10x8x3 m room, one uniform TX/RX pair, 360x90 rays, 5 GHz."""
    grid = grid or Grid(n_az=360, n_el=90, fle_L=2)
    rng = np.random.default_rng([2, seed_stream])
    room = (10.0, 8.0, 3.0)
    sc = draw_scene(rng, n, room, grid.K)
    p = draw_pair(rng, room, 5.0 * GHZ)
    return Batch([sc], [p], grid)


def training_step(seed_stream: int = 0, n: int = 200_000, grid: Grid | None = None):
    """Paper-scale scene plus a perturbed copy whose render is the L2 target.

    Returns (batch, perturbed_scene); every parameter entry of the copy gets
    N(0, 0.05) noise (quaternions are renormalised afterwards).
    """
    b = paper_scale(seed_stream, n, grid)
    rng = np.random.default_rng([3, seed_stream])
    s = b.scenes[0]
    noisy = lambda a: (a.astype(np.float64) + rng.normal(0.0, 0.05, size=a.shape)).astype(np.float32)
    q = noisy(s.quats).astype(np.float64)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    pert = Scene(noisy(s.means), noisy(s.log_scales), q.astype(np.float32), noisy(s.logits), noisy(s.coeffs))
    return b, pert


def batched(seed_stream: int = 0, n: int = 500_000, n_pairs: int = 256, grid: Grid | None = None) -> Batch:
    """One 500k-Gaussian room, 256 uniform TX/RX pairs, 360x90 rays, 5 GHz."""
    grid = grid or Grid(n_az=360, n_el=90, fle_L=2)
    rng = np.random.default_rng([4, seed_stream])
    room = (10.0, 8.0, 3.0)
    sc = draw_scene(rng, n, room, grid.K)
    pairs = [draw_pair(rng, room, 5.0 * GHZ) for _ in range(n_pairs)]
    return Batch([sc], pairs, grid)


def batched_uneven(seed_stream: int = 0, n_scenes: int = 16, n_lo: int = 20_000, n_hi: int = 1_000_000,
                   pairs_lo: int = 8, pairs_hi: int = 64, grid: Grid | None = None) -> Batch:
    """16 scenes with log-uniform sizes in [20k, 1M], 8-64 pairs each, carriers per pair."""
    grid = grid or Grid(n_az=360, n_el=90, fle_L=2)
    rng = np.random.default_rng([5, seed_stream])
    room = (10.0, 8.0, 3.0)
    sizes = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_scenes))).astype(np.int64)
    counts = rng.integers(pairs_lo, pairs_hi + 1, size=n_scenes)
    scenes, pairs = [], []
    for s in range(n_scenes):
        scenes.append(draw_scene(rng, int(sizes[s]), room, grid.K))
        for _ in range(int(counts[s])):
            f = float(rng.choice([2.4, 5.0, 5.8])) * GHZ
            pairs.append(draw_pair(rng, room, f, scene=s))
    return Batch(scenes, pairs, grid)


def cotangent(shape, seed: int, stream: int = 0) -> np.ndarray:
    """Seeded upstream gradient, CN(0,1) as real views, FP32."""
    rng = np.random.default_rng([9, seed, stream])
    return rng.normal(0.0, math.sqrt(0.5), size=tuple(shape) + (2,)).astype(np.float32)


def spectra(n_pairs: int, n_el: int, n_az: int, seed: int) -> tuple:
    """Seeded stand-ins for a rendered spectrum and a measured one: rays S_uv
    CN(0, 0.5) as real views [P, n_el, n_az, 2] FP32, and a target power
    spectrum [P, n_el, n_az] FP32 that is the power of a second such draw
    smoothed over 3 x 3 neighbours (measured spectra are smooth images)."""
    rng = np.random.default_rng([10, seed])
    sig = rng.normal(0.0, 0.5, size=(n_pairs, n_el, n_az, 2))
    other = rng.normal(0.0, 0.5, size=(n_pairs, n_el, n_az, 2))
    p = (other ** 2).sum(-1)
    pad = np.pad(p, ((0, 0), (1, 1), (1, 1)), mode="edge")
    t = sum(pad[:, i:i + n_el, j:j + n_az] for i in range(3) for j in range(3)) / 9.0
    return sig.astype(np.float32), t.astype(np.float32)
