"""CPU checks of the C ABI: the library loads, exports every function the
header declares, its structures match the ctypes mirrors, and host-side
validation rejects bad problems before anything is launched (no GPU)."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsrf.h")

from paper_2502_01826_amd import _lib  # noqa: E402
from paper_2502_01826_amd._lib import (GsrfDensityParams, GsrfGrid, GsrfLayout, GsrfPair, GsrfProblem,  # noqa: E402
                                      GsrfSgdLr)


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsrf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 9
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_struct_layout_matches_header():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "gsrf.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("sizeof_grid %zu\nsizeof_pair %zu\nsizeof_problem %zu\nsizeof_layout %zu\n",
         sizeof(gsrf_grid), sizeof(gsrf_pair), sizeof(gsrf_problem), sizeof(gsrf_layout));
  P(gsrf_pair, freq_hz); P(gsrf_pair, scene);
  P(gsrf_problem, n_gauss); P(gsrf_problem, grid); P(gsrf_problem, splat_capacity); P(gsrf_problem, workspace_bytes);
  P(gsrf_layout, n_records); P(gsrf_layout, n_tiles_az);
  printf("sizeof_sgd_lr %zu\n", sizeof(gsrf_sgd_lr));
  P(gsrf_sgd_lr, mean_steps); P(gsrf_sgd_lr, coeff);
  printf("sizeof_density %zu\n", sizeof(gsrf_density_params));
  P(gsrf_density_params, clone_step); P(gsrf_density_params, prune);
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        vals = dict(l.split() for l in subprocess.run([exe], capture_output=True, text=True).stdout.splitlines())
    assert int(vals["sizeof_grid"]) == ctypes.sizeof(GsrfGrid)
    assert int(vals["sizeof_pair"]) == ctypes.sizeof(GsrfPair) == 40
    assert int(vals["sizeof_problem"]) == ctypes.sizeof(GsrfProblem)
    assert int(vals["sizeof_layout"]) == ctypes.sizeof(GsrfLayout)
    assert int(vals["gsrf_pair.freq_hz"]) == GsrfPair.freq_hz.offset
    assert int(vals["gsrf_pair.scene"]) == GsrfPair.scene.offset
    for f in ("n_gauss", "grid", "splat_capacity", "workspace_bytes"):
        assert int(vals[f"gsrf_problem.{f}"]) == getattr(GsrfProblem, f).offset
    for f in ("n_records", "n_tiles_az"):
        assert int(vals[f"gsrf_layout.{f}"]) == getattr(GsrfLayout, f).offset
    assert int(vals["sizeof_sgd_lr"]) == ctypes.sizeof(GsrfSgdLr)
    for f in ("mean_steps", "coeff"):
        assert int(vals[f"gsrf_sgd_lr.{f}"]) == getattr(GsrfSgdLr, f).offset
    assert int(vals["sizeof_density"]) == ctypes.sizeof(GsrfDensityParams)
    for f in ("clone_step", "prune"):
        assert int(vals[f"gsrf_density_params.{f}"]) == getattr(GsrfDensityParams, f).offset


def _host_problem(n_gauss=10, n_pairs=2, grid=None, cap=1000):
    offs = np.array([0, n_gauss], np.int64)
    ps = np.zeros(n_pairs, np.int32)
    p = GsrfProblem()
    p.n_gauss = n_gauss
    p.n_scenes = 1
    p.scene_offsets = offs.ctypes.data
    p.pair_scene = ps.ctypes.data
    p.n_pairs = n_pairs
    p.grid = grid or GsrfGrid(360, 90, 0.0, 1.5707963, 2, 1.0, 1e-4, 0.99, 16, 16, 1)
    p.splat_capacity = cap
    return p, (offs, ps)


def test_workspace_size_and_layout():
    L = _lib.lib()
    p, keep = _host_problem()
    n = ctypes.c_size_t()
    assert L.gsrf_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    lay = GsrfLayout()
    assert L.gsrf_layout_of(ctypes.byref(p), ctypes.byref(lay)) == 0
    assert lay.n_records == 20 and lay.n_tiles == 23 * 6 and lay.n_tiles_az == 23
    offs = [lay.rec_key, lay.rec_rect, lay.rec_base, lay.counters, lay.sorted_klo, lay.sorted_val,
            lay.tile_start, lay.tile_end]
    assert all(o % 256 == 0 and o < n.value for o in offs)
    # bigger capacity, bigger workspace: 24 bytes per splat (emitted key/id
    # pairs, sorted key and id arrays, long-bucket scratch key and id), each
    # array rounded to 256 bytes
    p2, keep2 = _host_problem(cap=100000)
    n2 = ctypes.c_size_t()
    assert L.gsrf_workspace_size(ctypes.byref(p2), ctypes.byref(n2)) == 0
    assert n2.value - n.value >= (100000 - 1000) * 24 - 5 * 256


@pytest.mark.parametrize("mutate,needle", [
    (lambda p: setattr(p.grid, "tile_w", 5), "tile"),
    (lambda p: (setattr(p.grid, "tile_w", 8), setattr(p.grid, "tile_h", 4), setattr(p.grid, "lanes_per_ray", 1)),
     "32-ray tiles"),
    (lambda p: setattr(p.grid, "fle_L", 7), "fle_L"),
    (lambda p: setattr(p.grid, "lanes_per_ray", 3), "lanes_per_ray"),
    (lambda p: setattr(p.grid, "footprint", 2), "footprint"),
    (lambda p: setattr(p.grid, "depth_order", 2), "depth_order"),
    (lambda p: setattr(p.grid, "fle_eval", -1), "fle_eval"),
    (lambda p: setattr(p.grid, "transmittance", 3), "transmittance"),
    (lambda p: (setattr(p.grid, "transmittance", 1), setattr(p.grid, "lanes_per_ray", 1)), "two-phase"),
    (lambda p: (setattr(p.grid, "depth_order", 1), setattr(p.grid, "lanes_per_ray", 0),
                setattr(p, "hit_capacity", -5)), "hit_capacity"),
    (lambda p: setattr(p.grid, "n_az", 0), "grid size"),
    (lambda p: setattr(p.grid, "alpha_max", 1.0), "alpha_max"),
    (lambda p: setattr(p.grid, "el_hi", -0.5), "elevation"),
    (lambda p: setattr(p, "splat_capacity", -1), "splat_capacity"),
    (lambda p: setattr(p, "n_scenes", 0), "n_scenes"),
])
def test_validation_rejects_bad_problems(mutate, needle):
    L = _lib.lib()
    p, keep = _host_problem()
    mutate(p)
    n = ctypes.c_size_t()
    st = L.gsrf_workspace_size(ctypes.byref(p), ctypes.byref(n))
    assert st == _lib.GSRF_EINVAL
    assert needle in L.gsrf_last_error().decode()


def test_entry_points_reject_missing_device_pointers_without_launching():
    L = _lib.lib()
    p, keep = _host_problem()
    # no device pointers / workspace: every entry point must refuse on the host
    assert L.gsrf_project(ctypes.byref(p), None) == _lib.GSRF_EINVAL
    assert L.gsrf_bin_sort(ctypes.byref(p), None) == _lib.GSRF_EINVAL
    assert L.gsrf_render_fwd(ctypes.byref(p), None, None, None, None) == _lib.GSRF_EINVAL
    assert L.gsrf_render_bwd(ctypes.byref(p), *([None] * 9)) == _lib.GSRF_EINVAL
    n = ctypes.c_int64()
    assert L.gsrf_splat_count(ctypes.byref(p), ctypes.byref(n), None) == _lib.GSRF_EINVAL
    assert L.gsrf_status_str(2) == b"GSRF_ECAPACITY"


def test_multi_carrier_forward_validates_before_launching():
    L = _lib.lib()
    p, keep = _host_problem()
    assert L.gsrf_render_fwd_multi(ctypes.byref(p), 0, 1e6, None, None, None) == _lib.GSRF_EINVAL
    assert "n_freq" in L.gsrf_last_error().decode()
    assert L.gsrf_render_fwd_multi(ctypes.byref(p), 4, -1.0, None, None, None) == _lib.GSRF_EINVAL
    assert "freq_step" in L.gsrf_last_error().decode()
    p.grid.lanes_per_ray = 2
    assert L.gsrf_render_fwd_multi(ctypes.byref(p), 4, 1e6, None, None, None) == _lib.GSRF_ENOTSUP
    p.grid.lanes_per_ray = 0
    # valid request, but no device workspace: refused on the host
    assert L.gsrf_render_fwd_multi(ctypes.byref(p), 4, 1e6, None, None, None) == _lib.GSRF_EINVAL


def test_pair_packing_matches_struct():
    from paper_2502_01826_amd import pack_pairs
    import synth
    b = synth.tiny()
    a = pack_pairs(b.pairs)
    raw = a.view(np.uint8).tobytes()
    s = GsrfPair.from_buffer_copy(raw[:40])
    assert list(s.rx) == list(b.pairs[0].rx.astype(np.float32)) and s.freq_hz == 2.4e9 and s.scene == 0


def test_training_steps_validate_before_launching():
    L = _lib.lib()
    nb = ctypes.c_size_t()
    assert L.gsrf_loss_workspace_size(3, 90, 360, ctypes.byref(nb)) == _lib.GSRF_OK
    assert nb.value == 3 * (6 * 12) * 3 * 8          # 16 x 32 pixel tiles, three FP64 sums each
    assert L.gsrf_loss_workspace_size(0, 90, 360, ctypes.byref(nb)) == _lib.GSRF_OK and nb.value == 0
    assert L.gsrf_loss_workspace_size(1, 0, 360, ctypes.byref(nb)) == _lib.GSRF_EINVAL
    # missing device pointers, a NaN weight, bad sizes: refused on the host
    assert L.gsrf_loss_spectrum(None, None, 1, 9, 36, 1.0, 0.2, 0.1, None, None, None, None) == _lib.GSRF_EINVAL
    assert L.gsrf_loss_spectrum(None, None, 1, 9, 36, 1.0, float("nan"), 0.1, None, None, None, None) == \
        _lib.GSRF_EINVAL
    assert "lambda" in L.gsrf_last_error().decode()
    assert L.gsrf_loss_spectrum(None, None, 1, 9, 36, 0.0, 0.2, 0.1, None, None, None, None) == _lib.GSRF_EINVAL
    assert "power_scale" in L.gsrf_last_error().decode()
    assert L.gsrf_loss_spectrum(None, None, -1, 9, 36, 1.0, 0.2, 0.1, None, None, None, None) == _lib.GSRF_EINVAL
    # no pairs: nothing to do, nothing launched
    assert L.gsrf_loss_spectrum(None, None, 0, 9, 36, 1.0, 0.2, 0.1, None, None, None, None) == _lib.GSRF_OK
    assert L.gsrf_loss_single(None, None, 2, 7, None, None, None) == _lib.GSRF_EINVAL
    assert "kind" in L.gsrf_last_error().decode()
    assert L.gsrf_loss_single(None, None, 2, _lib.GSRF_LOSS_RSSI_DB, None, None, None) == _lib.GSRF_EINVAL
    assert L.gsrf_loss_single(None, None, 0, _lib.GSRF_LOSS_COMPLEX_L2, None, None, None) == _lib.GSRF_OK
    lr = GsrfSgdLr(1.6e-4, 1.6e-6, 30000, 0.01, 0.005, 0.01, 0.0025)
    assert L.gsrf_sgd_step(10, 2, *([None] * 10), ctypes.byref(lr), 0, None) == _lib.GSRF_EINVAL
    assert L.gsrf_sgd_step(0, 2, *([None] * 10), ctypes.byref(lr), 0, None) == _lib.GSRF_OK
    assert L.gsrf_sgd_step(0, 2, *([None] * 10), None, 0, None) == _lib.GSRF_EINVAL
    assert L.gsrf_sgd_step(0, 2, *([None] * 10), ctypes.byref(lr), -1, None) == _lib.GSRF_EINVAL
    assert L.gsrf_sgd_step(0, 7, *([None] * 10), ctypes.byref(lr), 0, None) == _lib.GSRF_EINVAL
    bad = GsrfSgdLr(0.0, 1.6e-6, 30000, 0.01, 0.005, 0.01, 0.0025)
    assert L.gsrf_sgd_step(0, 2, *([None] * 10), ctypes.byref(bad), 0, None) == _lib.GSRF_EINVAL
    bad = GsrfSgdLr(1.6e-4, 1.6e-6, 30000, -0.01, 0.005, 0.01, 0.0025)
    assert L.gsrf_sgd_step(0, 2, *([None] * 10), ctypes.byref(bad), 0, None) == _lib.GSRF_EINVAL


def test_density_control_validates_before_launching():
    L = _lib.lib()
    nb = ctypes.c_size_t()
    assert L.gsrf_density_workspace_size(200_000, ctypes.byref(nb)) == _lib.GSRF_OK
    assert nb.value == (200_000 // 1024 + 1 + 1) * 8
    dp = GsrfDensityParams(0.0002, 10.0, 0.004, 1.6, 1.6e-4, 1, 1)
    args = lambda n, cap, p: (n, 2, *([None] * 8), ctypes.byref(p) if p else None, cap, *([None] * 10))
    assert L.gsrf_density_control(*args(10, 20, dp)) == _lib.GSRF_EINVAL                 # no device pointers
    assert L.gsrf_density_control(*args(10, 19, dp)) == _lib.GSRF_EINVAL                 # capacity < 2 G
    assert "out_capacity" in L.gsrf_last_error().decode()
    assert L.gsrf_density_control(*args(10, 20, None)) == _lib.GSRF_EINVAL
    bad = GsrfDensityParams(0.0002, 10.0, 0.004, 1.0, 1.6e-4, 1, 1)                      # phi must exceed 1
    assert L.gsrf_density_control(*args(10, 20, bad)) == _lib.GSRF_EINVAL
    assert L.gsrf_grad_stats_accumulate(10, None, None, None, None) == _lib.GSRF_EINVAL
    assert L.gsrf_grad_stats_accumulate(0, None, None, None, None) == _lib.GSRF_OK


def test_tune_cache_round_trip(tmp_path):
    """The autotuner's cache: keys separate architecture, size class, grid,
    FLE degree, switches, direction and candidates; results survive a reload."""
    from paper_2502_01826_amd.batch import TuneCache, TuneResult, tune_key
    from synth import Grid
    g = Grid(n_az=360, n_el=90, fle_L=2)
    cand = ((8, 4, 0), (8, 8, 0))
    k = tune_key(g, 500_000, 256, False, cand, arch="gfx950")
    assert k == tune_key(g, 480_000, 250, False, cand, arch="gfx950")           # same size class
    assert k != tune_key(g, 500_000, 256, True, cand, arch="gfx950")           # adjoint included
    assert k != tune_key(g, 2_000_000, 256, False, cand, arch="gfx950")        # 4x the Gaussians
    assert k != tune_key(g, 500_000, 256, False, cand, arch="gfx942")          # another device
    assert k != tune_key(Grid(n_az=360, n_el=90, fle_L=3), 500_000, 256, False, cand, arch="gfx950")
    assert k != tune_key(g, 500_000, 256, False, cand[:1], arch="gfx950")
    path = str(tmp_path / "tune.json")
    c = TuneCache(path)
    assert c.get(k) is None
    c.put(k, TuneResult(best=(8, 8, 0), seconds={(8, 4, 0): 0.024, (8, 8, 0): 0.019}))
    r = TuneCache(path).get(k)
    assert r.cached and r.best == (8, 8, 0) and r.seconds == {(8, 4, 0): 0.024, (8, 8, 0): 0.019}


def test_multi_carrier_adjoint_validates_before_launching():
    L = _lib.lib()
    p, keep = _host_problem()
    none8 = [None] * 8
    assert L.gsrf_render_bwd_multi(ctypes.byref(p), 0, 1e6, *none8) == _lib.GSRF_EINVAL
    assert "n_freq" in L.gsrf_last_error().decode()
    assert L.gsrf_render_bwd_multi(ctypes.byref(p), 4097, 1e6, *none8) == _lib.GSRF_EINVAL
    assert L.gsrf_render_bwd_multi(ctypes.byref(p), 4, float("nan"), *none8) == _lib.GSRF_EINVAL
    p.grid.lanes_per_ray = 1
    assert L.gsrf_render_bwd_multi(ctypes.byref(p), 4, 1e6, *none8) == _lib.GSRF_ENOTSUP
    p.grid.lanes_per_ray = 0
    p.grid.transmittance = 1
    assert L.gsrf_render_bwd_multi(ctypes.byref(p), 4, 1e6, *none8) == _lib.GSRF_ENOTSUP
    p.grid.transmittance = 0
    assert L.gsrf_render_bwd_multi(ctypes.byref(p), 4, 1e6, *none8) == _lib.GSRF_EINVAL   # no workspace
