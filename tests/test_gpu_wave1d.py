"""The fused 1D step: passes of several steps per launch, each workgroup
advancing a window of cells held in LDS (halos of K + 1 cells for K steps),
against the unfused kernels bit for bit.

Both paths evaluate the same point formulas in the same order (no FP
contraction), so every field, every diagnostic record and the final
probabilities agree bit for bit.  The cases cover grids held in one window
(periodic axes wrapping inside it) and grids split into tiles (the windows of
a periodic axion running on around the grid, those of the other boundaries
clipped at the faces), a last tile owning a single cell, every axion boundary,
periodic and Mur EM faces, CW and Gaussian lasers, the moving window, record
cadences that break passes, and batches of runs of different lengths.  The
long runs carry the laser and the axion packet across every tile boundary and
into the far Mur face, where the halos' reach decides the result (the axion
current's E0 x grad phi term reads phi two cells from where B is updated).
"""
import numpy as np
import pytest

from paper_2406_16796_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ["E0Y", "E0Z", "B0Y", "B0Z", "E1Y", "E1Z", "B1Y", "B1Z", "PHI_OLD", "PHI_NEW"]
# cells of a single run's window and the most steps per pass (FP32, FP64);
# batches take windows of 512
WIN = {"f32": (256, 16), "f64": (256, 16)}


@pytest.fixture(scope="module")
def axf():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_16796_amd import axf as A
    A.lib()
    return A


def cfg_1d(n, ax_bc=W.AX_PERIODIC, em=W.EM_MUR, env=W.ENV_CW, pol=1):
    cfg = W.plane_wave_1d(nx=n, steps=0, m=0.3, g=0.02, a0=0.5, ax_bc=ax_bc)
    dx = cfg["dx"][0]
    cfg.update(packet_on=1, pk_amp=0.3, pk_k=1.0, pk_w=8.0, pk_x0=0.6 * n * dx, pk_dir=1, pml_n=30,
               laser_pol=pol)
    if pol == 2:
        cfg["bext"] = [0.0, 0.0, 1.0]
    if env == W.ENV_GAUSS:
        cfg.update(laser_env=W.ENV_GAUSS, fwhm=12.0, t_center=20.0)
    if em == W.EM_PERIODIC:
        cfg.update(em_bc=[W.EM_PERIODIC, 0, 0], laser_on=0, e_amp=0.0)
    return cfg


def k_ok(k, nem=5, nph=6):
    return k >= 2 and k % nem != 0 and k % nph not in (0, 1, nph - 1)


def pick(free, kmax):
    """The runtime's choice of pass length (wave1d_pick)."""
    anyk = 0
    for k in range(min(free, kmax), 1, -1):
        if not k_ok(k):
            continue
        if free - k != 1:
            return k
        anyk = anyk or k
    return anyk


def expected_launches(steps, kmax):
    out, left = 0, steps
    while left > 0:
        k = pick(left, kmax) if left >= 2 else 0
        if k < 2:
            out += 6
            left -= 1
        else:
            out += 1
            left -= k
    return out


def both(axf, cfg, prec, steps, diag_every=0):
    p = axf.F32 if prec == "f32" else axf.F64
    runs = []
    for path in (axf.PATH_PLAIN, axf.PATH_FUSED):
        r = axf.Run(cfg, precision=p, path=path, diag_every=diag_every)
        print("1d n=%d ax=%d em=%d %s path %d steps %d" % (cfg["n"][0], cfg["ax_bc"][0], cfg["em_bc"][0], prec,
                                                           path, steps), flush=True)
        r.step(steps)
        runs.append(r)
    return runs


def assert_same(runs, records=None):
    """Fields and a record of the current state equal bit for bit; `records`
    (the first run's records, read before: reading drains them) equal to the
    second run's."""
    for nm in FIELDS:
        a, b = runs[0].read(nm), runs[1].read(nm)
        assert np.array_equal(a, b), (nm, np.abs(a - b).max())
    ra, rb = runs[0].diag_now(), runs[1].diag_now()
    for key in ("h_phi", "h_em0", "h_em1", "p_gen", "p_conv", "x_laser"):
        assert ra[key] == rb[key], key
    if records is not None:
        db = runs[1].read_diag()
        assert len(records) == len(db) and len(records) > 0
        for x, y in zip(records, db):
            assert x == y


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("ax_bc", [W.AX_PERIODIC, W.AX_REFLECT, W.AX_OUTFLOW, W.AX_PML])
@pytest.mark.parametrize("size", ["one_window", "tiles"])
def test_fused_1d_equals_plain_bitwise(axf, prec, ax_bc, size):
    n = 200 if size == "one_window" else 2500
    runs = both(axf, cfg_1d(n, ax_bc), prec, 301)
    assert runs[1].uses_fused() and not runs[0].uses_fused()
    assert_same(runs)
    # one launch per pass; a single step left over takes the six unfused launches
    assert runs[1].last_step_timing()[1] == expected_launches(301, WIN[prec][1])


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", ["gauss_pol_z", "periodic_em_one_window", "periodic_em_tiles",
                                  "exact_window", "window_plus_one", "last_tile_one_cell", "two_cells"])
def test_fused_1d_shapes_equal_plain_bitwise(axf, prec, case):
    w, kmax = WIN[prec]
    own = w - 2 * (kmax + 1)
    cfg = {
        "gauss_pol_z": lambda: cfg_1d(2000, W.AX_OUTFLOW, env=W.ENV_GAUSS, pol=2),
        "periodic_em_one_window": lambda: cfg_1d(200, W.AX_PERIODIC, em=W.EM_PERIODIC),
        "periodic_em_tiles": lambda: cfg_1d(3 * own + 17, W.AX_PERIODIC, em=W.EM_PERIODIC),
        "exact_window": lambda: cfg_1d(w, W.AX_PERIODIC),
        "window_plus_one": lambda: cfg_1d(w + 1, W.AX_PML),
        "last_tile_one_cell": lambda: cfg_1d(2 * own + 1, W.AX_PERIODIC),
        "two_cells": lambda: cfg_1d(2, W.AX_REFLECT),
    }[case]()
    if case == "two_cells":
        cfg.update(packet_on=0)
    runs = both(axf, cfg, prec, 203)
    assert_same(runs)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("ax_bc", [W.AX_PERIODIC, W.AX_OUTFLOW, W.AX_PML])
def test_laser_across_tiles_bitwise(axf, prec, ax_bc):
    """Three tiles; the CW front (0.95 cells per step) crosses both tile
    boundaries and reaches x_max, the packet leaves through it."""
    w, kmax = WIN[prec]
    own = w - 2 * (kmax + 1)
    n = 2 * own + own // 2
    runs = both(axf, cfg_1d(n, ax_bc), prec, int(1.3 * n))
    assert_same(runs)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_records_break_passes_bitwise(axf, prec):
    """A record every 37 steps: the passes end before each record's step,
    which takes the unfused kernels, and every record is bit-identical."""
    runs = both(axf, cfg_1d(2500, W.AX_OUTFLOW), prec, 401, diag_every=37)
    plain_recs = runs[0].read_diag()
    assert len(plain_recs) == 11
    assert_same(runs, records=plain_recs)
    # the same steps in calls of uneven length
    p = axf.F32 if prec == "f32" else axf.F64
    r = axf.Run(cfg_1d(2500, W.AX_OUTFLOW), precision=p, path=axf.PATH_FUSED, diag_every=37)
    for k in (1, 3, 50, 2, 345):
        r.step(k)
    assert_same([runs[0], r], records=plain_recs)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_moving_window_1d_bitwise(axf, prec):
    cfg = cfg_1d(1500, W.AX_OUTFLOW, env=W.ENV_GAUSS)
    cfg.update(win_cells=8, win_t0=60.0)
    runs = both(axf, cfg, prec, 500)
    assert_same(runs)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batched_1d_passes_equal_runs_alone(axf, prec):
    """Runs of different lengths, boundaries and step counts in one batch:
    passes over every active run at once, each run bit-identical alone."""
    p = axf.F32 if prec == "f32" else axf.F64
    cfgs = [cfg_1d(2500, W.AX_PERIODIC), cfg_1d(300, W.AX_OUTFLOW), cfg_1d(1100, W.AX_PML, env=W.ENV_GAUSS),
            cfg_1d(700, W.AX_PERIODIC, em=W.EM_PERIODIC), cfg_1d(5000, W.AX_REFLECT)]
    steps = [301, 250, 123, 301, 77]
    b = axf.Batch(cfgs, precision=p, diag_every=50)
    b.step(steps)
    for cfg, ns, rb in zip(cfgs, steps, b.runs):
        brecs = rb.read_diag()
        for path in (axf.PATH_PLAIN, axf.PATH_FUSED):
            ra = axf.Run(cfg, precision=p, path=path, diag_every=50)
            ra.step(ns)
            assert_same([rb, ra], records=brecs)
