"""The two-step pass of the 2D wavefront step (temporal blocking) against the
one-step pass, through the C ABI.

A pass advances the interior two steps with the same point formulas in the
same order as two one-step passes, and the boundary frame with two one-step
launches, so fields, diagnostic records and probabilities must be the same
bits.  The one-step pass is itself tied to the oracle by the parity tests; one
two-step run is also compared with the oracle directly.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2406_16796_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ["E0X", "E0Y", "E0Z", "B0X", "B0Y", "B0Z", "E1X", "E1Y", "E1Z", "B1X", "B1Y", "B1Z",
          "PHI_OLD", "PHI_NEW"]


@pytest.fixture(scope="module")
def axf():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_16796_amd import axf as A
    A.lib()
    return A


def grid_2d(nx, ny, ax_bc, pml_n=8, seed=5):
    """A laser pulse entering through x_min, an axion packet moving against it
    inside the B slab: every component nonzero within a few steps."""
    cfg = W.gaussian_2d(n=nx, m=0.25, g=0.03, a0=0.5, waist_lam=1.5, fwhm_lam=1.5,
                        slab=(12, nx - 12), ax_bc=ax_bc, seed=seed)
    dx = cfg["dx"][0]
    cfg.update(n=[nx, ny, 1], y_c=0.5 * ny * dx, t_center=2.0, pml_n=pml_n, packet_on=1, pk_amp=0.2,
               pk_k=1.0, pk_w=3.0, pk_x0=0.55 * nx * dx, pk_y0=0.45 * ny * dx, pk_dir=-1)
    return cfg


def run_steps(axf, monkeypatch, cfg, prec, counts, pair, diag_every=0, ci=None):
    monkeypatch.setenv("AXF_WAVE_PAIR", "1" if pair else "0")
    if ci:
        monkeypatch.setenv("AXF_PAIR_CHUNK", str(ci))
    else:
        monkeypatch.delenv("AXF_PAIR_CHUNK", raising=False)
    run = axf.Run(dict(cfg, diag_every=diag_every), precision=prec, path=axf.PATH_FUSED)
    launches = 0
    for n in counts:
        run.step(n)
        launches += run.last_step_timing()[1]
    monkeypatch.delenv("AXF_WAVE_PAIR")
    return run, launches


def assert_same(a, b, label):
    for nm in FIELDS:
        x, y = a.read(nm), b.read(nm)
        assert np.array_equal(x, y), (label, nm, float(np.abs(x - y).max()))
    assert a.read_diag() == b.read_diag(), label
    assert a.diag_now() == b.diag_now(), label


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("bc", ["periodic", "outflow", "pml", "reflect"])
def test_pair_equals_single_bitwise(axf, monkeypatch, prec, bc):
    code = {"periodic": W.AX_PERIODIC, "outflow": W.AX_OUTFLOW, "pml": W.AX_PML, "reflect": W.AX_REFLECT}[bc]
    p = axf.F32 if prec == "f32" else axf.F64
    cfg = grid_2d(301, 213, code)
    counts = [1, 44, 17, 2]          # odd starts, diagnostics every 10 steps break pairs
    two, n2 = run_steps(axf, monkeypatch, cfg, p, counts, True, diag_every=10)
    one, n1 = run_steps(axf, monkeypatch, cfg, p, counts, False, diag_every=10)
    assert n1 == sum(counts)
    assert n2 < 0.75 * sum(counts), n2            # most steps went two at a time
    assert_same(two, one, "%s %s" % (prec, bc))


@pytest.mark.parametrize("ci", [8, 24, 32])
def test_pair_interior_chunks_bitwise(axf, monkeypatch, ci):
    cfg = grid_2d(420, 331, W.AX_PML, pml_n=20, seed=11)
    two, n2 = run_steps(axf, monkeypatch, cfg, axf.F32, [60], True, ci=ci)
    one, _ = run_steps(axf, monkeypatch, cfg, axf.F32, [60], False)
    assert n2 == 30
    assert_same(two, one, "ci %d" % ci)


def test_pair_small_grid_falls_back(axf, monkeypatch):
    """A grid with no interior for the pass steps one at a time, same bits."""
    cfg = grid_2d(120, 90, W.AX_OUTFLOW)
    two, n2 = run_steps(axf, monkeypatch, cfg, axf.F32, [31], True)
    one, _ = run_steps(axf, monkeypatch, cfg, axf.F32, [31], False)
    assert n2 == 31
    assert_same(two, one, "small")


def test_pair_matches_oracle(axf, monkeypatch):
    cfg = grid_2d(301, 213, W.AX_PML)
    run, n = run_steps(axf, monkeypatch, cfg, axf.F64, [120], True)
    assert n == 60
    ora = Oracle(cfg)
    ora.step(120)
    s0 = max(np.abs(ora.field(nm)).max() for nm in FIELDS[:6])
    s1 = max(np.abs(ora.field(nm)).max() for nm in FIELDS[6:12])
    sp = max(np.abs(ora.field(nm)).max() for nm in FIELDS[12:])
    assert s1 > 0 and sp > 0
    for k, nm in enumerate(FIELDS):
        scale = s0 if k < 6 else (s1 if k < 12 else sp)
        err = float(np.abs(run.read(nm) - ora.field(nm)).max())
        assert err <= 1e-10 * scale, (nm, err, scale)


def test_batched_pairs_equal_alone(axf, monkeypatch):
    """A batch of grids with a pass interior (different sizes, boundaries and
    diagnostic cadences, uneven step counts) takes two-step passes in its
    batched launches; every run ends bit-identical to the same run alone."""
    cfgs = [grid_2d(301, 213, W.AX_PML, seed=1), grid_2d(420, 331, W.AX_OUTFLOW, seed=2),
            grid_2d(260, 300, W.AX_PERIODIC, seed=3), grid_2d(333, 257, W.AX_REFLECT, seed=4)]
    for c, de in zip(cfgs, (0, 7, 10, 0)):
        c["diag_every"] = de
    counts = [[33, 40, 17, 0], [1, 28, 44, 51]]
    batch = axf.Batch(cfgs, precision=axf.F32)
    for c in counts:
        batch.step(c)
    for i, cfg in enumerate(cfgs):
        run = axf.Run(cfg, precision=axf.F32)
        for c in counts:
            if c[i]:
                run.step(c[i])
        assert batch.runs[i].steps_done == run.steps_done
        assert_same(batch.runs[i], run, "batched run %d" % i)
    batch.close()


@pytest.mark.parametrize("nx,ny", [(236, 36), (237, 43), (295, 37)])
def test_pair_smallest_interiors_bitwise(axf, monkeypatch, nx, ny):
    """Grids at the edge of having an interior for the pass (a one-segment,
    one-chunk core) and rows that leave a partial last chunk."""
    cfg = grid_2d(nx, ny, W.AX_OUTFLOW, seed=nx)
    two, n2 = run_steps(axf, monkeypatch, cfg, axf.F32, [24], True)
    one, _ = run_steps(axf, monkeypatch, cfg, axf.F32, [24], False)
    assert n2 == 12, n2
    assert_same(two, one, "%dx%d" % (nx, ny))
