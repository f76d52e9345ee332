"""The one-pass 3D march (one launch per step) against the unfused kernels and
the FP64 oracle.

The march evaluates the unfused kernels' point formulas in the same order (no
FP contraction), so the states must agree bit for bit.  The grids are chosen
so that the ways the march splits a grid all occur: several x segments with a
ragged last one, row groups whose last one holds only the nodal top row of a
Mur y axis, plane chunks whose last one holds only the nodal top plane, the
laser on the x_min face, and each axion boundary kind.
"""
import math

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


@pytest.fixture(autouse=True)
def march_in_both_precisions(monkeypatch):
    """FP64 runs take the tile walks by default; this file tests the march."""
    monkeypatch.setenv("AXF_M3", "1")


def box_3d(n, ax_bc=W.AX_OUTFLOW):
    """A focused pulse from x_min and a counter-propagating axion packet in a
    uniform B_ext along z, with all couplings strong enough to move every
    field within a few tens of steps."""
    cfg = W.focused_3d(n=n[0], steps=60, m=0.3, g=0.03, a0=0.5, waist_lam=0.8, fwhm_lam=1.5,
                       pk_amp=0.2, pk_w_lam=0.5)
    dx = cfg["dx"][0]
    cfg.update(n=list(n), y_c=0.5 * n[1] * dx, z_c=0.5 * n[2] * dx, pk_x0=0.5 * n[0] * dx,
               pk_y0=0.45 * n[1] * dx, pk_z0=0.55 * n[2] * dx, t_center=3.0, ax_bc=[ax_bc] * 3,
               pml_n=6)
    return cfg


def pair(axf, cfg, prec, steps, chunk=None, monkeypatch=None, diag_every=0):
    """The same run through the unfused kernels and through the march."""
    if chunk is not None:
        monkeypatch.setenv("AXF_M3_CHUNK", str(chunk))
    p = axf.F32 if prec == "f32" else axf.F64
    plain = axf.Run(cfg, precision=p, path=axf.PATH_PLAIN, diag_every=diag_every)
    plain.step(steps)
    march = axf.Run(cfg, precision=p, path=axf.PATH_FUSED, diag_every=diag_every)
    print("case", cfg["n"], prec, "chunk", chunk, "steps", steps, flush=True)
    march.step(steps)
    launches = march.last_step_timing()[1]
    return plain, march, launches


def assert_same(plain, march):
    for nm in FIELDS:
        a, b = plain.read(nm), march.read(nm)
        assert np.array_equal(a, b), (nm, np.abs(a - b).max(), np.abs(a).max())


# n = (x, y, z) cells: x + 1 = 131 nodal columns -> 3 segments (44, 44, 43);
# y + 1 = 41 nodal rows -> row groups of 10 own rows, the last one only the
# top nodal row (12 wavefronts per FP32 workgroup); z + 1 = 33 nodal planes
# in chunks of 16 -> the last chunk only the top nodal plane.
RAGGED = (130, 40, 32)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("chunk", [16, 0])
def test_march_equals_plain_mur_outflow(axf, prec, chunk, monkeypatch):
    cfg = box_3d(RAGGED)
    plain, march, launches = pair(axf, cfg, prec, 45, chunk, monkeypatch)
    assert launches == 45, launches
    assert_same(plain, march)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_march_equals_plain_reflect_x_faces(axf, prec, monkeypatch):
    """Mur x faces with a reflecting axion on the ragged grid: the x-face
    launch (both x faces in one wavefront per row, lanes 0-31 and 32-63) takes
    the reflecting ghost, two interior segments lie between the halves."""
    cfg = box_3d(RAGGED, W.AX_REFLECT)
    plain, march, _ = pair(axf, cfg, prec, 45, 16, monkeypatch)
    assert_same(plain, march)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_march_equals_plain_wide_x(axf, prec, monkeypatch):
    """257 nodal columns: 28 at x_min and 9 at x_max in the x-face wavefronts,
    four interior segments of 55 between them; the axion packet starts 8
    cells from the x_max face, so that it reaches that face's ghosts."""
    cfg = box_3d((256, 26, 22))
    cfg.update(pk_x0=(256 - 8) * cfg["dx"][0])
    plain, march, _ = pair(axf, cfg, prec, 40, 8, monkeypatch)
    assert_same(plain, march)


@pytest.mark.parametrize("ax_bc", [W.AX_PML, W.AX_REFLECT, W.AX_PERIODIC])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_march_equals_plain_axion_boundaries(axf, ax_bc, prec, monkeypatch):
    """Mur EM faces with each other axion boundary (periodic axion on a Mur EM
    axis wraps the axion alone)."""
    cfg = box_3d((70, 27, 23), ax_bc)
    plain, march, _ = pair(axf, cfg, prec, 40, 8, monkeypatch)
    assert_same(plain, march)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_march_equals_plain_periodic_random_state(axf, prec, monkeypatch):
    """A periodic box seeded with random data in every component, every
    coupling on: the wrap of columns, rows and planes (the last row group and
    plane chunk wrap past the top)."""
    monkeypatch.setenv("AXF_M3_CHUNK", "7")
    rng = np.random.default_rng(71)
    n = [67, 23, 19]
    dx = [0.4, 0.45, 0.5]
    dt = 0.9 / math.sqrt(sum(1 / h ** 2 for h in dx))
    cfg = dict(n=n, dx=dx, dt=dt, em_bc=[0, 0, 0], ax_bc=[0, 0, 0], m=0.5, g=0.3,
               bext=[0.2, -0.3, 0.4], slab_lo=3, slab_hi=51)
    p = axf.F32 if prec == "f32" else axf.F64
    data = {name: rng.standard_normal((n[2], n[1], n[0])) for name in FIELDS}
    runs = []
    for path in (axf.PATH_PLAIN, axf.PATH_FUSED):
        r = axf.Run(cfg, precision=p, path=path)
        for name in FIELDS:
            r.write(name, data[name])
        print("periodic", prec, "path", path, flush=True)
        r.step(30)
        runs.append(r)
    assert_same(*runs)


@pytest.mark.parametrize("n,prec", [((75, 26, 22), "f64"), ((130, 26, 22), "f32")])
def test_march_equals_plain_mixed_axes(axf, n, prec, monkeypatch):
    """Mur EM and an outflow axion along x only, periodic y and z (the 130
    cell FP32 grid takes the x-face launch, the narrow FP64 one the frame)."""
    cfg = box_3d(n)
    cfg.update(em_bc=[W.EM_MUR, W.EM_PERIODIC, W.EM_PERIODIC], ax_bc=[W.AX_OUTFLOW, W.AX_PERIODIC, W.AX_PERIODIC])
    plain, march, _ = pair(axf, cfg, prec, 40, 9, monkeypatch)
    assert_same(plain, march)


def test_march_diagnostic_records_equal_plain(axf, monkeypatch):
    """Records every 7 steps: the march stores the whole state of every step,
    so the records are those of the unfused path."""
    cfg = box_3d((70, 27, 23))
    plain, march, _ = pair(axf, cfg, "f32", 30, 8, monkeypatch, diag_every=7)
    assert plain.read_diag() == march.read_diag()
    assert_same(plain, march)


def test_march_fp64_matches_oracle(axf, monkeypatch):
    """The march in FP64 storage against the oracle: max error within 1e-10 of
    each order's scale, relative L2 error within 1e-11 for every field that
    does not vanish."""
    monkeypatch.setenv("AXF_M3_CHUNK", "12")
    cfg = box_3d((40, 30, 28))
    ora = Oracle(cfg)
    ora.step(50)
    run = axf.Run(cfg, precision=axf.F64, path=axf.PATH_FUSED)
    run.step(50)
    scales = {}
    for lo, hi in ((0, 6), (6, 12), (12, 14)):
        s = max(np.abs(ora.field(n)).max() for n in FIELDS[lo:hi])
        for n in FIELDS[lo:hi]:
            scales[n] = s
    for nm in FIELDS:
        g, o = run.read(nm), ora.field(nm)
        err = np.abs(g - o).max() / scales[nm]
        assert err <= 1e-10, (nm, err)
        no = float(np.linalg.norm(o))
        if no > 1e-6 * scales[nm] * math.sqrt(o.size):
            l2 = float(np.linalg.norm(g - o)) / no
            print(nm, "max %.2e L2 %.2e" % (err, l2), flush=True)
            assert l2 <= 1e-11, (nm, l2)
