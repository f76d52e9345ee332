"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle,
element by element on the same seeded synthetic inputs.

Tolerances (derived from the arithmetic, stated per test):
- FP64 storage: max |gpu - oracle| <= 1e-10 * max |oracle| per field, and the
  relative L2 error ||gpu - oracle|| / ||oracle|| <= 1e-11 for every field that
  does not vanish (its L2 norm above 1e-6 of the order's maximum times the
  square root of its size; a field that vanishes by symmetry holds rounding
  noise only, which the max bound covers); energies and the centroid within
  1e-11 relative.  The GPU stores the leapfrog form and multiplies by
  precomputed reciprocals, so the two differ by rounding only (a few ulp per
  step, growing linearly).
- FP32 storage: the per-field error is reported and bounded by 1e-4 of the
  order's maximum (a few FP32 roundings of 6e-8 per step over these runs'
  110-700 steps; measured at most 1.4e-5); the energies H_phi and H_gamma1
  by 2e-4 relative (twice the fields' relative error, squared sums
  accumulated in FP64) on these short runs (the long-run FP32 budget is
  checked by the probability tests).
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


def order_scales(ora):
    """Error scale per perturbation order: the largest oracle value of any
    component of that order (a component that vanishes by symmetry holds only
    rounding noise, so its own maximum is no scale)."""
    s0 = max(np.abs(ora.field(n)).max() for n in FIELDS[:6])
    s1 = max(np.abs(ora.field(n)).max() for n in FIELDS[6:12])
    sp = max(np.abs(ora.field(n)).max() for n in FIELDS[12:])
    return {n: (s0 if i < 6 else (s1 if i < 12 else sp)) for i, n in enumerate(FIELDS)}


def field_errors(run, ora):
    out = {}
    scales = order_scales(ora)
    for name in FIELDS:
        g, o = run.read(name), ora.field(name)
        assert g.shape == o.shape, name
        scale = scales[name]
        err = np.abs(g - o).max()
        out[name] = (err / scale) if scale > 0 else err
    return out


def field_l2_errors(run, ora):
    """Relative L2 error of every field that does not vanish."""
    out = {}
    scales = order_scales(ora)
    for name in FIELDS:
        g, o = run.read(name), ora.field(name)
        no = float(np.linalg.norm(o))
        if no > 1e-6 * scales[name] * math.sqrt(o.size):
            out[name] = float(np.linalg.norm(g - o)) / no
    return out


def check_fields(run, ora, tol, label, l2=None):
    errs = field_errors(run, ora)
    print(label, {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (label, k, v)
    if l2 is not None:
        errs2 = field_l2_errors(run, ora)
        print(label, "relative L2", {k: "%.2e" % v for k, v in errs2.items()}, flush=True)
        assert errs2, label
        for k, v in errs2.items():
            assert v <= l2, (label, "L2", k, v)


def check_energies(rec, ora, tol):
    h = ora.energies()
    for got, want in ((rec["h_phi"], h[0]), (rec["h_em0"], h[1]), (rec["h_em1"], h[2])):
        assert abs(got - want) <= tol * max(abs(want), 1e-300), (got, want)
    # the laser centroid (a position; 0 where B1z vanishes)
    xc = ora.laser_centroid()
    assert abs(rec["x_laser"] - xc) <= tol * max(abs(xc), 1.0), (rec["x_laser"], xc)


def small_1d(ax_bc, n=600):
    cfg = W.plane_wave_1d(nx=n, steps=700, m=0.3, g=0.02, a0=0.5, ax_bc=ax_bc)
    cfg.update(packet_on=1, pk_amp=0.3, pk_k=1.0, pk_w=8.0, pk_x0=0.6 * n * cfg["dx"][0], pk_dir=1,
               pml_n=30)
    return cfg


def small_2d(ax_bc, n=(90, 70)):
    cfg = W.gaussian_2d(n=n[0], steps=260, m=0.25, g=0.03, a0=0.5, waist_lam=1.2, fwhm_lam=1.5,
                        slab=(10, 70), ax_bc=ax_bc, seed=3)
    dx = cfg["dx"][0]
    cfg.update(n=[n[0], n[1], 1], y_c=0.5 * n[1] * dx, t_center=6.0, pml_n=8, packet_on=1,
               pk_amp=0.2, pk_k=1.0, pk_w=3.0, pk_x0=0.55 * n[0] * dx, pk_y0=0.4 * n[1] * dx, pk_dir=-1)
    return cfg


def small_3d(n=(36, 30, 28)):
    cfg = W.focused_3d(n=n[0], steps=110, m=0.3, g=0.03, a0=0.5, waist_lam=0.8, fwhm_lam=1.5,
                       pk_amp=0.2, pk_w_lam=0.5)
    dx = cfg["dx"][0]
    cfg.update(n=list(n), y_c=0.5 * n[1] * dx, z_c=0.5 * n[2] * dx, pk_y0=0.45 * n[1] * dx,
               pk_z0=0.55 * n[2] * dx, t_center=6.0)
    return cfg


def run_both(axf, cfg, precision, steps):
    ora = Oracle(cfg)
    ora.step(steps)
    run = axf.Run(cfg, precision=precision, path=cfg.get("path", 0))
    run.step(steps)
    run.sync()
    return run, ora


@pytest.mark.parametrize("ax_bc", [W.AX_PERIODIC, W.AX_REFLECT, W.AX_OUTFLOW, W.AX_PML])
def test_1d_fp64_matches_oracle(axf, ax_bc):
    cfg = small_1d(ax_bc)
    run, ora = run_both(axf, cfg, axf.F64, cfg["steps"])
    check_fields(run, ora, 1e-10, "1d bc%d" % ax_bc, l2=1e-11)
    check_energies(run.diag_now(), ora, 1e-11)


@pytest.mark.parametrize("ax_bc", [W.AX_OUTFLOW, W.AX_PML, W.AX_REFLECT])
def test_2d_fp64_matches_oracle(axf, ax_bc):
    cfg = small_2d(ax_bc)
    run, ora = run_both(axf, cfg, axf.F64, cfg["steps"])
    check_fields(run, ora, 1e-10, "2d bc%d" % ax_bc, l2=1e-11)
    check_energies(run.diag_now(), ora, 1e-11)


@pytest.mark.parametrize("ny", [64, 96])
def test_2d_fused_rows_multiple_of_chunk_match_oracle(axf, ny):
    """n_y a multiple of the fused kernel's row chunk: the last chunk holds only
    the nodal top row, and it alone reaches the top Mur ghost of E1."""
    cfg = small_2d(W.AX_PML, n=(130, ny))
    cfg["path"] = axf.PATH_FUSED
    run, ora = run_both(axf, cfg, axf.F64, 300)
    check_fields(run, ora, 1e-10, "2d fused ny=%d" % ny, l2=1e-11)


def test_3d_fused_planes_multiple_of_chunk_match_oracle(axf, monkeypatch):
    """The same for the 3D LDS-marching kernel along z (n_z = 128, one chunk of
    128 and a last chunk of the nodal top plane)."""
    monkeypatch.setenv("AXF_LDS_MARCH", "1")
    cfg = small_3d(n=(14, 12, 128))
    cfg.update(path=axf.PATH_FUSED, z_c=64 * cfg["dx"][0], pk_z0=100 * cfg["dx"][0])
    run, ora = run_both(axf, cfg, axf.F64, 90)
    check_fields(run, ora, 1e-10, "3d fused nz=128", l2=1e-11)


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_3d_fp64_matches_oracle(axf, path):
    cfg = dict(small_3d(), path=axf.PATH_PLAIN if path == "plain" else axf.PATH_FUSED)
    run, ora = run_both(axf, cfg, axf.F64, cfg["steps"])
    check_fields(run, ora, 1e-10, "3d " + path, l2=1e-11)
    check_energies(run.diag_now(), ora, 1e-11)


def test_3d_periodic_written_state_matches_oracle(axf):
    """Every component seeded with random data through axf_write_field, all
    couplings on, periodic box (exercises the write path and the wrap)."""
    rng = np.random.default_rng(21)
    n = [20, 18, 16]
    dx = [0.4, 0.45, 0.5]
    dt = 0.9 / math.sqrt(sum(1 / h ** 2 for h in dx))
    cfg = dict(n=n, dx=dx, dt=dt, em_bc=[0, 0, 0], ax_bc=[0, 0, 0], m=0.5, g=0.3,
               bext=[0.2, -0.3, 0.4], slab_lo=3, slab_hi=15)
    ora = Oracle(cfg)
    run = axf.Run(cfg, precision=axf.F64)
    for name in FIELDS:
        a = rng.standard_normal((n[2], n[1], n[0]))
        ora.field(name)[...] = a
        run.write(name, a)
    ora.refresh_initial()
    ora.step(60)
    run.step(60)
    check_fields(run, ora, 1e-10, "3d periodic", l2=1e-11)
    check_energies(run.diag_now(), ora, 1e-11)


def test_conversion_run_1d_4096_fp64(axf):
    """The 4096-cell, 3000-step CW conversion run: every field and the box
    energies against the oracle at the end."""
    cfg = W.plane_wave_1d()
    run, ora = run_both(axf, cfg, axf.F64, cfg["steps"])
    check_fields(run, ora, 1e-10, "1d 4096", l2=1e-11)
    check_energies(run.diag_now(), ora, 1e-11)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_3d_tiled_periodic_equals_plain_bitwise(axf, prec, monkeypatch):
    """Tile walks on a periodic box (random written state, every coupling on,
    18 planes: walks of 4 and a last one of 2): the E0 value a walk carries up
    to the next plane is the one that plane would compute, wrap or no wrap,
    so the state equals the unfused kernels' bit for bit."""
    monkeypatch.setenv("AXF_TILED", "1")
    monkeypatch.setenv("AXF_M3", "0")
    rng = np.random.default_rng(33)
    n = [20, 18, 18]
    dx = [0.4, 0.45, 0.5]
    dt = 0.9 / math.sqrt(sum(1 / h ** 2 for h in dx))
    cfg = dict(n=n, dx=dx, dt=dt, em_bc=[0, 0, 0], ax_bc=[0, 0, 0], m=0.5, g=0.3,
               bext=[0.2, -0.3, 0.4], slab_lo=3, slab_hi=15)
    p = axf.F32 if prec == "f32" else axf.F64
    data = {name: rng.standard_normal((n[2], n[1], n[0])) for name in FIELDS}
    runs = []
    for path in (axf.PATH_PLAIN, axf.PATH_FUSED):
        r = axf.Run(cfg, precision=p, path=path)
        for name in FIELDS:
            r.write(name, data[name])
        r.step(40)
        runs.append(r)
    for nm in FIELDS:
        assert np.array_equal(runs[0].read(nm), runs[1].read(nm)), nm


@pytest.mark.parametrize("kind", ["1d", "2d", "3d"])
def test_fp32_tracks_oracle(axf, kind):
    cfg = {"1d": small_1d(W.AX_OUTFLOW), "2d": small_2d(W.AX_PML), "3d": small_3d()}[kind]
    run, ora = run_both(axf, cfg, axf.F32, cfg["steps"])
    check_fields(run, ora, 1e-4, "fp32 " + kind)
    rec = run.diag_now()
    h = ora.energies()
    print("fp32", kind, "H_phi rel %.2e H_em1 rel %.2e" % (abs(rec["h_phi"] / h[0] - 1), abs(rec["h_em1"] / h[2] - 1)),
          flush=True)
    assert abs(rec["h_phi"] / h[0] - 1) < 2e-4
    assert abs(rec["h_em1"] / h[2] - 1) < 2e-4
    xc = ora.laser_centroid()
    assert xc > 0
    # FP32 fields within 1e-4 of their scale move the weighted mean by a
    # small fraction of a cell
    assert abs(rec["x_laser"] - xc) <= 1e-2 * cfg["dx"][0], (rec["x_laser"], xc)


def wide_2d(ax_bc, n=(300, 170)):
    """Large enough for interior wavefronts (clear of every face and PML layer)."""
    cfg = small_2d(ax_bc, n=n)
    cfg["pml_n"] = 10
    return cfg


@pytest.mark.parametrize("kind", ["2d_out", "2d_pml", "2d_ref", "2d_wide_pml", "2d_wide_out", "2d_lds", "3d",
                                  "3d_tiled", "3d_lds"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_equals_plain_bitwise(axf, kind, prec, monkeypatch):
    """The fused paths evaluate the same point formulas in the same order as
    the unfused kernels (no FP contraction), so the states agree bit for bit,
    boundaries included: the 2D wavefront kernels (the wide grids run both the
    interior and the boundary-frame kernels), the 3D semi-fused launches, and
    the LDS-marching kernels (2d_lds, 3d_lds).  In 3D the fused path is the
    one-pass march; 3d_tiled forces the tile-walk launches instead."""
    if kind.endswith("_lds"):
        monkeypatch.setenv("AXF_LDS_MARCH", "1")
    if kind == "3d_tiled":
        monkeypatch.setenv("AXF_TILED", "1")
        monkeypatch.setenv("AXF_M3", "0")
    else:
        monkeypatch.delenv("AXF_TILED", raising=False)
    cfg = {"2d_out": small_2d(W.AX_OUTFLOW), "2d_pml": small_2d(W.AX_PML), "2d_ref": small_2d(W.AX_REFLECT),
           "2d_wide_pml": wide_2d(W.AX_PML), "2d_wide_out": wide_2d(W.AX_OUTFLOW), "2d_lds": small_2d(W.AX_PML),
           "3d": small_3d(), "3d_tiled": small_3d(), "3d_lds": small_3d()}[kind]
    p = axf.F32 if prec == "f32" else axf.F64
    runs = []
    for path in (axf.PATH_PLAIN, axf.PATH_FUSED):
        r = axf.Run(cfg, precision=p, path=path)
        r.step(45)
        runs.append(r)
    for nm in FIELDS:
        assert np.array_equal(runs[0].read(nm), runs[1].read(nm)), nm


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_bit_reproducible_run_to_run(axf, prec):
    p = axf.F32 if prec == "f32" else axf.F64
    cfg = small_2d(W.AX_OUTFLOW)
    outs = []
    for _ in range(2):
        run = axf.Run(cfg, precision=p, diag_every=50)
        run.step(150)
        outs.append(([run.read(nm) for nm in FIELDS], run.read_diag()))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    assert outs[0][1] == outs[1][1]


def test_checkpoint_resume_is_bit_exact(axf):
    cfg = small_2d(W.AX_OUTFLOW)
    a = axf.Run(cfg, precision=axf.F32)
    a.step(120)
    b = axf.Run(cfg, precision=axf.F32)
    b.step(50)
    blob = b.state()
    c = axf.Run(cfg, precision=axf.F32)
    c.load_state(blob)
    c.step(70)
    for nm in FIELDS:
        assert np.array_equal(a.read(nm), c.read(nm)), nm


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_checkpoint_restored_into_the_same_run(axf, kind):
    """A laser run checkpointed at step 32, stepped 20 more (which refills
    the laser table) and restored into the same run continues as a fresh
    run restored from the same checkpoint: the restored table's levels are
    not taken for those the run held before."""
    cfg = small_2d(W.AX_OUTFLOW) if kind == "2d" else small_3d((130, 40, 32))
    a = axf.Run(cfg, precision=axf.F32)
    a.step(32)
    blob = a.state()
    a.step(20)
    a.load_state(blob)
    a.step(45)
    b = axf.Run(cfg, precision=axf.F32)
    b.load_state(blob)
    b.step(45)
    for nm in FIELDS:
        assert np.array_equal(a.read(nm), b.read(nm)), nm


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_coupling_scaled_out_bit_exact(axf, prec):
    """g -> 4 g: phi x 4, E1/B1 x 16 exactly, because the stored fields are the
    coupling-free scaled ones (power-of-two scales)."""
    p = axf.F32 if prec == "f32" else axf.F64
    base = small_2d(W.AX_PML)
    base["packet_on"] = 0
    outs = []
    for g in (3e-3, 12e-3):
        run = axf.Run(dict(base, g=g), precision=p)
        run.step(120)
        outs.append(run)
    for nm in FIELDS:
        f = 4.0 if nm.startswith("PHI") else (16.0 if nm[1] == "1" else 1.0)
        assert np.array_equal(outs[1].read(nm), f * outs[0].read(nm)), nm
