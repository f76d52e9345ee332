"""Batches and the continuous-batching server through the C ABI.

A batched launch runs each run's own single-run body with the run's own step
counter, so every run of a batch (and every served request) must be
bit-identical to the same run stepped alone: fields, diagnostic records and
final probabilities.  The alone runs are themselves tied to the oracle by the
parity tests; one batched run is also compared with the oracle directly.
"""
import time

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2406_16796_amd import workloads as W
from test_gpu_pair import pass_available

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


def mixed_runs():
    """1D, 2D and 3D runs of uneven sizes and boundary kinds."""
    out = []
    for n, bc in ((300, W.AX_PERIODIC), (701, W.AX_OUTFLOW), (1100, W.AX_PML)):
        c = W.plane_wave_1d(nx=n, m=0.3, g=0.02, a0=0.5, ax_bc=bc, omega=1.3)
        c.update(packet_on=1, pk_amp=0.2, pk_k=1.0, pk_w=6.0, pk_x0=0.5 * n * c["dx"][0], pml_n=12)
        out.append(c)
    for (nx, ny), bc in (((40, 30), W.AX_OUTFLOW), ((290, 160), W.AX_PML), ((130, 61), W.AX_REFLECT)):
        c = W.gaussian_2d(n=nx, m=0.25, g=0.03, a0=0.5, waist_lam=1.2, fwhm_lam=1.5,
                          slab=(5, nx - 5), ax_bc=bc, seed=nx)
        dx = c["dx"][0]
        c.update(n=[nx, ny, 1], y_c=0.5 * ny * dx, t_center=6.0, pml_n=6, packet_on=1, pk_amp=0.2,
                 pk_k=1.0, pk_w=2.5, pk_x0=0.6 * nx * dx, pk_y0=0.4 * ny * dx, pk_dir=-1)
        out.append(c)
    c = W.focused_3d(n=20, m=0.3, g=0.03, a0=0.5, waist_lam=0.8, fwhm_lam=1.5, pk_amp=0.2, pk_w_lam=0.5)
    dx = c["dx"][0]
    c.update(n=[20, 18, 16], y_c=9 * dx, z_c=8 * dx, pk_y0=8 * dx, pk_z0=8 * dx, t_center=6.0)
    out.append(c)
    return out


def alone(axf, cfg, prec, counts, diag_every=0):
    run = axf.Run(dict(cfg, diag_every=cfg.get("diag_every", diag_every)), precision=prec)
    for n in counts:
        if n:
            run.step(n)
    return run


def assert_same(a, b, label):
    for nm in FIELDS:
        assert np.array_equal(a.read(nm), b.read(nm)), (label, nm)
    assert a.read_diag() == b.read_diag(), label
    assert a.diag_now() == b.diag_now(), label


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_equals_alone_bitwise(axf, prec):
    p = axf.F32 if prec == "f32" else axf.F64
    cfgs = mixed_runs()
    counts = [[45, 0, 120, 77, 150, 33, 60], [20, 71, 0, 90, 5, 64, 17]]
    batch = axf.Batch(cfgs, precision=p, diag_every=10)
    for c in counts:
        batch.step(c)
    for i, cfg in enumerate(cfgs):
        ref = alone(axf, cfg, p, [c[i] for c in counts], diag_every=10)
        assert batch.runs[i].steps_done == ref.steps_done
        assert_same(batch.runs[i], ref, "run %d" % i)
    batch.close()


def test_large_3d_run_in_a_batch_equals_alone(axf):
    """A 200^3 FP32 run, alone in its group (the batched unfused phases),
    beside a 1D run: both equal the runs stepped alone (the 3D one through
    the one-pass march), diagnostic records included, through two calls
    that start on different steps."""
    big = W.focused_3d(n=200, m=0.3, g=0.03, a0=0.5, waist_lam=0.8, fwhm_lam=1.5, pk_amp=0.2, pk_w_lam=0.5)
    dx = big["dx"][0]
    big.update(pk_x0=0.5 * 200 * dx, t_center=3.0)
    one = mixed_runs()[1]
    cfgs = [big, one]
    counts = [[23, 40], [14, 9]]
    batch = axf.Batch(cfgs, precision=axf.F32, diag_every=7)
    print("batch 200^3 + 1d", flush=True)
    for c in counts:
        batch.step(c)
    for i, cfg in enumerate(cfgs):
        ref = alone(axf, cfg, axf.F32, [c[i] for c in counts], diag_every=7)
        assert batch.runs[i].steps_done == ref.steps_done
        assert_same(batch.runs[i], ref, "run %d" % i)
        ref.close()
    batch.close()


def wide_runs():
    """2D runs wide enough for four-step passes (the first two) and one that
    only has an interior for two-step passes."""
    out = []
    for (nx, ny), bc in (((470, 150), W.AX_PML), ((520, 170), W.AX_PERIODIC), ((300, 140), W.AX_OUTFLOW)):
        c = W.gaussian_2d(n=nx, m=0.25, g=0.03, a0=0.5, waist_lam=1.2, fwhm_lam=1.5,
                          slab=(5, nx - 5), ax_bc=bc, seed=nx)
        dx = c["dx"][0]
        c.update(n=[nx, ny, 1], y_c=0.5 * ny * dx, t_center=6.0, pml_n=6, packet_on=1, pk_amp=0.2,
                 pk_k=1.0, pk_w=2.5, pk_x0=0.6 * nx * dx, pk_y0=0.4 * ny * dx, pk_dir=-1)
        out.append(c)
    return out


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_four_step_passes_equal_alone(axf, prec):
    """Batched four-step passes (wherever no record and no laser-table fill
    falls inside one), beside a group of two-step passes, with uneven step
    counts: every run bit-identical to the run stepped alone."""
    p = axf.F32 if prec == "f32" else axf.F64
    cfgs = wide_runs()
    f64 = prec == "f64"
    assert [pass_available(c, 4, f64=f64) for c in cfgs] == [True, True, False]
    assert pass_available(cfgs[2], 2, f64=f64)
    counts = [[61, 45, 70], [37, 0, 29], [4, 9, 2]]
    batch = axf.Batch(cfgs, precision=p, diag_every=9)
    for c in counts:
        batch.step(c)
    for i, cfg in enumerate(cfgs):
        ref = alone(axf, cfg, p, [c[i] for c in counts], diag_every=9)
        assert batch.runs[i].steps_done == ref.steps_done
        assert_same(batch.runs[i], ref, "run %d" % i)
    batch.close()


def test_batch_mixed_diag_cadence_equals_alone(axf):
    """Runs with different diagnostic cadences (and none) in one group."""
    cfgs = mixed_runs()[3:6]
    for c, de in zip(cfgs, (0, 7, 12)):
        c["diag_every"] = de
    batch = axf.Batch(cfgs, precision=axf.F32)
    batch.step([50, 50, 50])
    for i, cfg in enumerate(cfgs):
        assert_same(batch.runs[i], alone(axf, cfg, axf.F32, [50]), "cadence %d" % i)


def test_batched_run_matches_oracle(axf):
    cfgs = mixed_runs()
    batch = axf.Batch(cfgs, precision=axf.F64)
    batch.step([80] * len(cfgs))
    for i in (1, 4):
        ora = Oracle(cfgs[i])
        ora.step(80)
        s1 = max(np.abs(ora.field(n)).max() for n in FIELDS[6:12])
        s0 = max(np.abs(ora.field(n)).max() for n in FIELDS[:6])
        sp = max(np.abs(ora.field(n)).max() for n in FIELDS[12:])
        for k, nm in enumerate(FIELDS):
            scale = s0 if k < 6 else (s1 if k < 12 else sp)
            err = np.abs(batch.runs[i].read(nm) - ora.field(nm)).max()
            assert err <= 1e-10 * scale, (i, nm, err, scale)


def test_batch_view_cannot_be_stepped_or_destroyed_alone(axf):
    batch = axf.Batch(mixed_runs()[:2], precision=axf.F32)
    view = batch.runs[0]
    with pytest.raises(axf.AxfError):
        view.step(1)
    assert axf.lib().axf_destroy(view._h) != 0
    with pytest.raises(axf.AxfError):
        batch.step([-1, 3])


def wait_all(srv, ids, timeout=60.0):
    got = {}
    t0 = time.time()
    while len(got) < len(ids):
        for r in srv.poll():
            got[r["id"]] = r
        if time.time() - t0 > timeout:
            raise AssertionError("server results missing after %.0f s: %s" % (timeout, set(ids) - set(got)))
        time.sleep(0.005)
    return got


def test_server_results_equal_alone(axf):
    """Requests arriving while others run are admitted as memory and slots free
    up; each result equals the same run alone, bit for bit."""
    cfgs = mixed_runs()
    steps = [130, 40, 95, 150, 60, 110, 35]
    sizes = [axf.footprint(c, precision=axf.F32) for c in cfgs]
    # a pool that holds the three largest runs at once: admission must wait
    pool = sum(sorted(sizes)[-3:]) + (1 << 20)
    srv = axf.Server(pool, max_slots=3, macro_steps=16)
    ids = []
    for k, (c, n) in enumerate(zip(cfgs, steps)):
        ids.append(srv.submit(c, n))
        if k % 3 == 2:
            time.sleep(0.02)
    res = wait_all(srv, ids)
    srv.close()
    for rid, c, n in zip(ids, cfgs, steps):
        r = res[rid]
        assert r["status"] == 0, r
        assert r["steps"] == n
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        ref = alone(axf, c, axf.F32, [n]).diag_now()
        assert r["final"] == ref, (rid, r["final"], ref)


def test_server_cancel_and_oversized(axf):
    srv = axf.Server(64 << 20, max_slots=2, macro_steps=8)
    big = W.gaussian_2d(n=4096)
    with pytest.raises(axf.AxfError):
        srv.submit(big, 10)
    c = mixed_runs()[4]
    a = srv.submit(c, 100000)
    b = srv.submit(c, 20)
    time.sleep(0.05)
    srv.cancel(a)
    res = wait_all(srv, [a, b])
    assert res[a]["status"] == 1
    assert res[b]["status"] == 0
    st = srv.stats()
    assert st["resident"] == 0 and st["queued"] == 0 and st["bytes_used"] == 0
    srv.close()


def test_tuned_shape_is_used_and_results_unchanged(axf):
    """The tuner picks a launch shape for the size class; runs created after it
    use that shape, and their results are the same bits as with the default."""
    cfg = mixed_runs()[4]
    ref = axf.Run(cfg, precision=axf.F32)
    ref.step(60)
    axf.tune_reset()
    choice = axf.tune(cfg, precision=axf.F32, steps=8)
    # one-step shapes and the multi-step shapes this grid has an interior for
    # (two steps: 290 columns are too few for three)
    assert choice["path"] == axf.PATH_FUSED and choice["candidates"] >= 10
    assert choice["chunk"] > 0 and choice["prefetch"] > 0
    assert choice["steps_per_pass"] in (1, 2)
    assert (choice["frame_chunk"] > 0) == (choice["steps_per_pass"] > 1)
    assert choice["ms_per_step"] <= choice["default_ms_per_step"] * 1.5
    run = axf.Run(cfg, precision=axf.F32)
    run.step(60)
    axf.tune_reset()
    for nm in FIELDS:
        assert np.array_equal(run.read(nm), ref.read(nm)), nm
    plain = axf.tune(mixed_runs()[0], precision=axf.F32, steps=4)
    assert plain["path"] == axf.PATH_PLAIN
