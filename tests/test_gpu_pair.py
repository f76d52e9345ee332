"""Passes of several steps of the 2D wavefront step (temporal blocking) against
the one-step pass, through the C ABI.

A pass advances the interior two, three or four steps with the same point formulas
in the same order as one-step passes, and the boundary frame with one-step
launches, so fields, diagnostic records and probabilities must be the same
bits.  The one-step pass is itself tied to the oracle by the parity tests; one
run of each pass length is also compared with the oracle directly.

The number of launches a call makes is checked against a model of the
runtime's choice: at each step the longest pass (up to the run's limit) that
the grid has an interior for, that fits the steps left, and that no
diagnostic record falls inside (on any of its steps but the first: a record
of the first step reads the state before the pass and E of the next step,
which such a pass also stores).
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


def default_shape(ns):
    """The built-in rows per interior / frame wavefront of an ns-step pass."""
    return (16, 8) if ns >= 4 else (12, 6)


def pass_available(cfg, ns, ci=None, cf=None, f64=False):
    """Whether the grid (Mur EM on x and y) has an interior for an ns-step pass:
    columns x0 - lo .. x0 - lo + 63 and rows c0 - 3 ns - 1 .. c0 + ci + ns clear
    of the face ghost ring (and of a damping layer in FP64), and a core of one
    segment and one frame chunk inside ns - 1 rings."""
    if ci is None or cf is None:
        ci, cf = default_shape(ns)
    n0, n1 = int(cfg["n"][0]), int(cfg["n"][1])
    nn1 = n1 + 1
    # the margin is the face ghost ring, and a damping layer in FP64 or when
    # wider than the run's 64-entry profile table
    pml = int(cfg.get("pml_n", 20))
    pml = pml if (f64 or pml > 64) else 0
    mxg = 1 + (pml if cfg["ax_bc"][0] == W.AX_PML else 0)
    myg = 1 + (pml if cfg["ax_bc"][1] == W.AX_PML else 0)
    wid, lo = 66 - 4 * ns, 2 * ns - 1
    sx0 = -(-(mxg + lo) // wid)
    r = n0 - 1 - mxg - (63 - lo)
    sx1 = r // wid + 1 if r >= 0 else 0
    cy0 = -(-(myg + 3 * ns + 1) // ci)
    r = n1 - 1 - myg - ns - ci
    cy1 = r // ci + 1 if r >= 0 else 0
    if ci % cf:
        return False
    nchf, k = -(-nn1 // cf), ci // cf
    if cy1 * k > nchf - 1:
        cy1 = (nchf - 1) // k
    need = 2 * (ns - 1) + 1
    return sx1 - sx0 >= need and (cy1 - cy0) * k >= need


def model_launches(cfg, counts, nmax, diag_every, ci=None, cf=None, f64=False):
    avail = {k: pass_available(cfg, k, ci=ci, cf=cf, f64=f64) for k in range(2, nmax + 1)}
    due = lambda s: diag_every > 0 and s % diag_every == 0
    step, launches = 0, 0
    for n in counts:
        it = 0
        while it < n:
            ns = 1
            for k in range(nmax, 1, -1):
                if avail[k] and n - it >= k and not any(due(step + q) for q in range(1, k)):
                    ns = k
                    break
            step += ns
            it += ns
            launches += 1
    return launches


def run_steps(axf, monkeypatch, cfg, prec, counts, ns, diag_every=0, ci=None, cf=None):
    """ns = 1: one step per pass; 2, 3 or 4: passes of up to ns steps."""
    monkeypatch.setenv("AXF_WAVE_PASS", "1" if ns > 1 else "0")
    monkeypatch.setenv("AXF_PASS_STEPS", str(max(ns, 2)))
    for name, v in (("AXF_PASS_CHUNK", ci), ("AXF_PASS_FRAME", cf)):
        if v:
            monkeypatch.setenv(name, str(v))
        else:
            monkeypatch.delenv(name, raising=False)
    run = axf.Run(dict(cfg, diag_every=diag_every), precision=prec, path=axf.PATH_FUSED)
    launches = 0
    for n in counts:
        run.step(n)
        launches += run.last_step_timing()[1]
    monkeypatch.delenv("AXF_WAVE_PASS")
    monkeypatch.delenv("AXF_PASS_STEPS")
    return run, launches


def assert_same(a, b, label):
    for nm in FIELDS:
        x, y = a.read(nm), b.read(nm)
        assert np.array_equal(x, y), (label, nm, float(np.abs(x - y).max()))
    assert a.read_diag() == b.read_diag(), label
    assert a.diag_now() == b.diag_now(), label


@pytest.mark.parametrize("ns", [2, 3, 4])
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("bc", ["periodic", "outflow", "pml", "reflect"])
def test_pass_equals_single_bitwise(axf, monkeypatch, ns, prec, bc):
    code = {"periodic": W.AX_PERIODIC, "outflow": W.AX_OUTFLOW, "pml": W.AX_PML, "reflect": W.AX_REFLECT}[bc]
    p = axf.F32 if prec == "f32" else axf.F64
    cfg = grid_2d(420, 331, code)
    assert pass_available(cfg, ns, f64=prec == "f64")
    counts = [1, 44, 17, 2]          # odd starts; diagnostics every 10 steps break passes
    multi, nm = run_steps(axf, monkeypatch, cfg, p, counts, ns, diag_every=10)
    one, n1 = run_steps(axf, monkeypatch, cfg, p, counts, 1, diag_every=10)
    assert n1 == sum(counts)
    assert nm == model_launches(cfg, counts, ns, 10, f64=prec == "f64"), nm
    assert nm < (0.75 if ns == 2 else 0.6) * sum(counts), nm
    assert_same(multi, one, "%d steps %s %s" % (ns, prec, bc))


@pytest.mark.parametrize("ns", [2, 3, 4])
@pytest.mark.parametrize("ci,cf", [(8, 8), (24, 8), (36, 6), (16, 4)])
def test_pass_interior_chunks_bitwise(axf, monkeypatch, ns, ci, cf):
    cfg = grid_2d(420 if ns < 4 else 520, 331, W.AX_PML, pml_n=20, seed=11)
    assert pass_available(cfg, ns, ci=ci, cf=cf)
    multi, nm = run_steps(axf, monkeypatch, cfg, axf.F32, [60], ns, ci=ci, cf=cf)
    one, _ = run_steps(axf, monkeypatch, cfg, axf.F32, [60], 1)
    assert nm == model_launches(cfg, [60], ns, 0, ci=ci, cf=cf), nm
    assert nm < 60
    assert_same(multi, one, "%d steps ci %d cf %d" % (ns, ci, cf))


def test_pass_small_grid_falls_back(axf, monkeypatch):
    """A grid with no interior for any pass steps one at a time; one with an
    interior for two steps but not three takes two-step passes; same bits."""
    for nx, ny, want in ((120, 90, 31), (301, 213, 16)):
        cfg = grid_2d(nx, ny, W.AX_OUTFLOW)
        multi, nm = run_steps(axf, monkeypatch, cfg, axf.F32, [31], 3)
        one, _ = run_steps(axf, monkeypatch, cfg, axf.F32, [31], 1)
        assert nm == want == model_launches(cfg, [31], 3, 0), (nx, ny, nm)
        assert_same(multi, one, "small %dx%d" % (nx, ny))


@pytest.mark.parametrize("ns", [2, 3, 4])
def test_pass_matches_oracle(axf, monkeypatch, ns):
    cfg = grid_2d(420, 331, W.AX_PML)
    run, n = run_steps(axf, monkeypatch, cfg, axf.F64, [120], ns)
    assert n == 120 // ns
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
    batched launches; every run ends bit-identical to the same run alone
    (which takes three-step passes where it can)."""
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


def smallest_grid(ns):
    """The narrowest and then the shortest grid with an interior for an
    ns-step pass (the innermost core one segment and one chunk)."""
    nx = next(x for x in range(64, 1000) if pass_available(grid_2d(x, 400, W.AX_OUTFLOW), ns))
    ny = next(y for y in range(8, 1000) if pass_available(grid_2d(nx, y, W.AX_OUTFLOW), ns))
    return nx, ny


@pytest.mark.parametrize("ns", [2, 3, 4])
@pytest.mark.parametrize("dx,dy", [(0, 0), (1, 7), (59, 1)])
def test_pass_smallest_interiors_bitwise(axf, monkeypatch, ns, dx, dy):
    """Grids at the edge of having an interior for the pass (one column or
    row fewer has none) and a little beyond, with rows that leave a partial
    last chunk."""
    nx0, ny0 = smallest_grid(ns)
    nx, ny = nx0 + dx, ny0 + dy
    cfg = grid_2d(nx, ny, W.AX_OUTFLOW, seed=nx)
    assert pass_available(cfg, ns)
    assert not pass_available(grid_2d(nx0 - 1, ny0, W.AX_OUTFLOW), ns)
    assert not pass_available(grid_2d(nx0, ny0 - 1, W.AX_OUTFLOW), ns)
    steps = 6 * ns
    multi, nm = run_steps(axf, monkeypatch, cfg, axf.F32, [steps], ns)
    one, _ = run_steps(axf, monkeypatch, cfg, axf.F32, [steps], 1)
    assert nm == steps // ns == model_launches(cfg, [steps], ns, 0), nm
    assert_same(multi, one, "%d steps %dx%d" % (ns, nx, ny))



@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_pass_one_interior_launch_bitwise(axf, monkeypatch, prec):
    """Three-step passes with the interior in one launch (AXF_PASS_RING=0,
    frame k leaving out core k) instead of core and ring launches: the same
    bits as one-step passes and as the split passes."""
    p = axf.F32 if prec == "f32" else axf.F64
    cfg = grid_2d(420, 331, W.AX_PML, seed=17)
    counts = [2, 37]
    split, ns = run_steps(axf, monkeypatch, cfg, p, counts, 3)
    monkeypatch.setenv("AXF_PASS_RING", "0")
    whole, nw = run_steps(axf, monkeypatch, cfg, p, counts, 3)
    monkeypatch.delenv("AXF_PASS_RING")
    one, _ = run_steps(axf, monkeypatch, cfg, p, counts, 1)
    assert nw == ns == model_launches(cfg, counts, 3, 0, f64=prec == "f64"), (nw, ns)
    assert_same(whole, one, "three steps, one interior launch")
    assert_same(split, one, "three steps, core and ring")


def random_cases(count=16, seed=2406):
    """Seeded random grids, boundaries, chunk shapes, pass lengths and step
    sequences (with the pass model's availability, so every case takes
    passes of the length it asks for)."""
    rng = np.random.default_rng(seed)
    bcs = [W.AX_PERIODIC, W.AX_OUTFLOW, W.AX_PML, W.AX_REFLECT]
    shapes = [(8, 8), (12, 6), (16, 8), (16, 4), (20, 10), (24, 8)]
    out = []
    while len(out) < count:
        ns = int(rng.integers(2, 5))
        ci, cf = shapes[int(rng.integers(len(shapes)))]
        nx, ny = int(rng.integers(300, 720)), int(rng.integers(120, 520))
        bc = bcs[int(rng.integers(len(bcs)))]
        pml = int(rng.integers(4, 24))
        cfg = grid_2d(nx, ny, bc, pml_n=pml, seed=int(rng.integers(1, 1000)))
        if not pass_available(cfg, ns, ci=ci, cf=cf):
            continue
        counts = [int(v) for v in rng.integers(1, 23, size=3)]
        de = int(rng.choice([0, 5, 7, 11]))
        out.append((ns, ci, cf, cfg, counts, de))
    return out


@pytest.mark.parametrize("case", range(16))
def test_pass_random_grids_bitwise(axf, monkeypatch, case):
    ns, ci, cf, cfg, counts, de = random_cases()[case]
    multi, nm = run_steps(axf, monkeypatch, cfg, axf.F32, counts, ns, diag_every=de, ci=ci, cf=cf)
    one, _ = run_steps(axf, monkeypatch, cfg, axf.F32, counts, 1, diag_every=de)
    assert nm == model_launches(cfg, counts, ns, de, ci=ci, cf=cf), nm
    assert_same(multi, one, "case %d: %d steps, %s rows, grid %s, counts %s, diag %d"
                % (case, ns, (ci, cf), cfg["n"][:2], counts, de))
