"""The moving window (Sec. III.B) on the GPU: against the oracle moving on
the same schedule, fused against unfused bit for bit in 2D and 3D, and
through a checkpoint."""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2406_16796_amd import workloads as W
from window_common import FIELDS, oracle_windowed, pulse_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def axf():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_16796_amd import axf as A
    A.lib()
    return A


def scales(ora):
    out = {}
    for lo, hi in ((0, 6), (6, 12), (12, 14)):
        s = max(np.abs(ora.field(n)).max() for n in FIELDS[lo:hi])
        for n in FIELDS[lo:hi]:
            out[n] = s
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_window_matches_oracle(axf, prec):
    """600 steps, 256 columns moved in moves of 8, the 2D default path."""
    cfg = pulse_2d(240)
    steps = 600
    ora, moved = oracle_windowed(Oracle, cfg, steps)
    run = axf.Run(cfg, precision=axf.F64 if prec == "f64" else axf.F32)
    print("window 2d", prec, "fused", run.uses_fused(), flush=True)
    run.step(steps)
    assert moved == 256
    sc = scales(ora)
    worst = {n: float(np.abs(run.read(n) - ora.field(n)).max()) / sc[n] for n in FIELDS}
    print({k: "%.1e" % v for k, v in worst.items()}, flush=True)
    assert max(worst.values()) <= (1e-10 if prec == "f64" else 1e-4), worst
    rec = run.diag_now()
    assert rec["finite"] == 1 and rec["p_gen"] > 0
    run.close()


def window_3d(nx=96):
    cfg = W.focused_3d(n=96, steps=0, m=0.3, g=0.03, a0=0.5, waist_lam=0.8, fwhm_lam=1.0, pk_amp=0.0,
                       pk_w_lam=0.5)
    n = [nx, 30, 26]
    dx = cfg["dx"][0]
    tau0 = cfg["fwhm"] / math.sqrt(2.0 * math.log(2.0))
    cfg.update(n=n, y_c=0.5 * n[1] * dx, z_c=0.5 * n[2] * dx, x_focus=20 * dx, t_center=3.0 * tau0, packet_on=0,
               win_cells=8, win_t0=6.5 * tau0)
    return cfg


@pytest.mark.parametrize("kind", ["2d", "3d", "3d_wide"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_window_fused_equals_plain_bitwise(axf, kind, prec):
    """3d_wide: 131 nodal columns, wide enough for the march's x-face launch
    in FP32 (face values staged per block) while the window moves."""
    cfg = pulse_2d(240) if kind == "2d" else (window_3d() if kind == "3d" else window_3d(130))
    steps = 400 if kind == "2d" else 200
    p = axf.F64 if prec == "f64" else axf.F32
    runs = []
    for path in (axf.PATH_PLAIN, axf.PATH_FUSED):
        r = axf.Run(cfg, precision=p, path=path)
        print("window", kind, prec, "path", path, flush=True)
        r.step(steps)
        runs.append(r)
    for n in FIELDS:
        assert np.array_equal(runs[0].read(n), runs[1].read(n)), n


def test_window_checkpoint_resumes_bitwise(axf):
    """A state written between moves carries the window's place: the
    restored run moves on the same schedule as the uninterrupted one."""
    cfg = pulse_2d(240)
    a = axf.Run(cfg, precision=axf.F32)
    a.step(450)
    b = axf.Run(cfg, precision=axf.F32)
    b.step(300)
    blob = b.state()
    c = axf.Run(cfg, precision=axf.F32)
    c.load_state(blob)
    c.step(150)
    for n in FIELDS:
        assert np.array_equal(a.read(n), c.read(n)), n
