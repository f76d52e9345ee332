"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function declared in include/axf.h, and its pure host calls (footprint,
extents, configuration checks) behave as documented."""
import os
import re

import pytest

from paper_2406_16796_amd import axf
from paper_2406_16796_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "axf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(axf_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 25
    L = axf.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(axf.EXPORTS)


def test_footprint_and_extents_follow_the_layout():
    cfg = W.focused_3d(n=64)
    nn = axf.extents(cfg)
    assert nn == (65, 65, 65)               # Mur axes carry the extra node plane
    f32 = axf.footprint(cfg, precision=axf.F32)
    f64 = axf.footprint(cfg, precision=axf.F64)
    # 3D keeps 2 time slots of the 12 EM arrays + 3 axion levels + 3 scratch,
    # rows padded to whole 128-byte lines: 96 floats, 80 doubles; each array
    # is followed by a 64 KiB sink for the stores of points a march wavefront
    # does not own
    arr32, arr64 = 96 * 65 * 65 * 4 + 65536, 80 * 65 * 65 * 8 + 65536
    assert 30 * arr32 <= f32 < 35 * arr32      # + 216 boundary planes, diagnostics
    assert 30 * arr64 <= f64 < 35 * arr64
    one_d = W.plane_wave_1d(nx=1000)
    assert axf.extents(one_d) == (1001, 1, 1)
    # 2D keeps 5 slots and 6 levels (its passes write up to four steps ahead)
    two_d = W.gaussian_2d(n=256)
    arr2 = 272 * 256 * 4
    assert 69 * arr2 <= axf.footprint(two_d, precision=axf.F32) < 80 * arr2


def test_512_cubed_fp32_footprint():
    """The 512^3 FP32 run: 30 arrays of 544 x 513 x 513 floats (17.2 GB) and
    the boundary planes; 3D runs keep two E/B slots and three axion levels,
    1D and 2D runs five and six."""
    b = axf.footprint(W.focused_3d(), precision=axf.F32)
    assert 30 * 544 * 513 * 513 * 4 < b < 17.6e9, b


@pytest.mark.parametrize("mutate,code", [
    (lambda c: c.update(dt=10.0), axf.EUNSTABLE),
    (lambda c: c.update(ndim=4), axf.EINVAL),
    (lambda c: c.update(laser_pol=2), axf.EINVAL),          # 2D keeps the in-plane polarisation
    (lambda c: c.update(em_bc=[0, 1, 0]), axf.EINVAL),      # laser needs a Mur x_min face
    (lambda c: c.update(pml_n=3000), axf.EINVAL),
    (lambda c: c.update(n=[4096, 4096, 2]), axf.EINVAL),    # ndim 2 needs n_z = 1
])
def test_invalid_configurations_are_rejected(mutate, code):
    cfg = W.gaussian_2d(n=256)
    cfg["ndim"] = 2
    mutate(cfg)
    with pytest.raises(axf.AxfError) as e:
        axf.footprint(cfg)
    assert e.value.code == code


def test_one_d_rejects_longitudinal_bext():
    cfg = W.plane_wave_1d(nx=512)
    cfg["bext"] = [0.5, 1.0, 0.0]
    with pytest.raises(axf.AxfError) as e:
        axf.footprint(cfg)
    assert e.value.code == axf.EINVAL


def test_batch_footprint_is_the_sum_of_run_footprints():
    """Host-only: the batch carves each run at a 256-byte boundary after the
    launch table, so its footprint is the sum of the runs' plus the table."""
    cfgs = [W.plane_wave_1d(nx=1000), W.gaussian_2d(n=64), W.plane_wave_1d(nx=3000)]
    total = axf.batch_footprint(cfgs, precision=axf.F32)
    runs = sum((axf.footprint(c, precision=axf.F32) + 255) // 256 * 256 for c in cfgs)
    assert runs < total <= runs + 64 * 1024
    bad = dict(cfgs[1], dt=10.0)
    with pytest.raises(axf.AxfError):
        axf.batch_footprint([cfgs[0], bad], precision=axf.F32)


@pytest.mark.parametrize("mutate", [
    lambda c: c.update(win_cells=65),
    lambda c: c.update(win_cells=-1),
    lambda c: c.update(win_t0=0.0),                      # the window moves after the first step
    lambda c: c.update(em_bc=[0, 1, 0], laser_on=0),     # a moving window needs Mur x faces
])
def test_moving_window_settings_are_checked(mutate):
    cfg = W.gaussian_2d(n=256)
    cfg.update(win_cells=8, win_t0=10.0)
    axf.footprint(cfg)
    mutate(cfg)
    with pytest.raises(axf.AxfError) as e:
        axf.footprint(cfg)
    assert e.value.code == axf.EINVAL


def test_batches_take_fixed_windows_only():
    cfg = W.gaussian_2d(n=64)
    cfg.update(win_cells=8, win_t0=10.0)
    with pytest.raises(axf.AxfError):
        axf.batch_footprint([W.plane_wave_1d(nx=1000), cfg], precision=axf.F32)
