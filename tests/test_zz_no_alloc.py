"""axf_diag_now_static (the diagnostic record with its partials in the
library's static device workspace) against axf_diag_now, through the C ABI.

The two fold the same FP64 point sums in different orders, so the records
agree to FP64 rounding: every energy and probability within 1e-12 relative,
the step, time and finiteness flag exactly.  Two calls in a row, the second
on a smaller grid, show that a call leaves nothing behind that the next one
reads; the row counts cover the default, one workgroup folding every block,
and a count that leaves a ragged last fold.
"""
import pytest

from paper_2406_16796_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("h_phi", "h_em0", "h_em1", "p_gen", "p_conv", "x_laser")


@pytest.fixture(scope="module")
def axf():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_16796_amd import axf as A
    A.lib()
    return A


def same_record(a, b, tol=1e-12):
    assert a["step"] == b["step"] and a["t"] == b["t"] and a["finite"] == b["finite"], (a, b)
    for k in KEYS:
        scale = max(abs(a[k]), abs(b[k]))
        assert abs(a[k] - b[k]) <= tol * scale, (k, a[k], b[k])


def run_of(axf, cfg, prec, steps):
    r = axf.Run(cfg, precision=prec)
    r.step(steps)
    return r


def cases():
    big = W.focused_3d(n=96, steps=60, m=0.3, g=0.03, a0=0.5, waist_lam=0.8, fwhm_lam=1.5, pk_amp=0.2,
                       pk_w_lam=0.5)
    big["t_center"] = 3.0
    small = W.gaussian_2d(n=300, steps=40, g=0.03, a0=0.5, waist_lam=2.0, fwhm_lam=2.0, slab=(20, 280))
    small["t_center"] = 3.0
    return big, small


@pytest.mark.parametrize("prec_name", ["f32", "f64"])
def test_static_diag_equals_diag_now_twice(axf, prec_name):
    prec = axf.F32 if prec_name == "f32" else axf.F64
    big, small = cases()
    for cfg, steps, rows in ((big, 40, 0), (small, 30, 0), (small, 31, 1), (big, 41, 77)):
        print("static diag", cfg["name"], cfg["n"], prec_name, "steps", steps, "rows", rows, flush=True)
        r = run_of(axf, cfg, prec, steps)
        ref = r.diag_now()
        got = r.diag_now_static(rows)
        assert ref["h_em0"] > 0 and ref["h_phi"] > 0 and ref["h_em1"] > 0, ref
        same_record(ref, got)
        # a second call on the same state reads nothing the first one left
        same_record(ref, r.diag_now_static(rows))
        r.close()


def test_static_diag_rejects_rows_beyond_workspace(axf):
    _, small = cases()
    r = run_of(axf, small, axf.F32, 1)
    for rows in (-1, 1025, 1 << 20):
        with pytest.raises(RuntimeError, match="static diagnostic workspace"):
            r.diag_now_static(rows)
    r.close()
