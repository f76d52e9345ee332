"""The numbers the paper prints, recomputed from their stated inputs.

Fixture: tests/golden/paper_printed_values.json (each entry cites its
passage).  The Sec. II.B example fixes the scale separation that makes the
first-order fields unrepresentable next to the zero-order ones in one FP64
variable; the oracle and the GPU path store the orders apart because of it.
"""
import json
import math
import os

import numpy as np

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))

# CODATA 2018
C = 299792458.0
ME = 9.1093837015e-31
QE = 1.602176634e-19
HBAR = 1.054571817e-34
MU0 = 1.25663706212e-6
GEV = 1e9 * QE


def test_fps_worked_example_recomputed():
    """Sec. II.B: a0 = 100 at 800 nm gives E0 = 4e14 V/m; with B0 = E0/c and
    g = 2.7e-13 hbar/GeV the generated axion field is g E0 B0 / (2 mu0 hbar k0^2)
    = 5.7e9 1/s and the first-order field g phi B0 c = 4e-13 V/m."""
    ex = GOLDEN["fps_worked_example"]
    tol = ex["printed_precision"]
    k0 = 2.0 * math.pi / ex["wavelength_m"]
    e0 = ex["a0"] * ME * C * (C * k0) / QE
    assert abs(e0 / ex["E0_V_per_m"] - 1.0) < tol
    b0 = e0 / C
    g = ex["g_hbar_per_GeV"] * HBAR / GEV          # coupling in s (hbar / GeV)
    phi = g * e0 * b0 / (2.0 * MU0 * HBAR * k0 * k0)
    assert abs(phi / ex["axion_field_per_s"] - 1.0) < tol
    e1 = g * phi * b0 * C
    assert abs(e1 / ex["E1_V_per_m"] - 1.0) < tol


def test_fps_worked_example_spacing():
    """Sec. II.B: E0 = 4e14 V/m is 1.xxx * 2^48, so its FP64 spacing is
    2^-52 * 2^48 = 0.0625 V/m, and E1 ~ 4e-13 V/m added to it is lost."""
    ex = GOLDEN["fps_worked_example"]
    e0 = ex["E0_V_per_m"]
    assert math.frexp(e0)[1] - 1 == ex["E0_binary_exponent"]
    assert np.spacing(e0) == ex["E0_spacing_V_per_m"]
    assert e0 + ex["E1_V_per_m"] == e0
    assert np.float32(ex["E1_V_per_m"]) != 0


def test_couplings_are_the_printed_ones():
    assert GOLDEN["dfsz_coupling"]["g_hbar_per_GeV"] == 2.65e-13
    assert GOLDEN["boundary_reflectivity"]["outflow"] == GOLDEN["boundary_reflectivity"]["pml"] == 0.01
