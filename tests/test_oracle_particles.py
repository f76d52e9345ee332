"""Pins of the oracle's particle side (Sec. II.B): cold electrons pushed by
the zero-order fields, their first-order perturbations, and the currents
j0, j1 they deposit.

- Boris push: one electron gyrating in a uniform B_z keeps |u| exactly and
  turns by 2 atan(B dt / (2 gamma)) per step (the closed form of the Boris
  rotation); its orbit has the gyro-radius |u| / B.
- Cold plasma oscillation: a uniform first-order momentum perturbation of a
  periodic plasma is the k = 0 Langmuir mode; the leapfrog of E and u gives
  E^{n+1} + E^{n-1} = (2 - omega_p^2 dt^2) E^n exactly (omega_p^2 = n).
- Linearisation (the FPS expansion of Sec. II.B): the first-order fields
  and particle perturbations of a run equal the derivative of the zero-order
  run with respect to the same perturbation, taken by central differences
  of two zero-order runs (error O(eps^2)).  A drifting plasma crossing a
  laser in a static B makes every term of the expansion non-zero
  (E_p's grad S . x1 term, v0 x B_p, v1 x B_nop, j1's grad S . x1 term).
  Copies of the oracle with one term dropped or a sign flipped fail it.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle.oracle import Oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def plasma_1d(n=64, ppc=2, dens=0.01, u=(0.0, 0.0, 0.0), bz=0.0, em=O.EM_PERIODIC, laser=False):
    dx = 2 * math.pi / 20
    cfg = dict(n=[n, 1, 1], dx=[dx, 1.0, 1.0], dt=0.9 * dx, em_bc=[em, 0, 0], ax_bc=[0, 0, 0],
               bext=[0.0, 0.0, bz], ppc=[ppc, 1], plasma_n=dens, plasma_lo=0, plasma_hi=n, plasma_u=list(u))
    if em == O.EM_MUR:
        cfg.update(plasma_lo=4, plasma_hi=n - 4)
    if laser:
        cfg.update(laser_on=1, laser_pol=1, laser_env=O.ENV_CW, omega=1.0, e_amp=0.05, ramp_periods=2.0)
    return cfg


def test_boris_gyration_closed_form():
    """A single electron (negligible density) in B_z: the momentum rotates
    counter-clockwise by theta = 2 atan(B dt / (2 gamma)) per step."""
    B, u0 = 0.7, 0.6
    cfg = plasma_1d(n=16, ppc=1, dens=1e-30, u=(u0, 0.0, 0.0), bz=B)
    cfg.update(plasma_lo=5, plasma_hi=6)
    o = Oracle(cfg)
    assert o.n_particles == 1
    gam = math.sqrt(1 + u0 * u0)
    theta = 2 * math.atan(B * cfg["dt"] / (2 * gam))
    x0 = o.particles("x")[0]
    for step in range(1, 40):
        o.step(1)
        ux, uy = o.particles("ux")[0], o.particles("uy")[0]
        assert math.hypot(ux, uy) == pytest.approx(u0, abs=1e-14)
        assert ux == pytest.approx(u0 * math.cos(step * theta), abs=1e-12)
        assert uy == pytest.approx(u0 * math.sin(step * theta), abs=1e-12)
    # x moves on a circle of radius |u| / B (x only in 1D: within 2 r of the start)
    L = cfg["n"][0] * cfg["dx"][0]
    dxp = (o.particles("x")[0] - x0 + L / 2) % L - L / 2
    assert abs(dxp) <= 2 * u0 / B + 1e-12


def test_cold_plasma_oscillation_recurrence():
    """k = 0 Langmuir mode in the first-order fields: uniform u1x on a
    periodic uniform plasma, E1x^{n+1} + E1x^{n-1} = (2 - n dt^2) E1x^n."""
    dens = 0.04
    cfg = plasma_1d(n=32, ppc=3, dens=dens)
    o = Oracle(cfg)
    o.particles("u1x")[:] = 1e-3
    o.redeposit()
    o.refresh_initial()
    e = []
    for _ in range(120):
        o.step(1)
        e.append(o.field("E1X")[0, 0, :32].copy())
    e = np.array(e)
    assert np.ptp(e[:, 0]) > 1e-6
    # uniform in x
    assert np.abs(e - e[:, :1]).max() <= 1e-12 * np.abs(e).max()
    c = 2 - dens * cfg["dt"] ** 2
    res = e[2:, 0] + e[:-2, 0] - c * e[1:-1, 0]
    assert np.abs(res).max() <= 1e-12 * np.abs(e).max()
    # the drift of the first-order x1 is (u1 at t) integrated: back to ~0 each period
    w = 2 * math.asin(math.sqrt(dens) * cfg["dt"] / 2) / cfg["dt"]
    assert w == pytest.approx(math.sqrt(dens), rel=2e-3)


FD_FIELDS = ["E%s%s" % (o, c) for o in "0" for c in "XYZ"] + ["B0X", "B0Y", "B0Z"]
PERTURB = {"ux": "u1x", "uy": "u1y", "uz": "u1z"}


def linearisation_case():
    """Drifting plasma (u = (0.3, 0.2, 0.1)) in B_z = 0.4 with a laser
    entering through x_min, Mur x faces; the perturbation is a smooth
    momentum pattern."""
    cfg = plasma_1d(n=96, ppc=2, dens=0.02, u=(0.3, 0.2, 0.1), bz=0.4, em=O.EM_MUR, laser=True)
    cfg.update(plasma_lo=8, plasma_hi=88)
    return cfg


def fd_mismatch(library=None, steps=60, eps=1e-5):
    cfg = linearisation_case()

    def run(sign, first):
        o = Oracle(cfg, library=library)
        x = o.particles("x")
        pat = {"ux": 0.05 * np.sin(x / 3.0), "uy": 0.04 * np.cos(x / 5.0), "uz": 0.03 * np.sin(x / 7.0 + 1.0)}
        for name, dv in pat.items():
            if first:
                o.particles(PERTURB[name])[:] = dv
            else:
                o.particles(name)[:] += sign * eps * dv
        o.redeposit()
        o.refresh_initial()
        o.step(steps)
        return o

    plus, minus, lin = run(+1, False), run(-1, False), run(0, True)
    worst = 0.0
    for f0 in ("E0X", "E0Y", "E0Z", "B0X", "B0Y", "B0Z"):
        f1 = f0.replace("0", "1", 1)
        fd = (plus.field(f0) - minus.field(f0)) / (2 * eps)
        got = lin.field(f1)
        scale = max(np.abs(fd).max(), 1e-300)
        worst = max(worst, np.abs(fd - got).max() / scale if np.abs(fd).max() > 0 else np.abs(got).max())
    for z, o1 in (("x", "x1"), ("ux", "u1x"), ("uy", "u1y"), ("uz", "u1z")):
        fd = (plus.particles(z) - minus.particles(z)) / (2 * eps)
        got = lin.particles(o1)
        worst = max(worst, np.abs(fd - got).max() / np.abs(fd).max())
    # the laser is zero order: the first-order run carries it too, in E0
    assert np.abs(lin.field("E0Y")).max() > 1e-3
    return worst


def test_first_order_particles_are_the_derivative_of_the_push():
    worst = fd_mismatch()
    print("FD mismatch %.2e" % worst)
    assert worst < 1e-6


PLANTS = [
    ("Ep[c] = f1 + gf;", "Ep[c] = f1;"),                                   # drop grad S . x1 E0
    ("Bp[c] = f1 + gf;", "Bp[c] = f1;"),                                   # drop grad S . x1 B0
    ("deposit(s, s->J[1][c], c, X, dX, qw * dv[c], qw * v[c]);",
     "deposit(s, s->J[1][c], c, X, dX, qw * dv[c], 0.0);"),                # drop j1's grad S . x1 term
    ("dv[q] = (g * g * du[q] - u[q] * ud) / (g * g * g);",
     "dv[q] = (g * g * du[q] + u[q] * ud) / (g * g * g);"),                # sign in v1
]


@pytest.mark.parametrize("plant", range(len(PLANTS)))
def test_planted_mistakes_fail_the_linearisation(plant, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "axion_oracle.c")).read()
    old, new = PLANTS[plant]
    assert src.count(old) == 1, old
    bad = tmp_path / "axion_oracle_planted.c"
    bad.write_text(src.replace(old, new))
    (tmp_path / "axion_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "axion_oracle.h")).read())
    lib = O.load(O.build(force=True, src=str(bad), out=str(tmp_path / "libplanted.so")))
    worst = fd_mismatch(library=lib)
    print("planted %d: FD mismatch %.2e" % (plant, worst))
    assert worst > 1e-3
