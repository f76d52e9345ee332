"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a discrete dispersion relation
(exact normal modes of the Yee and Klein-Gordon leapfrogs), a discrete
invariant, a continuum identity that the scheme keeps exactly, scaling
symmetry, the method of images, or an exact-rational re-implementation on a
tiny grid.  None of them re-calls the oracle to get its expected value.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle.oracle import Oracle, laser_centroid

F = ["E0X", "E0Y", "E0Z", "B0X", "B0Y", "B0Z", "E1X", "E1Y", "E1Z", "B1X", "B1Y", "B1Z"]


def periodic_cfg(n, dx, dt, **kw):
    cfg = dict(n=list(n), dx=list(dx), dt=dt, em_bc=[0, 0, 0], ax_bc=[0, 0, 0])
    cfg.update(kw)
    return cfg


def positions(n, dx, nodal_axis=None, centred_axis=None, kind="E", comp=0):
    """Coordinate grids (z, y, x order) of a component: E_c nodal along c,
    B_c centred along c, phi centred everywhere."""
    coords = []
    for d in range(3):
        idx = np.arange(n[d], dtype=float)
        if kind == "phi":
            nodal = False
        elif kind == "E":
            nodal = (d == comp)
        else:
            nodal = (d != comp)
        coords.append(idx * dx[d] if nodal else (idx + 0.5) * dx[d])
    z, y, x = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    return x, y, z


# ---------------------------------------------------------------- dispersion

def yee_mode(n, dx, dt, kvec, e_hat):
    """Exact discrete plane wave of the Yee leapfrog: K_d = (2/dx_d) sin(k_d dx_d/2),
    Omega = |K|, omega = (2/dt) asin(Omega dt/2); E_hat is made orthogonal to K
    and B_hat = K x E_hat / Omega."""
    K = np.array([2.0 / dx[d] * math.sin(kvec[d] * dx[d] / 2.0) for d in range(3)])
    Om = float(np.linalg.norm(K))
    e = np.array(e_hat, dtype=float)
    e = e - K * (e @ K) / (K @ K)
    e /= np.linalg.norm(e)
    b = np.cross(K, e) / Om
    omega = 2.0 / dt * math.asin(Om * dt / 2.0)
    return e, b, omega


@pytest.mark.parametrize("axis,pol", [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])
def test_yee_plane_wave_each_axis(axis, pol):
    n = [1, 1, 1]
    n[axis] = 40
    dx = [1.0, 1.0, 1.0]
    dx[axis] = 0.3
    dt = 0.95 * 0.3
    kv = [0.0, 0.0, 0.0]
    kv[axis] = 2 * math.pi * 3 / (40 * 0.3)
    eh = [0.0, 0.0, 0.0]
    eh[pol] = 1.0
    _check_yee_mode(n, dx, dt, kv, eh, nsteps=150)


def test_yee_oblique_mode_3d():
    n = [12, 10, 8]
    dx = [0.5, 0.4, 0.45]
    dt = 0.9 / math.sqrt(sum(1 / h ** 2 for h in dx))
    kv = [2 * math.pi * m / (n[d] * dx[d]) for d, m in enumerate([1, 2, 1])]
    _check_yee_mode(n, dx, dt, kv, [0.3, -0.2, 1.0], nsteps=60)


def _check_yee_mode(n, dx, dt, kv, eh, nsteps):
    e, b, omega = yee_mode(n, dx, dt, kv, eh)
    o = Oracle(periodic_cfg(n, dx, dt))
    ch = math.cos(omega * dt / 2)

    def phase(kind, c, t):
        x, y, z = positions(n, dx, kind=kind, comp=c)
        return kv[0] * x + kv[1] * y + kv[2] * z - omega * t

    for c in range(3):
        o.field(F[c])[...] = ch * e[c] * np.cos(phase("E", c, 0.0))
        o.field(F[3 + c])[...] = b[c] * np.cos(phase("B", c, 0.0))
    o.refresh_initial()
    o.step(nsteps)
    T = nsteps * dt
    for c in range(3):
        np.testing.assert_allclose(o.field(F[c]), ch * e[c] * np.cos(phase("E", c, T)), rtol=0, atol=5e-12)
        np.testing.assert_allclose(o.field(F[3 + c]), b[c] * np.cos(phase("B", c, T)), rtol=0, atol=5e-12)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_klein_gordon_discrete_dispersion(ndim):
    """phi = cos(k.r - omega t) with (2/dt)^2 sin^2(omega dt/2) =
    sum_d (2/dx_d)^2 sin^2(k_d dx_d/2) + m^2, the discrete form of the
    Klein-Gordon dispersion omega^2 = k^2 + m^2 (Sec. II.A, eq. wave_axion)."""
    n = [24, 18, 10][:ndim] + [1] * (3 - ndim)
    dx = [0.35, 0.3, 0.4][:ndim] + [1.0] * (3 - ndim)
    dt = 0.9 / math.sqrt(sum(1 / dx[d] ** 2 for d in range(ndim)))
    m = 0.7
    kv = [2 * math.pi * (d + 1) / (n[d] * dx[d]) if d < ndim else 0.0 for d in range(3)]
    Om2 = sum((2 / dx[d] * math.sin(kv[d] * dx[d] / 2)) ** 2 for d in range(3)) + m * m
    omega = 2 / dt * math.asin(math.sqrt(Om2) * dt / 2)
    o = Oracle(periodic_cfg(n, dx, dt, m=m))
    x, y, z = positions(n, dx, kind="phi")
    kr = kv[0] * x + kv[1] * y + kv[2] * z
    o.field("PHI_OLD")[...] = np.cos(kr + omega * dt / 2)
    o.field("PHI_NEW")[...] = np.cos(kr - omega * dt / 2)
    o.refresh_initial()
    N = 200
    o.step(N)
    np.testing.assert_allclose(o.field("PHI_OLD"), np.cos(kr - omega * (N - 0.5) * dt), rtol=0, atol=2e-11)
    np.testing.assert_allclose(o.field("PHI_NEW"), np.cos(kr - omega * (N + 0.5) * dt), rtol=0, atol=2e-11)
    # continuum limit of the same relation for a resolved mode: omega^2 = k^2 + m^2 + O(dx^2)
    k1 = 2 * math.pi / (n[0] * dx[0])
    Om2 = (2 / dx[0] * math.sin(k1 * dx[0] / 2)) ** 2 + m * m
    w1 = 2 / dt * math.asin(math.sqrt(Om2) * dt / 2)
    assert abs(w1 ** 2 - (k1 * k1 + m * m)) / (k1 * k1 + m * m) < (k1 * dx[0]) ** 2 / 6


# ---------------------------------------------------------------- invariants

def roll(a, d, s):
    """value at index i + s along axis d (arrays are (z, y, x))."""
    return np.roll(a, -s, axis=2 - d)


def np_curl_B(B, dx):
    """(curl B) at E points, periodic, forward differences."""
    Bx, By, Bz = B
    return [(roll(Bz, 1, 1) - Bz) / dx[1] - (roll(By, 2, 1) - By) / dx[2],
            (roll(Bx, 2, 1) - Bx) / dx[2] - (roll(Bz, 0, 1) - Bz) / dx[0],
            (roll(By, 0, 1) - By) / dx[0] - (roll(Bx, 1, 1) - Bx) / dx[1]]


def test_em_energy_invariant():
    """|B^n|^2 + <E^{n-1/2}, E^{n+1/2}> is constant for the Yee leapfrog in a
    periodic box (the two curls are adjoint); E^{n+-1/2} = E^n -+ (dt/2) curl B^n."""
    rng = np.random.default_rng(11)
    n, dx = [9, 7, 6], [0.4, 0.5, 0.45]
    dt = 0.9 / math.sqrt(sum(1 / h ** 2 for h in dx))
    o = Oracle(periodic_cfg(n, dx, dt))
    for name in F:
        o.field(name)[...] = rng.standard_normal(o.field(name).shape)
    o.refresh_initial()

    def invariant():
        tot = []
        for off in (0, 6):
            E = [o.field(F[off + c]) for c in range(3)]
            B = [o.field(F[off + 3 + c]) for c in range(3)]
            cb = np_curl_B(B, dx)
            tot.append(sum((B[c] ** 2).sum() + (E[c] ** 2).sum() - (dt / 2) ** 2 * (cb[c] ** 2).sum()
                           for c in range(3)))
        return tot

    w0 = invariant()
    o.step(80)
    w1 = invariant()
    for a, b in zip(w0, w1):
        assert abs(a - b) / abs(a) < 1e-12


def test_klein_gordon_energy_invariant():
    """|phi^{L+1} - phi^L|^2/dt^2 + sum_d <D+ phi^{L+1}, D+ phi^L> + m^2 <phi^{L+1}, phi^L>
    is constant for the axion leapfrog without source (periodic box)."""
    rng = np.random.default_rng(12)
    n, dx = [10, 8, 7], [0.4, 0.3, 0.5]
    dt = 0.9 / math.sqrt(sum(1 / h ** 2 for h in dx))
    m = 0.8
    o = Oracle(periodic_cfg(n, dx, dt, m=m))
    o.field("PHI_OLD")[...] = rng.standard_normal(o.field("PHI_OLD").shape)
    o.field("PHI_NEW")[...] = rng.standard_normal(o.field("PHI_OLD").shape)
    o.refresh_initial()

    def invariant():
        a, b = o.field("PHI_OLD"), o.field("PHI_NEW")
        q = (((b - a) / dt) ** 2).sum() + m * m * (a * b).sum()
        for d in range(3):
            q += (((roll(a, d, 1) - a) / dx[d]) * ((roll(b, d, 1) - b) / dx[d])).sum()
        return q

    q0 = invariant()
    o.step(120)
    assert abs(invariant() - q0) / abs(q0) < 1e-12


def test_div_b_stays_zero_with_mur_laser_and_axion():
    """div B0 = div B1 = 0 (Sec. II.A/B): the discrete divergence of the
    discrete curl vanishes, also next to Mur faces and with all couplings on."""
    from paper_2406_16796_amd import workloads as W
    cfg = W.focused_3d(n=24, steps=0, m=0.3, g=0.05, waist_lam=0.6, fwhm_lam=1.0, pk_amp=0.1,
                       pk_w_lam=0.6)
    cfg["t_center"] = 6.0
    o = Oracle(cfg)
    o.step(50)
    dx, n = cfg["dx"], cfg["n"]
    for off in (3, 9):
        Bx, By, Bz = (o.field(F[off + c]) for c in range(3))
        # divergence at nodes whose three neighbouring B points all exist
        div = ((Bx[1:n[2], 1:n[1], 1:n[0]] - Bx[1:n[2], 1:n[1], 0:n[0] - 1]) / dx[0]
               + (By[1:n[2], 1:n[1], 1:n[0]] - By[1:n[2], 0:n[1] - 1, 1:n[0]]) / dx[1]
               + (Bz[1:n[2], 1:n[1], 1:n[0]] - Bz[0:n[2] - 1, 1:n[1], 1:n[0]]) / dx[2])
        scale = max(np.abs(Bx).max(), np.abs(By).max(), np.abs(Bz).max()) / dx[0]
        assert scale > 0.0
        assert np.abs(div).max() <= 1e-12 * scale


def test_gauss_law_with_axion_charge_is_kept():
    """div E1 + g B0 . grad(phi) is constant in time (Sec. II.B, eq. divergence-e1
    with rho1 = 0): with E0 = 0 and a uniform static B0 the scheme keeps the
    discrete form (central gradient of phi^n at centres, face divergence of E1)
    exactly, because the axion current is the time difference of g phi B0."""
    n, dx = [32, 28, 1], [0.3, 0.35, 1.0]
    dt = 0.9 / math.sqrt(1 / dx[0] ** 2 + 1 / dx[1] ** 2)
    g = 0.3
    bext = [0.6, 0.8, 0.25]
    cfg = periodic_cfg(n, dx, dt, g=g, m=0.4, bext=bext, slab_lo=0, slab_hi=n[0], packet_on=1,
                       pk_amp=1.0, pk_k=1.5, pk_w=2.0, pk_x0=4.0, pk_y0=4.5, pk_dir=1)
    o = Oracle(cfg)

    def residual():
        ex, ey = o.field("E1X")[0], o.field("E1Y")[0]
        div = (np.roll(ex, -1, 1) - ex) / dx[0] + (np.roll(ey, -1, 0) - ey) / dx[1]
        ph = 0.5 * (o.field("PHI_OLD")[0] + o.field("PHI_NEW")[0])
        gx = (np.roll(ph, -1, 1) - np.roll(ph, 1, 1)) / (2 * dx[0])
        gy = (np.roll(ph, -1, 0) - np.roll(ph, 1, 0)) / (2 * dx[1])
        return div + g * (bext[0] * gx + bext[1] * gy)

    r0 = residual()
    o.step(90)
    r1 = residual()
    assert np.abs(r0).max() > 1e-3
    assert np.abs(o.field("E1X")).max() > 1e-3
    np.testing.assert_allclose(r1, r0, rtol=0, atol=1e-12 * np.abs(r0).max())


# ------------------------------------------------------------ symmetries

def test_linearity_in_g_is_bit_exact():
    """The perturbation chain E0 -> phi -> E1/B1 is linear: g -> 4 g multiplies
    the generated phi by exactly 4 and E1, B1 by exactly 16 (binary scaling)."""
    from paper_2406_16796_amd import workloads as W
    base = W.gaussian_2d(n=80, steps=0, m=0.1, g=3e-3, slab=(10, 60), waist_lam=1.5, fwhm_lam=2.0)
    base["t_center"] = 8.0
    base["pml_n"] = 8
    runs = []
    for g in (3e-3, 12e-3):
        cfg = dict(base, g=g)
        o = Oracle(cfg)
        o.step(120)
        runs.append(o)
    a, b = runs
    assert np.abs(a.field("PHI_NEW")).max() > 0
    assert np.array_equal(b.field("PHI_NEW"), 4.0 * a.field("PHI_NEW"))
    assert np.array_equal(b.field("PHI_OLD"), 4.0 * a.field("PHI_OLD"))
    for name in F[6:]:
        assert np.array_equal(b.field(name), 16.0 * a.field(name)), name
    for name in F[:6]:
        assert np.array_equal(b.field(name), a.field(name)), name


def test_conversion_fields_linear_in_g_bit_exact():
    """Axion -> photon: with no laser, E1 and B1 scale exactly with g."""
    base = periodic_cfg([40, 30, 1], [0.3, 0.3, 1.0], 0.2, m=0.2, bext=[0.0, 1.0, 0.5],
                        slab_lo=0, slab_hi=40, packet_on=1, pk_amp=1.0, pk_k=1.0, pk_w=2.5,
                        pk_x0=6.0, pk_y0=4.5, pk_dir=1)
    outs = []
    for g in (1e-3, 8e-3):
        o = Oracle(dict(base, g=g))
        o.step(70)
        outs.append(o)
    for name in F[6:]:
        assert np.array_equal(outs[1].field(name), 8.0 * outs[0].field(name)), name
    assert np.abs(outs[0].field("E1Y")).max() > 0


def test_periodic_translation_is_exact():
    """Shifting the initial data of a periodic box by whole cells shifts the
    result by the same cells, bit for bit."""
    rng = np.random.default_rng(5)
    n, dx = [10, 9, 1], [0.4, 0.45, 1.0]
    dt = 0.9 / math.sqrt(1 / dx[0] ** 2 + 1 / dx[1] ** 2)
    cfg = periodic_cfg(n, dx, dt, g=0.2, m=0.5, bext=[0.3, -0.4, 0.7], slab_lo=0, slab_hi=n[0])
    init = {name: rng.standard_normal((1, n[1], n[0])) for name in F + ["PHI_OLD", "PHI_NEW"]}
    sx, sy = 3, 4
    runs = []
    for shift in ((0, 0), (sx, sy)):
        o = Oracle(cfg)
        for name, arr in init.items():
            o.field(name)[...] = np.roll(np.roll(arr, shift[0], axis=2), shift[1], axis=1)
        o.refresh_initial()
        o.step(25)
        runs.append(o)
    for name in init:
        ref = np.roll(np.roll(runs[0].field(name), sx, axis=2), sy, axis=1)
        assert np.array_equal(runs[1].field(name), ref), name


def test_reflect_boundary_equals_method_of_images():
    """Reflect (zero gradient, phi_{-1/2} = phi_{1/2}, Sec. II.D) on both x faces
    is the periodic evolution of the data mirrored about the faces."""
    rng = np.random.default_rng(6)
    nx, ny = 16, 12
    dx = [0.3, 0.35, 1.0]
    dt = 0.9 / math.sqrt(1 / dx[0] ** 2 + 1 / dx[1] ** 2)
    a0 = rng.standard_normal((1, ny, nx))
    a1 = a0 + 0.1 * rng.standard_normal((1, ny, nx))
    A = Oracle(periodic_cfg([nx, ny, 1], dx, dt, m=0.6, ax_bc=[1, 0, 0]))
    A.field("PHI_OLD")[...] = a0
    A.field("PHI_NEW")[...] = a1
    A.refresh_initial()
    B = Oracle(periodic_cfg([2 * nx, ny, 1], dx, dt, m=0.6))
    B.field("PHI_OLD")[...] = np.concatenate([a0[..., ::-1], a0], axis=2)
    B.field("PHI_NEW")[...] = np.concatenate([a1[..., ::-1], a1], axis=2)
    B.refresh_initial()
    A.step(60)
    B.step(60)
    for name in ("PHI_OLD", "PHI_NEW"):
        np.testing.assert_allclose(A.field(name), B.field(name)[..., nx:], rtol=0,
                                   atol=1e-13 * np.abs(B.field(name)).max())


def test_fps_worked_example_ulp():
    """Sec. II.B: E0 = 4e14 V/m has a double-precision step of 2^-4 = 0.0625 V/m,
    so E1 ~ 4e-13 V/m added to it is lost, which is why the orders are stored apart."""
    e0 = 4e14
    assert np.spacing(e0) == 0.0625
    assert math.frexp(e0)[1] - 1 == 48
    assert e0 + 4e-13 == e0
    assert np.float32(4e-13) != 0


# ------------------------------------------------- exact-rational brute force

def _fr_roll(a, d, s):
    return np.roll(a, -s, axis=2 - d)


class RationalScheme:
    """The step of Sec. II.C in exact rationals on a periodic grid, in two forms:
    the paper's half-step form (E, B co-timed) and the leapfrog form (E at
    half-integer times).  Written with numpy object arrays of Fractions."""

    def __init__(self, dx, dt, m, g, bext):
        self.dx, self.dt, self.m, self.g, self.bext = dx, dt, m, g, bext
        self.h = dt / 2

    def curlB(self, B):
        dx = self.dx
        Bx, By, Bz = B
        return [(_fr_roll(Bz, 1, 1) - Bz) / dx[1] - (_fr_roll(By, 2, 1) - By) / dx[2],
                (_fr_roll(Bx, 2, 1) - Bx) / dx[2] - (_fr_roll(Bz, 0, 1) - Bz) / dx[0],
                (_fr_roll(By, 0, 1) - By) / dx[0] - (_fr_roll(Bx, 1, 1) - Bx) / dx[1]]

    def curlE(self, E):
        dx = self.dx
        Ex, Ey, Ez = E
        return [(Ez - _fr_roll(Ez, 1, -1)) / dx[1] - (Ey - _fr_roll(Ey, 2, -1)) / dx[2],
                (Ex - _fr_roll(Ex, 2, -1)) / dx[2] - (Ez - _fr_roll(Ez, 0, -1)) / dx[0],
                (Ey - _fr_roll(Ey, 0, -1)) / dx[0] - (Ex - _fr_roll(Ex, 1, -1)) / dx[1]]

    def ebar(self, E):
        return [(_fr_roll(E[c], c, 1) + E[c]) / 2 for c in range(3)]

    def bbar(self, B):
        out = []
        for c in range(3):
            a, b = [d for d in range(3) if d != c]
            v = B[c] + _fr_roll(B[c], a, 1) + _fr_roll(B[c], b, 1) + _fr_roll(_fr_roll(B[c], a, 1), b, 1)
            out.append(v / 4 + self.bext[c])
        return out

    def source_C(self, E0, B0, pa, pb):
        e, b = self.ebar(E0), self.bbar(B0)
        dtp = (pb - pa) / self.dt
        pm = (pa + pb) / 2
        gp = [(_fr_roll(pm, d, 1) - _fr_roll(pm, d, -1)) / (2 * self.dx[d]) for d in range(3)]
        cr = [e[1] * gp[2] - e[2] * gp[1], e[2] * gp[0] - e[0] * gp[2], e[0] * gp[1] - e[1] * gp[0]]
        return [dtp * b[c] - cr[c] for c in range(3)]

    def face(self, C):
        return [(_fr_roll(C[c], c, -1) + C[c]) / 2 for c in range(3)]

    def phi_next(self, E0h, B0h, pa, pb):
        e, b = self.ebar(E0h), self.bbar(B0h)
        sax = self.g * (e[0] * b[0] + e[1] * b[1] + e[2] * b[2])
        lap = sum((_fr_roll(pb, d, 1) - 2 * pb + _fr_roll(pb, d, -1)) / (self.dx[d] ** 2) for d in range(3))
        return 2 * pb - pa + self.dt ** 2 * (lap - self.m ** 2 * pb + sax)

    def literal_step(self, st):
        E0, B0, E1, B1, pa, pb = st
        h, g = self.h, self.g
        S = self.face(self.source_C(E0, B0, pa, pb))
        cb0, cb1 = self.curlB(B0), self.curlB(B1)
        E0 = [E0[c] + h * cb0[c] for c in range(3)]
        E1 = [E1[c] + h * (cb1[c] - g * S[c]) for c in range(3)]
        ce0, ce1 = self.curlE(E0), self.curlE(E1)
        B0 = [B0[c] - h * ce0[c] for c in range(3)]
        B1 = [B1[c] - h * ce1[c] for c in range(3)]
        pn = self.phi_next(E0, B0, pa, pb)
        B0 = [B0[c] - h * ce0[c] for c in range(3)]
        B1 = [B1[c] - h * ce1[c] for c in range(3)]
        cb0 = self.curlB(B0)
        E0 = [E0[c] + h * cb0[c] for c in range(3)]
        S = self.face(self.source_C(E0, B0, pb, pn))
        cb1 = self.curlB(B1)
        E1 = [E1[c] + h * (cb1[c] - g * S[c]) for c in range(3)]
        return E0, B0, E1, B1, pb, pn

    def to_leapfrog(self, st):
        E0, B0, E1, B1, pa, pb = st
        h, g = self.h, self.g
        S = self.face(self.source_C(E0, B0, pa, pb))
        cb0, cb1 = self.curlB(B0), self.curlB(B1)
        return ([E0[c] - h * cb0[c] for c in range(3)], B0,
                [E1[c] - h * (cb1[c] - g * S[c]) for c in range(3)], B1, pa, pb)

    def leapfrog_step(self, st):
        E0m, B0, E1m, B1, pa, pb = st
        dt, g = self.dt, self.g
        cb0 = self.curlB(B0)
        E0h = [E0m[c] + dt * cb0[c] for c in range(3)]
        E0n = [(E0m[c] + E0h[c]) / 2 for c in range(3)]
        S = self.face(self.source_C(E0n, B0, pa, pb))
        cb1 = self.curlB(B1)
        E1h = [E1m[c] + dt * (cb1[c] - g * S[c]) for c in range(3)]
        ce0, ce1 = self.curlE(E0h), self.curlE(E1h)
        B0n = [B0[c] - dt * ce0[c] for c in range(3)]
        B1n = [B1[c] - dt * ce1[c] for c in range(3)]
        pn = self.phi_next(E0h, [(B0[c] + B0n[c]) / 2 for c in range(3)], pa, pb)
        return E0h, B0n, E1h, B1n, pb, pn

    def co_timed(self, st):
        """E^n = (E^{n-1/2} + E^{n+1/2}) / 2 from a leapfrog state."""
        E0m, B0, E1m, B1, pa, pb = st
        nxt = self.leapfrog_step(st)
        return ([(E0m[c] + nxt[0][c]) / 2 for c in range(3)], B0,
                [(E1m[c] + nxt[2][c]) / 2 for c in range(3)], B1, pa, pb)


def test_brute_force_exact_rationals_both_forms_and_oracle():
    """On a 5x4x3 periodic grid with every coupling on and dyadic inputs: the
    paper's half-step form and the leapfrog form agree exactly in rationals
    (which is what licenses the GPU's leapfrog storage), and the FP64 oracle
    stays within a few ulp per step of the exact result."""
    n = (5, 4, 3)
    dx = [Fraction(1, 2), Fraction(1, 2), Fraction(1, 2)]
    dt = Fraction(1, 4)
    m, g = Fraction(1, 2), Fraction(3, 8)
    bext = [Fraction(1, 4), Fraction(-1, 2), Fraction(3, 4)]
    rng = np.random.default_rng(7)

    def dy():
        a = np.empty((n[2], n[1], n[0]), dtype=object)
        for idx, v in np.ndenumerate(rng.integers(-32, 33, size=a.shape)):
            a[idx] = Fraction(int(v), 64)
        return a

    st = ([dy() for _ in range(3)], [dy() for _ in range(3)], [dy() for _ in range(3)],
          [dy() for _ in range(3)], dy(), dy())
    scheme = RationalScheme(dx, dt, m, g, bext)
    nsteps = 4
    lit, lf = st, scheme.to_leapfrog(st)
    for _ in range(nsteps):
        lit = scheme.literal_step(lit)
        lf = scheme.leapfrog_step(lf)
    lf_ct = scheme.co_timed(lf)
    for a_list, b_list in zip(lit[:4], lf_ct[:4]):
        for a, b in zip(a_list, b_list):
            assert (a == b).all()
    assert (lit[4] == lf_ct[4]).all() and (lit[5] == lf_ct[5]).all()

    cfg = periodic_cfg(list(n), [float(v) for v in dx], float(dt), m=float(m), g=float(g),
                       bext=[float(v) for v in bext], slab_lo=0, slab_hi=n[0])
    o = Oracle(cfg)
    names = F + ["PHI_OLD", "PHI_NEW"]
    init = list(st[0]) + list(st[1]) + list(st[2]) + list(st[3]) + [st[4], st[5]]
    for name, arr in zip(names, init):
        o.field(name)[...] = arr.astype(float)
    o.refresh_initial()
    o.step(nsteps)
    final = list(lit[0]) + list(lit[1]) + list(lit[2]) + list(lit[3]) + [lit[4], lit[5]]
    for name, arr in zip(names, final):
        exact = arr.astype(float)
        scale = max(np.abs(exact).max(), 1.0)
        assert np.abs(o.field(name) - exact).max() <= 1e-13 * scale, name


# ---------------------------------------------------------------- laser centroid

def test_laser_centroid_closed_forms():
    """x_laser = sum x B1z^2 / sum B1z^2 with B1z on the x nodes (x = i dx):
    one point sits at its node; two points weigh by the square (not the
    value); a profile even about a node has its centroid there; no field
    gives 0."""
    b = np.zeros((1, 3, 7))
    b[0, 1, 4] = 3.0
    assert laser_centroid(b, 0.5) == 2.0
    b = np.zeros((2, 4, 9))
    b[0, 1, 2] = 1.0
    b[1, 3, 6] = -2.0
    # (1 * 2 + 4 * 6) / (1 + 4) = 26/5 columns
    assert laser_centroid(b, 0.5) == pytest.approx(float(Fraction(26, 5) * Fraction(1, 2)), rel=1e-15)
    x = np.arange(21)
    prof = np.exp(-0.5 * ((x - 10) / 3.0) ** 2)
    rows = np.array([0.3, 1.0, 2.5])[:, None]
    assert laser_centroid((rows * prof)[None], 0.25) == pytest.approx(2.5, rel=1e-14)
    assert laser_centroid(np.zeros((1, 2, 5)), 1.0) == 0.0


def conversion_cfg(x0):
    # a box long enough in x (48) that the packet and its photons stay far
    # from its ends: a centroid moves with a shift only while nothing wraps
    return periodic_cfg([160, 30, 1], [0.3, 0.3, 1.0], 0.2, m=0.2, g=5e-3, bext=[0.0, 1.0, 0.5],
                        slab_lo=0, slab_hi=160, packet_on=1, pk_amp=1.0, pk_k=1.0, pk_w=2.5,
                        pk_x0=x0, pk_y0=4.5, pk_dir=1)


def test_laser_centroid_of_oracle_run():
    """The oracle's x_laser of the photons an axion packet generates: the sum
    written out over every B1z point of the grid, and a whole-cell shift of
    the packet in a periodic box (uniform field everywhere) shifts it by
    exactly those cells."""
    o = Oracle(conversion_cfg(20.0))
    o.step(20)
    b = o.field("B1Z")
    num = den = 0.0
    for k in range(o.n[2]):
        for j in range(o.nn[1]):
            for i in range(o.nn[0]):
                num += i * 0.3 * b[k, j, i] ** 2
                den += b[k, j, i] ** 2
    assert den > 0
    xc = o.laser_centroid()
    assert xc == pytest.approx(num / den, rel=1e-13)
    s = Oracle(conversion_cfg(20.0 + 3 * 0.3))
    s.step(20)
    assert s.laser_centroid() - xc == pytest.approx(0.9, abs=1e-9)
