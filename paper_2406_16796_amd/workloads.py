"""Seeded synthetic run descriptions for the conversion workloads.

This module only chooses parameters: grid sizes, spacings, boundary kinds,
laser and axion-packet settings, and the random draws of the scans.  It holds
none of the scheme's arithmetic, so both the GPU library's tests and the CPU
oracle take their inputs from here.

Units: natural units with c = 1, frequencies, wave numbers and masses in
units of the reference laser frequency omega_0 = k_0 (so the reference
wavelength is 2*pi).  Field amplitudes are normalised: a laser of normalised
vector potential a0 at frequency omega has peak field a0*omega.  These are the
units of the generation and conversion benchmarks of Sec. III (their packet is
sin(k_0 eta), their probability formula is in natural units).

A run description is a plain dict whose keys are the fields of the C run
configuration (n, dx, dt, em_bc, ax_bc, ...), plus "steps" and "name".
"""
import math

import numpy as np

BASE_SEED = 2406167960

EM_PERIODIC, EM_MUR = 0, 1
AX_PERIODIC, AX_REFLECT, AX_OUTFLOW, AX_PML = 0, 1, 2, 3
ENV_CW, ENV_GAUSS = 0, 1

TWO_PI = 2.0 * math.pi


def _base(n, dx, dt):
    return dict(n=list(n), dx=list(dx), dt=dt, em_bc=[0, 0, 0], ax_bc=[0, 0, 0],
                pml_n=20, pml_sigma_dt=0.2, m=0.0, g=0.0, bext=[0.0, 0.0, 0.0],
                slab_lo=0, slab_hi=n[0], laser_on=0, laser_pol=1, laser_env=ENV_CW,
                omega=1.0, e_amp=0.0, ramp_periods=4.0, fwhm=0.0, t_center=0.0,
                waist=0.0, x_focus=0.0, y_c=0.0, z_c=0.0, cep=0.0, packet_on=0,
                pk_amp=0.0, pk_k=1.0, pk_w=1.0, pk_x0=0.0, pk_y0=0.0, pk_z0=0.0, pk_dir=1)


def yee_dt(dx, ndim, courant=0.95):
    """Time step at `courant` times the Yee stability limit of the active axes."""
    return courant / math.sqrt(sum(1.0 / (h * h) for h in dx[:ndim]))


def plane_wave_1d(nx=4096, steps=3000, m=0.1, g=1e-4, a0=1e-3, b0=1.0, ppw=20, omega=1.0,
                  ax_bc=AX_PERIODIC):
    """1D CW plane wave (E along y) entering through x_min into a uniform
    transverse B0 along y; Mur EM boundaries.  Default: the 4096-cell,
    3000-step FP64 conversion run (lambda/20, dt = 0.95 dx)."""
    lam = TWO_PI / omega
    dx = lam / ppw
    # dt = 0.95 dx unless that passes the Klein-Gordon limit of the leapfrog,
    # dx / sqrt(1 + (m dx / 2)^2) (heavy axions on coarse grids): then 0.95 of it
    limit = dx / math.sqrt(1.0 + (m * dx / 2.0) ** 2)
    cfg = _base([nx, 1, 1], [dx, 1.0, 1.0], 0.95 * dx if 0.95 * dx <= limit else 0.95 * limit)
    cfg.update(em_bc=[EM_MUR, 0, 0], ax_bc=[ax_bc, 0, 0], m=m, g=g, bext=[0.0, b0, 0.0],
               laser_on=1, laser_pol=1, laser_env=ENV_CW, omega=omega, e_amp=a0 * omega,
               ramp_periods=4.0, steps=steps, name="1d_cw_%d" % nx)
    return cfg


def gaussian_2d(n=4096, steps=6000, m=0.0, g=1e-5, a0=1e-2, ppw=16, waist_lam=8.0,
                fwhm_lam=10.0, slab=(1024, 3072), ax_bc=AX_PML, seed=1):
    """2D Gaussian pulse (E in plane, along y) crossing a slab of uniform
    B0 along y.  Default: 4096^2 cells at lambda/16, 6000 steps, waist 8
    lambda, FWHM 10 lambda, a0 = 1e-2, seeded CEP, axion PML, Mur EM."""
    rng = np.random.default_rng(BASE_SEED + 1 + 1000 * seed)
    lam = TWO_PI
    dx = lam / ppw
    cfg = _base([n, n, 1], [dx, dx, 1.0], yee_dt([dx, dx], 2))
    lo, hi = slab
    cfg.update(em_bc=[EM_MUR, EM_MUR, 0], ax_bc=[ax_bc, ax_bc, 0], m=m, g=g,
               bext=[0.0, 1.0, 0.0], slab_lo=int(lo), slab_hi=int(hi),
               laser_on=1, laser_pol=1, laser_env=ENV_GAUSS, omega=1.0, e_amp=a0,
               fwhm=fwhm_lam * lam, t_center=3.0 * fwhm_lam * lam, waist=waist_lam * lam,
               x_focus=0.5 * (lo + hi) * dx, y_c=0.5 * n * dx,
               cep=float(rng.uniform(0.0, TWO_PI)), steps=steps, name="2d_gauss_%d_m%g" % (n, m))
    return cfg


def gaussian_2d_window(win_cells=8, **kw):
    """The 2D Gaussian-pulse run (gaussian_2d) with a moving window from the
    first step on (Sec. III.B): each time the light has crossed win_cells
    columns, the window moves by as many."""
    cfg = gaussian_2d(**kw)
    cfg.update(win_cells=win_cells, win_t0=cfg["dt"], name="%s_window%d" % (cfg["name"], win_cells))
    return cfg


def focused_3d(n=512, steps=2000, m=0.3, g=1e-4, a0=1e-2, ppw=12, waist_lam=6.0,
               fwhm_lam=10.0, pk_amp=1e-3, pk_w_lam=5.0, seed=2):
    """3D focused Gaussian pulse (E along z) from x_min plus a counter-
    propagating Gaussian axion packet from the x_max side, in a uniform B0
    along z; Mur EM and outflow axion boundaries.  Default: 512^3 cells at
    lambda/12, 2000 steps."""
    rng = np.random.default_rng(BASE_SEED + 2 + 1000 * seed)
    lam = TWO_PI
    dx = lam / ppw
    L = n * dx
    cfg = _base([n, n, n], [dx, dx, dx], yee_dt([dx, dx, dx], 3))
    w = pk_w_lam * lam
    cfg.update(em_bc=[EM_MUR] * 3, ax_bc=[AX_OUTFLOW] * 3, m=m, g=g, bext=[0.0, 0.0, 1.0],
               laser_on=1, laser_pol=2, laser_env=ENV_GAUSS, omega=1.0, e_amp=a0,
               fwhm=fwhm_lam * lam, t_center=3.0 * fwhm_lam * lam, waist=waist_lam * lam,
               x_focus=0.5 * L, y_c=0.5 * L, z_c=0.5 * L, cep=float(rng.uniform(0.0, TWO_PI)),
               packet_on=1, pk_amp=pk_amp, pk_k=1.0, pk_w=w, pk_x0=max(0.5 * L, L - 3.0 * w),
               pk_y0=0.5 * L, pk_z0=0.5 * L, pk_dir=-1, steps=steps, name="3d_focus_%d" % n)
    return cfg


def weak_laser_plasma_2d(nx=12000, ny=100, n0=3e-3, pulse_fwhm_periods=2.0, plasma_from_lam=2.0,
                         b_over_bc=1e-20, plasma=True):
    """The FPS check of Sec. III.D: a laser so weak (its magnetic field 1e-20
    B_c) that it is carried by the first-order fields alone, propagating
    along x through a plasma of density n0 (critical densities) magnetised
    along z by B_c = m_e omega_p / e (normalised: B_c = omega_p =
    sqrt(n0), so omega_c = omega_p), polarised along y (perpendicular to
    B_c: the extraordinary wave).  Box 40 x 100 lambda0 on 12000 x 100
    cells (lambda0/300 along x), Mur x faces, periodic y; cold electrons,
    one per cell, at rest in the cells from plasma_from_lam to 2 cells before
    x_max; a Gaussian plane-wave pulse of pulse_fwhm_periods periods (FWHM).
    plasma=False: the same run in vacuum."""
    lam = TWO_PI
    dx, dy = 40.0 * lam / nx, 100.0 * lam / ny
    cfg = _base([nx, ny, 1], [dx, dy, 1.0], yee_dt([dx, dy], 2))
    bc = math.sqrt(n0)
    fwhm = pulse_fwhm_periods * lam
    tau0 = fwhm / math.sqrt(2.0 * math.log(2.0))
    cfg.update(ndim=2, em_bc=[EM_MUR, EM_PERIODIC, 0], ax_bc=[AX_OUTFLOW, AX_PERIODIC, 0], m=0.0, g=0.0,
               bext=[0.0, 0.0, bc], slab_lo=0, slab_hi=nx, laser_on=1, laser_pol=1, laser_env=ENV_GAUSS,
               laser_order=1, omega=1.0, e_amp=b_over_bc * bc, fwhm=fwhm, t_center=3.0 * tau0, waist=0.0,
               name="fps_weak_laser_%dx%d" % (nx, ny))
    if plasma:
        cfg.update(ppc=[1, 1], plasma_n=n0, plasma_lo=int(round(plasma_from_lam * lam / dx)), plasma_hi=nx - 2,
                   plasma_u=[0.0, 0.0, 0.0])
    return cfg


def xmode_group_velocity(n0, omega=1.0, omega_c=None):
    """Group velocity of the extraordinary wave in a cold magnetised plasma
    (Sec. III.D): eta^2 = 1 - (wp^2/w^2)(w^2 - wp^2)/(w^2 - wp^2 - wc^2) and
    v_g = c eta / (eta^2 + w^2 d(eta^2)/d(w^2)), the derivative in closed
    form; wc = wp when omega_c is None."""
    a = n0
    c2 = a if omega_c is None else omega_c ** 2
    w = omega * omega
    eta2 = 1.0 - (a / w) * (w - a) / (w - a - c2)
    # d/dw of (a/w)(w - a)/(w - a - c2)
    f = (w - a) / (w * (w - a - c2))
    df = ((w * (w - a - c2)) - (w - a) * (2.0 * w - a - c2)) / (w * (w - a - c2)) ** 2
    deta2 = -a * df
    eta = math.sqrt(eta2)
    return eta / (eta2 + w * deta2), eta


def packet_2d(n=400, ppw=10, m=None, w_lam=5.0, ax_bc=AX_OUTFLOW, steps=None):
    """Left-moving Gaussian axion packet of the boundary check of Sec. III.A:
    box [-20, 20] lambda squared on 400x400 cells, w = 5 lambda, k = k_0,
    m = 1 meV at 800 nm (1 meV / 1.55 eV = 6.45e-4 omega_0).  The origin of
    the grid is the box corner, so the box centre is at 20 lambda."""
    lam = TWO_PI
    dx = lam / ppw
    if m is None:
        m = 1e-3 / 1.5498
    cfg = _base([n, n, 1], [dx, dx, 1.0], yee_dt([dx, dx], 2))
    L = n * dx
    if steps is None:
        steps = int(round(0.75 * L / cfg["dt"]))
    cfg.update(em_bc=[0, 0, 0], ax_bc=[ax_bc, ax_bc, 0], m=m, g=0.0, packet_on=1, pk_amp=1.0,
               pk_k=1.0, pk_w=w_lam * lam, pk_x0=0.5 * L, pk_y0=0.5 * L, pk_dir=-1,
               steps=steps, name="2d_packet_%d" % n)
    return cfg


def scan_runs(count=512, seed=0, n1d=(1024, 65536), n2d=(256, 1024), steps=(1000, 5000),
              frac_1d=0.5):
    """Parameter scan of independent conversion runs: half 1D (CW, periodic
    axion), half 2D (Gaussian pulse, PML axion); m log-uniform in [1e-3, 1],
    g log-uniform in [1e-6, 1e-3], B0 uniform in [0.5, 2], omega uniform in
    [0.5, 4]; 16 cells per laser wavelength; Mur EM."""
    rng = np.random.default_rng(BASE_SEED + 3 + 1000 * seed)
    runs = []
    for r in range(count):
        is1d = r < int(round(frac_1d * count))
        m = float(10.0 ** rng.uniform(-3.0, 0.0))
        g = float(10.0 ** rng.uniform(-6.0, -3.0))
        b0 = float(rng.uniform(0.5, 2.0))
        omega = float(rng.uniform(0.5, 4.0))
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        if is1d:
            nx = int(round(10.0 ** rng.uniform(math.log10(n1d[0]), math.log10(n1d[1]))))
            cfg = plane_wave_1d(nx=nx, steps=nsteps, m=m, g=g, a0=1e-2, b0=b0, ppw=16, omega=omega)
        else:
            side = int(round(10.0 ** rng.uniform(math.log10(n2d[0]), math.log10(n2d[1]))))
            lam = TWO_PI / omega
            dx = lam / 16
            cfg = _base([side, side, 1], [dx, dx, 1.0], yee_dt([dx, dx], 2))
            L = side * dx
            cfg.update(em_bc=[EM_MUR, EM_MUR, 0], ax_bc=[AX_PML, AX_PML, 0], m=m, g=g,
                       bext=[0.0, b0, 0.0], laser_on=1, laser_pol=1, laser_env=ENV_GAUSS,
                       omega=omega, e_amp=1e-2 * omega, fwhm=4.0 * lam, t_center=12.0 * lam,
                       waist=L / 6.0, x_focus=0.5 * L, y_c=0.5 * L,
                       cep=float(rng.uniform(0.0, TWO_PI)), steps=nsteps)
        cfg["name"] = "scan_%03d" % r
        runs.append(cfg)
    return runs


def serving_requests(count=2000, rate=100.0, seed=0, frac_3d=0.1, n3d=(128, 256)):
    """Poisson arrival trace of conversion requests: 90% drawn like the scan,
    10% 3D with side log-uniform in [128, 256]; steps uniform in [1000, 5000].
    Returns a list of (arrival_time_s, cfg)."""
    rng = np.random.default_rng(BASE_SEED + 4 + 1000 * seed)
    scan = scan_runs(count=count, seed=seed + 17)
    order = rng.permutation(count)     # the scan lists its 1D runs first
    out, t = [], 0.0
    for r in range(count):
        t += float(rng.exponential(1.0 / rate))
        if rng.uniform() < frac_3d:
            side = int(round(10.0 ** rng.uniform(math.log10(n3d[0]), math.log10(n3d[1]))))
            cfg = focused_3d(n=side, steps=int(rng.integers(1000, 5001)), seed=100 + r)
            cfg["name"] = "req3d_%04d" % r
        else:
            cfg = dict(scan[int(order[r])])
            cfg["name"] = "req_%04d" % r
        out.append((t, cfg))
    return out


def active_cells(cfg):
    n = cfg["n"]
    return int(n[0]) * int(n[1]) * int(n[2])
