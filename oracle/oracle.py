"""ctypes wrapper of the FP64 CPU oracle (oracle/axion_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the package smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never imports it.

A run is described by a plain dict whose keys are the fields of
``ora_config`` (see axion_oracle.h); missing keys take neutral defaults.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

EM_PERIODIC, EM_MUR = 0, 1
AX_PERIODIC, AX_REFLECT, AX_OUTFLOW, AX_PML = 0, 1, 2, 3
ENV_CW, ENV_GAUSS = 0, 1

FIELD_IDS = {name: i for i, name in enumerate(
    ["E0X", "E0Y", "E0Z", "B0X", "B0Y", "B0Z",
     "E1X", "E1Y", "E1Z", "B1X", "B1Y", "B1Z", "PHI_OLD", "PHI_NEW"])}


class OraConfig(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3), ("dt", ctypes.c_double),
        ("em_bc", ctypes.c_int * 3), ("ax_bc", ctypes.c_int * 3),
        ("pml_n", ctypes.c_int), ("pml_sigma_dt", ctypes.c_double),
        ("m", ctypes.c_double), ("g", ctypes.c_double),
        ("bext", ctypes.c_double * 3), ("slab_lo", ctypes.c_int), ("slab_hi", ctypes.c_int),
        ("laser_on", ctypes.c_int), ("laser_pol", ctypes.c_int), ("laser_env", ctypes.c_int),
        ("omega", ctypes.c_double), ("e_amp", ctypes.c_double), ("ramp_periods", ctypes.c_double),
        ("fwhm", ctypes.c_double), ("t_center", ctypes.c_double), ("waist", ctypes.c_double),
        ("x_focus", ctypes.c_double), ("y_c", ctypes.c_double), ("z_c", ctypes.c_double),
        ("cep", ctypes.c_double),
        ("packet_on", ctypes.c_int),
        ("pk_amp", ctypes.c_double), ("pk_k", ctypes.c_double), ("pk_w", ctypes.c_double),
        ("pk_x0", ctypes.c_double), ("pk_y0", ctypes.c_double), ("pk_z0", ctypes.c_double),
        ("pk_dir", ctypes.c_int),
        ("laser_order", ctypes.c_int), ("ppc", ctypes.c_int * 2), ("plasma_n", ctypes.c_double),
        ("plasma_lo", ctypes.c_int), ("plasma_hi", ctypes.c_int), ("plasma_u", ctypes.c_double * 3),
    ]


def build(force=False, src=None, out=None, defines=()):
    """Compile liboracle.so with gcc (plain -O2, no FP contraction).  `src`,
    `out` and `defines` build another copy of the source (the tests'
    planted-mistake variants, the literal reading of Sec. II.C) into another
    library."""
    src = src or os.path.join(HERE, "axion_oracle.c")
    out = out or LIB_PATH
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=gnu99", "-Wall", "-I", HERE] + ["-D" + d for d in defines] + ["-o", out + ".tmp", src, "-lm"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = load(LIB_PATH)
    return _lib


def load(path):
    """A built oracle library with its call signatures declared."""
    L = ctypes.CDLL(path)
    L.ora_create.argtypes = [ctypes.POINTER(OraConfig), ctypes.POINTER(ctypes.c_void_p)]
    L.ora_create.restype = ctypes.c_int
    L.ora_destroy.argtypes = [ctypes.c_void_p]
    L.ora_extents.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
    L.ora_field.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.ora_field.restype = ctypes.POINTER(ctypes.c_double)
    L.ora_axion_ghost.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.ora_axion_ghost.restype = ctypes.POINTER(ctypes.c_double)
    L.ora_refresh_initial.argtypes = [ctypes.c_void_p]
    L.ora_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
    L.ora_shift_window.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.ora_shift_window.restype = ctypes.c_int
    L.ora_step_count.argtypes = [ctypes.c_void_p]
    L.ora_step_count.restype = ctypes.c_long
    L.ora_energies.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    L.ora_incident.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_double] * 4
    L.ora_incident.restype = ctypes.c_double
    L.ora_particles.argtypes = [ctypes.c_void_p]
    L.ora_particles.restype = ctypes.c_long
    L.ora_particle_array.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.ora_particle_array.restype = ctypes.POINTER(ctypes.c_double)
    L.ora_current.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.ora_current.restype = ctypes.POINTER(ctypes.c_double)
    L.ora_redeposit.argtypes = [ctypes.c_void_p]
    L.ora_redeposit.restype = None
    L.ora_threads.restype = ctypes.c_int
    L.ora_set_threads.argtypes = [ctypes.c_int]
    L.ora_set_threads.restype = None
    return L


def make_config(cfg):
    c = OraConfig()
    c.n[:] = [int(v) for v in cfg.get("n", [1, 1, 1])]
    c.dx[:] = [float(v) for v in cfg.get("dx", [1.0, 1.0, 1.0])]
    c.dt = float(cfg["dt"])
    c.em_bc[:] = [int(v) for v in cfg.get("em_bc", [0, 0, 0])]
    c.ax_bc[:] = [int(v) for v in cfg.get("ax_bc", [0, 0, 0])]
    c.pml_n = int(cfg.get("pml_n", 20))
    c.pml_sigma_dt = float(cfg.get("pml_sigma_dt", 0.2))
    c.m = float(cfg.get("m", 0.0))
    c.g = float(cfg.get("g", 0.0))
    c.bext[:] = [float(v) for v in cfg.get("bext", [0.0, 0.0, 0.0])]
    c.slab_lo = int(cfg.get("slab_lo", 0))
    c.slab_hi = int(cfg.get("slab_hi", c.n[0]))
    for key in ("laser_on", "laser_pol", "laser_env", "packet_on", "pk_dir"):
        setattr(c, key, int(cfg.get(key, 0)))
    for key in ("omega", "e_amp", "ramp_periods", "fwhm", "t_center", "waist", "x_focus",
                "y_c", "z_c", "cep", "pk_amp", "pk_k", "pk_w", "pk_x0", "pk_y0", "pk_z0"):
        setattr(c, key, float(cfg.get(key, 0.0)))
    c.laser_order = int(cfg.get("laser_order", 0))
    c.ppc[:] = [int(v) for v in cfg.get("ppc", [0, 1])]
    c.plasma_n = float(cfg.get("plasma_n", 0.0))
    c.plasma_lo = int(cfg.get("plasma_lo", 0))
    c.plasma_hi = int(cfg.get("plasma_hi", c.n[0]))
    c.plasma_u[:] = [float(v) for v in cfg.get("plasma_u", [0.0, 0.0, 0.0])]
    if c.laser_on and c.omega == 0.0:
        raise ValueError("laser needs omega > 0")
    return c


def laser_centroid(b1z, dx):
    """Laser centroid along x (Sec. III.D, the weak-laser benchmark): the mean
    of x over the grid weighted by the first-order field squared,
    x_laser = sum x B1z^2 / sum B1z^2, summed over every B1z point of the
    grid (the paper's double integral over x and y, a triple one in 3D).  B1z
    lies on the z edges of the cells, i.e. on the x nodes: the point of
    column i is at x = i dx.  0 where B1z vanishes everywhere.

    b1z: array (..., nx) of the grid's B1z points, column i last."""
    b = np.asarray(b1z, dtype=np.float64)
    w = b * b
    tot = w.sum()
    if tot == 0.0:
        return 0.0
    x = np.arange(b.shape[-1], dtype=np.float64) * dx
    return float((w * x).sum() / tot)


class Oracle:
    """One FP64 oracle run; arrays are numpy views on the oracle's memory."""

    def __init__(self, cfg, library=None):
        """`library`: another build of the oracle (load()); the default one otherwise."""
        self._L = library or lib()
        self._cfg = make_config(cfg)
        h = ctypes.c_void_p()
        if self._L.ora_create(ctypes.byref(self._cfg), ctypes.byref(h)) != 0:
            raise ValueError("oracle rejected the configuration")
        self._h = h
        nn = (ctypes.c_int * 3)()
        self._L.ora_extents(h, nn)
        self.nn = tuple(nn)
        self.n = tuple(self._cfg.n)

    def close(self):
        if self._h:
            self._L.ora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field(self, name):
        """Array of field `name` with shape (nn_z, nn_y, nn_x): a live view."""
        p = self._L.ora_field(self._h, FIELD_IDS[name])
        nz, ny, nx = self.nn[2], self.nn[1], self.nn[0]
        return np.ctypeslib.as_array(p, shape=(nz * ny * nx,)).reshape(nz, ny, nx)

    def axion_ghost(self, d, side, level):
        p = self._L.ora_axion_ghost(self._h, d, side, level)
        if not p:
            return None
        a, b = [e for e in range(3) if e != d]
        return np.ctypeslib.as_array(p, shape=(self.nn[a] * self.nn[b],)).reshape(self.nn[b], self.nn[a])

    def refresh_initial(self):
        self._L.ora_refresh_initial(self._h)

    def step(self, nsteps=1):
        self._L.ora_step(self._h, int(nsteps))

    def shift_window(self, cells):
        """Move the window `cells` columns along +x (Sec. III.B)."""
        if self._L.ora_shift_window(self._h, int(cells)) != 0:
            raise ValueError("window move rejected")

    @property
    def step_count(self):
        return self._L.ora_step_count(self._h)

    def energies(self):
        out = (ctypes.c_double * 3)()
        self._L.ora_energies(self._h, out)
        return tuple(out)

    def laser_centroid(self):
        """x_laser of B1z at the current integer time (B_z points: every x and
        y node, the cell centres along z)."""
        b = self.field("B1Z")[:self.n[2], :self.nn[1], :self.nn[0]]
        return laser_centroid(b, float(self._cfg.dx[0]))

    def threads(self):
        return self._L.ora_threads()

    @staticmethod
    def set_threads(n):
        """Threads of the oracle's loops from now on (timing only)."""
        lib().ora_set_threads(int(n))

    PARTICLE_IDS = {"x": 0, "y": 1, "z": 2, "ux": 3, "uy": 4, "uz": 5, "x1": 6, "y1": 7, "z1": 8,
                    "u1x": 9, "u1y": 10, "u1z": 11, "w": 12}

    @property
    def n_particles(self):
        return self._L.ora_particles(self._h)

    def particles(self, name):
        """Particle array `name` (x, y, z, ux, uy, uz, their first-order
        x1 ... u1z, w): a live view."""
        p = self._L.ora_particle_array(self._h, self.PARTICLE_IDS[name])
        if not p:
            return None
        return np.ctypeslib.as_array(p, shape=(self.n_particles,))

    def current(self, order, comp):
        """j of order 0/1, component 0-2 at the E points (t_n): a live view."""
        p = self._L.ora_current(self._h, int(order), int(comp))
        if not p:
            return None
        nz, ny, nx = self.nn[2], self.nn[1], self.nn[0]
        return np.ctypeslib.as_array(p, shape=(nz * ny * nx,)).reshape(nz, ny, nx)

    def redeposit(self):
        """j at t_n again from the particle arrays (after editing them)."""
        self._L.ora_redeposit(self._h)

    def incident(self, comp, x, y, z, t):
        return self._L.ora_incident(self._h, comp, x, y, z, t)
