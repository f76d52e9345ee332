"""ctypes binding of libaxf.so (include/axf.h): argument marshalling only.

Every step of the solver runs in the library's HIP kernels.  PyTorch is used
for device memory (a uint8 tensor the library carves its arrays from) and for
the HIP stream handle.  Loading fails loudly if libaxf.so is missing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaxf.so")

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, EBUSY, ENOTFOUND, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
F32, F64 = 0, 1
PATH_AUTO, PATH_PLAIN, PATH_FUSED = 0, 1, 2

FIELDS = ["E0X", "E0Y", "E0Z", "B0X", "B0Y", "B0Z", "E1X", "E1Y", "E1Z", "B1X", "B1Y", "B1Z",
          "PHI_OLD", "PHI_NEW"]
FIELD_ID = {n: i for i, n in enumerate(FIELDS)}

EXPORTS = [
    "axf_last_error", "axf_version", "axf_footprint", "axf_extents", "axf_create", "axf_write_field",
    "axf_step", "axf_read_field", "axf_read_particles", "axf_diag_now", "axf_diag_now_static", "axf_read_diag", "axf_state_bytes", "axf_read_state",
    "axf_write_state", "axf_sync", "axf_steps_done", "axf_path_in_use", "axf_destroy", "axf_last_step_timing",
    "axf_tune", "axf_tune_reset", "axf_batch_footprint", "axf_batch_create", "axf_batch_step", "axf_batch_run", "axf_batch_destroy",
    "axf_server_create", "axf_server_submit", "axf_server_cancel", "axf_server_poll", "axf_server_stats",
    "axf_server_destroy", "axf_config_from_si", "axf_axion_coupling",
]


class AxfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("axf error %d: %s" % (code, msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double * 3),
        ("dt", ctypes.c_double), ("precision", ctypes.c_int32),
        ("em_bc", ctypes.c_int32 * 3), ("ax_bc", ctypes.c_int32 * 3),
        ("pml_n", ctypes.c_int32), ("pml_sigma_dt", ctypes.c_double),
        ("m", ctypes.c_double), ("g", ctypes.c_double), ("bext", ctypes.c_double * 3),
        ("slab_lo", ctypes.c_int32), ("slab_hi", ctypes.c_int32),
        ("laser_on", ctypes.c_int32), ("laser_pol", ctypes.c_int32), ("laser_env", ctypes.c_int32),
        ("omega", ctypes.c_double), ("e_amp", ctypes.c_double), ("ramp_periods", ctypes.c_double),
        ("fwhm", ctypes.c_double), ("t_center", ctypes.c_double), ("waist", ctypes.c_double),
        ("x_focus", ctypes.c_double), ("y_c", ctypes.c_double), ("z_c", ctypes.c_double),
        ("cep", ctypes.c_double),
        ("packet_on", ctypes.c_int32),
        ("pk_amp", ctypes.c_double), ("pk_k", ctypes.c_double), ("pk_w", ctypes.c_double),
        ("pk_x0", ctypes.c_double), ("pk_y0", ctypes.c_double), ("pk_z0", ctypes.c_double),
        ("pk_dir", ctypes.c_int32),
        ("diag_every", ctypes.c_int32), ("path", ctypes.c_int32),
        ("win_t0", ctypes.c_double), ("win_cells", ctypes.c_int32),
        ("laser_order", ctypes.c_int32), ("ppc", ctypes.c_int32 * 2), ("plasma_n", ctypes.c_double),
        ("plasma_lo", ctypes.c_int32), ("plasma_hi", ctypes.c_int32), ("plasma_u", ctypes.c_double * 3),
    ]


class DiagRecord(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double), ("h_phi", ctypes.c_double),
                ("h_em0", ctypes.c_double), ("h_em1", ctypes.c_double), ("p_gen", ctypes.c_double),
                ("p_conv", ctypes.c_double), ("finite", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("x_laser", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class Tuning(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("chunk", ctypes.c_int32), ("prefetch", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("steps_per_pass", ctypes.c_int32), ("frame_chunk", ctypes.c_int32),
                ("ms_per_step", ctypes.c_double), ("default_ms_per_step", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("cells", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("final", DiagRecord)]


_lib = None


class Si(ctypes.Structure):
    """axf_si: SI inputs of a run."""
    _fields_ = [("lambda0", ctypes.c_double), ("lambda_laser", ctypes.c_double),
                ("dx", ctypes.c_double * 3), ("dt", ctypes.c_double), ("m_a", ctypes.c_double),
                ("g_agg", ctypes.c_double), ("bext", ctypes.c_double * 3), ("e_amp", ctypes.c_double),
                ("fwhm", ctypes.c_double), ("t_center", ctypes.c_double), ("waist", ctypes.c_double),
                ("x_focus", ctypes.c_double), ("y_c", ctypes.c_double), ("z_c", ctypes.c_double)]


def lib():
    """Load libaxf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libaxf.so is not built (run __graft_entry__.build() or "
                           "python paper_2406_16796_amd/build.py)")
    # PyTorch ships its own HIP runtime (same soname as /opt/rocm's): load it
    # first so that libaxf binds to that one runtime instead of a second copy.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, dp = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "axf_last_error": ([], ctypes.c_char_p), "axf_version": ([], ctypes.c_char_p),
        "axf_footprint": ([P(Config), P(sz)], ctypes.c_int),
        "axf_extents": ([P(Config), P(i32)], ctypes.c_int),
        "axf_create": ([P(Config), vp, sz, vp, P(vp)], ctypes.c_int),
        "axf_write_field": ([vp, i32, vp, sz, i32], ctypes.c_int),
        "axf_step": ([vp, i64], ctypes.c_int),
        "axf_read_field": ([vp, i32, vp, sz, i32], ctypes.c_int),
        "axf_read_particles": ([vp, i32, P(dp), i64, P(i64)], ctypes.c_int),
        "axf_diag_now": ([vp, P(DiagRecord)], ctypes.c_int),
        "axf_diag_now_static": ([vp, i32, P(DiagRecord)], ctypes.c_int),
        "axf_read_diag": ([vp, P(DiagRecord), i32, P(i32)], ctypes.c_int),
        "axf_state_bytes": ([vp, P(sz)], ctypes.c_int),
        "axf_read_state": ([vp, vp, sz], ctypes.c_int),
        "axf_write_state": ([vp, vp, sz], ctypes.c_int),
        "axf_sync": ([vp], ctypes.c_int),
        "axf_steps_done": ([vp, P(i64)], ctypes.c_int),
        "axf_path_in_use": ([vp, P(i32)], ctypes.c_int),
        "axf_destroy": ([vp], ctypes.c_int),
        "axf_last_step_timing": ([vp, P(dp), P(i64)], ctypes.c_int),
        "axf_tune": ([P(Config), vp, sz, vp, i32, P(Tuning)], ctypes.c_int),
        "axf_tune_reset": ([], ctypes.c_int),
        "axf_batch_footprint": ([P(Config), i32, P(sz)], ctypes.c_int),
        "axf_batch_create": ([P(Config), i32, vp, sz, vp, P(vp)], ctypes.c_int),
        "axf_batch_step": ([vp, P(i64)], ctypes.c_int),
        "axf_batch_run": ([vp, i32, P(vp)], ctypes.c_int),
        "axf_batch_destroy": ([vp], ctypes.c_int),
        "axf_server_create": ([vp, sz, i32, i32, vp, P(vp)], ctypes.c_int),
        "axf_server_submit": ([vp, P(Config), i64, P(ctypes.c_uint64)], ctypes.c_int),
        "axf_server_cancel": ([vp, ctypes.c_uint64], ctypes.c_int),
        "axf_server_poll": ([vp, P(Result), i32, P(i32)], ctypes.c_int),
        "axf_server_stats": ([vp, P(i32), P(i32), P(sz)], ctypes.c_int),
        "axf_server_destroy": ([vp], ctypes.c_int),
        "axf_config_from_si": ([P(Si), P(Config)], ctypes.c_int),
        "axf_axion_coupling": ([dp, dp, P(dp)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(rc):
    if rc != 0:
        raise AxfError(rc, lib().axf_last_error().decode())
    return rc


def make_config(cfg, precision=F64, diag_every=0, path=PATH_AUTO):
    """axf_config from a run description dict (keys as in the C struct)."""
    c = Config()
    n = [int(v) for v in cfg["n"]]
    c.ndim = int(cfg.get("ndim", 3 if n[2] > 1 else (2 if n[1] > 1 else 1)))
    c.n[:] = n
    c.dx[:] = [float(v) for v in cfg["dx"]]
    c.dt = float(cfg["dt"])
    c.precision = int(cfg.get("precision", precision))
    c.em_bc[:] = [int(v) for v in cfg.get("em_bc", [0, 0, 0])]
    c.ax_bc[:] = [int(v) for v in cfg.get("ax_bc", [0, 0, 0])]
    c.pml_n = int(cfg.get("pml_n", 20))
    c.pml_sigma_dt = float(cfg.get("pml_sigma_dt", 0.2))
    c.m = float(cfg.get("m", 0.0))
    c.g = float(cfg.get("g", 0.0))
    c.bext[:] = [float(v) for v in cfg.get("bext", [0.0, 0.0, 0.0])]
    c.slab_lo = int(cfg.get("slab_lo", 0))
    c.slab_hi = int(cfg.get("slab_hi", n[0]))
    for key in ("laser_on", "laser_pol", "laser_env", "packet_on", "pk_dir"):
        setattr(c, key, int(cfg.get(key, 1 if key == "pk_dir" else 0)))
    for key in ("omega", "e_amp", "ramp_periods", "fwhm", "t_center", "waist", "x_focus", "y_c",
                "z_c", "cep", "pk_amp", "pk_k", "pk_w", "pk_x0", "pk_y0", "pk_z0"):
        setattr(c, key, float(cfg.get(key, 0.0)))
    c.diag_every = int(cfg.get("diag_every", diag_every))
    c.path = int(cfg.get("path", path))
    c.win_t0 = float(cfg.get("win_t0", 0.0))
    c.win_cells = int(cfg.get("win_cells", 0))
    c.laser_order = int(cfg.get("laser_order", 0))
    c.ppc[:] = [int(v) for v in cfg.get("ppc", [0, 1])]
    c.plasma_n = float(cfg.get("plasma_n", 0.0))
    c.plasma_lo = int(cfg.get("plasma_lo", 0))
    c.plasma_hi = int(cfg.get("plasma_hi", n[0]))
    c.plasma_u[:] = [float(v) for v in cfg.get("plasma_u", [0.0, 0.0, 0.0])]
    return c


def config_from_si(si, cfg):
    """`cfg` (a run description dict with at least "n") with dx, dt, m, g,
    bext, omega, e_amp, fwhm, t_center, waist, x_focus, y_c and z_c converted
    from the SI inputs `si` (a dict with the keys of axf_si; missing keys 0)
    by axf_config_from_si."""
    s = Si()
    for key, _ in Si._fields_:
        v = si.get(key, 0.0)
        if key in ("dx", "bext"):
            getattr(s, key)[:] = [float(x) for x in (list(v) + [0.0, 0.0, 0.0])[:3]] if v else [0.0] * 3
        else:
            setattr(s, key, float(v))
    c = make_config(dict(cfg, dx=cfg.get("dx", [1.0, 1.0, 1.0]), dt=cfg.get("dt", 1.0)))
    check(lib().axf_config_from_si(ctypes.byref(s), ctypes.byref(c)))
    out = dict(cfg)
    out["ndim"] = c.ndim
    out["dx"], out["bext"] = list(c.dx), list(c.bext)
    for key in ("dt", "m", "g", "omega", "e_amp", "fwhm", "t_center", "waist", "x_focus", "y_c", "z_c"):
        out[key] = getattr(c, key)
    return out


def axion_coupling(m_a_eV, c_gamma):
    """g_agg [hbar GeV^-1] of an axion model of mass m_a_eV and photon
    coupling c_gamma (axf_axion_coupling)."""
    g = ctypes.c_double()
    check(lib().axf_axion_coupling(float(m_a_eV), float(c_gamma), ctypes.byref(g)))
    return g.value


def footprint(cfg, **kw):
    c = make_config(cfg, **kw)
    b = ctypes.c_size_t()
    check(lib().axf_footprint(ctypes.byref(c), ctypes.byref(b)))
    return b.value


def extents(cfg, **kw):
    c = make_config(cfg, **kw)
    nn = (ctypes.c_int32 * 3)()
    check(lib().axf_extents(ctypes.byref(c), nn))
    return tuple(nn)


def _torch():
    import torch
    return torch


def device_buffer(nbytes, device="cuda:0"):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def current_stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def tune(cfg, precision=F32, steps=20, stream=None):
    """Time the fused 2D launch shapes on a scratch run of this configuration
    and record the best for runs of its size class; returns the choice."""
    c = make_config(cfg, precision=precision)
    nbytes = footprint(cfg, precision=precision)
    scratch = device_buffer(nbytes)
    out = Tuning()
    check(lib().axf_tune(ctypes.byref(c), ctypes.c_void_p(scratch.data_ptr()), scratch.numel(),
                         stream if stream is not None else current_stream(), int(steps), ctypes.byref(out)))
    del scratch
    return {k: getattr(out, k) for k, _ in out._fields_}


def tune_reset():
    check(lib().axf_tune_reset())


class Run:
    """One run on the GPU; the device buffer is a torch uint8 tensor it keeps alive."""

    def __init__(self, cfg, precision=F64, diag_every=0, path=PATH_AUTO, buffer=None, stream=None):
        self.cfg = make_config(cfg, precision=precision, diag_every=diag_every, path=path)
        self.nbytes = footprint(cfg, precision=precision, diag_every=diag_every, path=path)
        self.nn = extents(cfg, precision=precision, diag_every=diag_every, path=path)
        self.buffer = buffer if buffer is not None else device_buffer(self.nbytes)
        self.stream = stream if stream is not None else current_stream()
        h = ctypes.c_void_p()
        check(lib().axf_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.buffer.data_ptr()),
                               self.buffer.numel(), self.stream, ctypes.byref(h)))
        self._h = h
        self._owned = True

    @classmethod
    def _view(cls, handle, cfg_struct, nn):
        self = cls.__new__(cls)
        self._h = handle
        self.cfg = cfg_struct
        self.nn = nn
        self._owned = False
        return self

    def close(self):
        if getattr(self, "_h", None) and self._owned:
            lib().axf_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps=1):
        check(lib().axf_step(self._h, int(nsteps)))

    def sync(self):
        check(lib().axf_sync(self._h))

    @property
    def steps_done(self):
        v = ctypes.c_int64()
        check(lib().axf_steps_done(self._h, ctypes.byref(v)))
        return v.value

    def uses_fused(self):
        v = ctypes.c_int32()
        check(lib().axf_path_in_use(self._h, ctypes.byref(v)))
        return v.value == PATH_FUSED

    def read(self, name):
        """Field `name` at the current time as float64, shape (nn_z, nn_y, nn_x)."""
        out = np.empty(self.nn[2] * self.nn[1] * self.nn[0], dtype=np.float64)
        check(lib().axf_read_field(self._h, FIELD_ID[name], out.ctypes.data_as(ctypes.c_void_p),
                                   out.nbytes, 0))
        return out.reshape(self.nn[2], self.nn[1], self.nn[0])

    PARTICLE_ID = {"x": 0, "y": 1, "z": 2, "ux": 3, "uy": 4, "uz": 5, "x1": 6, "y1": 7, "z1": 8,
                   "u1x": 9, "u1y": 10, "u1z": 11, "w": 12}

    def read_particles(self, name):
        """Particle array `name` (x, y, z, ux, uy, uz, the first-order x1 ...
        u1z, w) at the current time as float64 (axf_read_particles)."""
        cnt = int(self.cfg.ppc[0]) * max(1, int(self.cfg.ppc[1]) if self.cfg.n[1] > 1 else 1) * \
            (int(self.cfg.plasma_hi) - int(self.cfg.plasma_lo)) * int(self.cfg.n[1])
        out = np.empty(max(cnt, 1), dtype=np.float64)
        n = ctypes.c_int64()
        check(lib().axf_read_particles(self._h, self.PARTICLE_ID[name],
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size,
                                       ctypes.byref(n)))
        return out[:n.value]

    def write(self, name, arr):
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(arr, dtype=np.float64),
                                                 (self.nn[2], self.nn[1], self.nn[0])))
        check(lib().axf_write_field(self._h, FIELD_ID[name], a.ctypes.data_as(ctypes.c_void_p), a.nbytes, 0))

    def diag_now(self):
        rec = DiagRecord()
        check(lib().axf_diag_now(self._h, ctypes.byref(rec)))
        return rec.as_dict()

    def diag_now_static(self, rows=0):
        rec = DiagRecord()
        check(lib().axf_diag_now_static(self._h, int(rows), ctypes.byref(rec)))
        return rec.as_dict()

    def read_diag(self, max_records=4096):
        buf = (DiagRecord * max_records)()
        n = ctypes.c_int32()
        check(lib().axf_read_diag(self._h, buf, max_records, ctypes.byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]

    def state(self):
        b = ctypes.c_size_t()
        check(lib().axf_state_bytes(self._h, ctypes.byref(b)))
        out = np.empty(b.value, dtype=np.uint8)
        check(lib().axf_read_state(self._h, out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def load_state(self, blob):
        blob = np.ascontiguousarray(blob, dtype=np.uint8)
        check(lib().axf_write_state(self._h, blob.ctypes.data_as(ctypes.c_void_p), blob.nbytes))

    def last_step_timing(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        check(lib().axf_last_step_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def _configs(cfgs, precision, diag_every, path):
    arr = (Config * len(cfgs))()
    for i, c in enumerate(cfgs):
        arr[i] = make_config(c, precision=precision, diag_every=diag_every, path=path)
    return arr


def batch_footprint(cfgs, precision=F32, diag_every=0, path=PATH_AUTO):
    arr = _configs(cfgs, precision, diag_every, path)
    b = ctypes.c_size_t()
    check(lib().axf_batch_footprint(arr, len(cfgs), ctypes.byref(b)))
    return b.value


class Batch:
    """Independent runs in one device buffer, advanced by batched launches.
    `runs[i]` are borrowed views with the Run read/diag/state methods."""

    def __init__(self, cfgs, precision=F32, diag_every=0, path=PATH_AUTO, stream=None):
        self.count = len(cfgs)
        self._cfgs = _configs(cfgs, precision, diag_every, path)
        self.nbytes = batch_footprint(cfgs, precision, diag_every, path)
        self.buffer = device_buffer(self.nbytes)
        self.stream = stream if stream is not None else current_stream()
        h = ctypes.c_void_p()
        check(lib().axf_batch_create(self._cfgs, self.count, ctypes.c_void_p(self.buffer.data_ptr()),
                                     self.buffer.numel(), self.stream, ctypes.byref(h)))
        self._h = h
        self.runs = []
        for i, c in enumerate(cfgs):
            v = ctypes.c_void_p()
            check(lib().axf_batch_run(self._h, i, ctypes.byref(v)))
            nn = extents(c, precision=precision, diag_every=diag_every, path=path)
            self.runs.append(Run._view(v, self._cfgs[i], nn))

    def step(self, nsteps):
        """Advance run i by nsteps[i] (an int applies to every run)."""
        if np.isscalar(nsteps):
            nsteps = [int(nsteps)] * self.count
        arr = (ctypes.c_int64 * self.count)(*[int(v) for v in nsteps])
        check(lib().axf_batch_step(self._h, arr))

    def sync(self):
        _torch().cuda.synchronize()

    def close(self):
        if getattr(self, "_h", None):
            lib().axf_batch_destroy(self._h)
        self._h = None
        self.runs = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over a device pool of `pool_bytes`."""

    def __init__(self, pool_bytes, max_slots=64, macro_steps=100, stream=None):
        self.pool = device_buffer(pool_bytes)
        self.stream = stream if stream is not None else current_stream()
        h = ctypes.c_void_p()
        check(lib().axf_server_create(ctypes.c_void_p(self.pool.data_ptr()), self.pool.numel(), int(max_slots),
                                      int(macro_steps), self.stream, ctypes.byref(h)))
        self._h = h

    def submit(self, cfg, nsteps, precision=F32, diag_every=0, path=PATH_AUTO):
        c = make_config(cfg, precision=precision, diag_every=diag_every, path=path)
        rid = ctypes.c_uint64()
        check(lib().axf_server_submit(self._h, ctypes.byref(c), int(nsteps), ctypes.byref(rid)))
        return rid.value

    def cancel(self, rid):
        check(lib().axf_server_cancel(self._h, ctypes.c_uint64(rid)))

    def poll(self, max_results=256):
        buf = (Result * max_results)()
        n = ctypes.c_int32()
        check(lib().axf_server_poll(self._h, buf, max_results, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            r = buf[i]
            out.append({"id": r.id, "status": r.status, "steps": r.steps, "cells": r.cells,
                        "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
                        "final": r.final.as_dict()})
        return out

    def stats(self):
        q, r, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        check(lib().axf_server_stats(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b)))
        return {"queued": q.value, "resident": r.value, "bytes_used": b.value}

    def close(self):
        if getattr(self, "_h", None):
            lib().axf_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
