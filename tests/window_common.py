"""Run descriptions and the move schedule shared by the moving-window tests."""
import math

from paper_2406_16796_amd import workloads as W

FIELDS = ["E0X", "E0Y", "E0Z", "B0X", "B0Y", "B0Z", "E1X", "E1Y", "E1Z", "B1X", "B1Y", "B1Z",
          "PHI_OLD", "PHI_NEW"]


def window_target(cfg, n):
    """Columns the window has moved by the start of step n (the library's rule)."""
    cells = cfg.get("win_cells", 0)
    if cells <= 0 or n < 1:
        return 0
    t = n * cfg["dt"]
    if t < cfg["win_t0"]:
        return 0
    return cells * int(math.floor((t - cfg["win_t0"]) / (cells * cfg["dx"][0])))


def pulse_2d(nx, ny=64, cells=8):
    """2D: a short Gaussian pulse (waist and FWHM 1.5 wavelengths, a0 = 0.5)
    entering through x_min into a uniform B_ext along y from column 40 on,
    m = 0.3, g = 0.03, outflow axion; the window moves from the time the
    pulse is in (3.5 envelope widths past its peak at x = 0)."""
    c = W.gaussian_2d(n=nx, steps=0, m=0.3, g=0.03, a0=0.5, waist_lam=1.5, fwhm_lam=1.5, slab=(40, 10 ** 6),
                      ax_bc=W.AX_OUTFLOW)
    dx = c["dx"][0]
    c.update(n=[nx, ny, 1], y_c=0.5 * ny * dx, x_focus=30 * dx, slab_hi=10 ** 6, pml_n=8)
    tau0 = c["fwhm"] / math.sqrt(2.0 * math.log(2.0))
    c.update(win_cells=cells, win_t0=c["t_center"] + 3.5 * tau0)
    return c


def oracle_windowed(Oracle, cfg, steps, library=None):
    """The oracle run with the window moved on the library's schedule."""
    o = Oracle(cfg, library=library)
    moved = 0
    for n in range(steps):
        want = window_target(cfg, n)
        while moved < want:
            o.shift_window(cfg["win_cells"])
            moved += cfg["win_cells"]
        o.step(1)
    return o, moved
