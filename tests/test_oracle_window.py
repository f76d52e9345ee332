"""Pin of the oracle's moving window (Sec. III.B): the window follows the
pulse at c, so nothing inside it depends on what lies behind its trailing
edge.  A windowed run therefore equals a static run on a box long enough to
hold the whole path, on the window's columns, except within a few cells of
the trailing edge (where the static run's wake, and the window's Mur face
and outflow ghosts, differ) - to rounding, since a move only relabels the
columns."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from window_common import FIELDS, oracle_windowed, pulse_2d


def test_windowed_equals_static_run_behind_the_pulse():
    steps = 600
    cw = pulse_2d(240)
    cs = dict(pulse_2d(600), win_cells=0)
    ow, moved = oracle_windowed(Oracle, cw, steps)
    os_ = Oracle(cs)
    os_.step(steps)
    assert moved >= 200
    for lo, hi in ((0, 6), (6, 12), (12, 14)):
        scale = max(np.abs(os_.field(n)).max() for n in FIELDS[lo:hi])
        for name in FIELDS[lo:hi]:
            a = ow.field(name)
            b = os_.field(name)[:, :, moved:moved + a.shape[2]]
            err = np.abs(a - b)[:, :, 40:].max() / scale
            print(name, "%.1e" % err)
            assert err <= 1e-12, (name, err)


def test_window_moves_are_checked():
    o = Oracle(pulse_2d(120))
    with pytest.raises(ValueError):
        o.shift_window(8)            # no step taken yet
    o.step(1)
    for bad in (0, 65, 120):
        with pytest.raises(ValueError):
            o.shift_window(bad)
    o.shift_window(8)
