"""Host model of the x split of the one-pass 3D march with an x-face launch.

The march's interior launch has no boundary code, so each of its wavefronts
must load 64 columns inside the grid's cells [0, n0); the x-face launch gives
each row one wavefront for both x faces: lanes 0-31 hold columns -2 .. 29
(28 own at x_min, lanes 2-29, two halo lanes above), lanes 32-63 hold columns
xc1 - 2 .. xc1 + 29 (two halo lanes below, then the last nb columns up to the
nodal top column n0).  The rule below is the one the library applies when it
lays out an FP32 run whose plane chunks' face records fit in LDS (FP64 runs
and longer chunks leave the face columns to the frame launch): the fewest interior segments of equal width w <= 60 between
the halves, nb in [1, 28] (so that an x_max own lane stays two lanes clear of
lane 63, as in a segment), and the last segment's loads below n0, tried
where the frame's split into segments has an interior one.  The model
checks, for every width from 40 to 4200 cells, that the own columns cover each
nodal column exactly once and that no lane of either launch reads outside the
grid; where the rule finds no split the faces go to the frame launch.
"""
import pytest


def split(n0):
    """(ns, w, nb, xc1) of the rule, or None when the faces go to the frame.
    The rule is tried only where the frame's own split (segments of at most
    60 columns) has an interior segment, i.e. segment 1's loads stay inside."""
    nn0 = n0 + 1
    nseg = (nn0 + 59) // 60
    wid = (nn0 + nseg - 1) // nseg
    if nseg < 2 or wid + 61 > n0 - 1:
        return None
    xa, rem = 28, nn0 - 28
    ns = 1
    while ns * 33 <= rem:
        for w in range(60, 32, -1):
            nb = rem - ns * w
            if nb < 1 or nb > 28 or xa + (ns - 1) * w + 61 > n0 - 1:
                continue
            return ns, w, nb, xa + ns * w
        ns += 1
    return None


def lanes_of_x_face(n0, xc1):
    """(lane, column, own) of one x-face wavefront."""
    out = []
    for lane in range(64):
        gx = lane - 2 if lane < 32 else xc1 - 34 + lane
        own = (2 <= lane < 30) if lane < 32 else (lane >= 34 and gx <= n0)
        out.append((lane, gx, own))
    return out


@pytest.mark.parametrize("lo,hi", [(40, 1100), (1100, 2200), (2200, 3200), (3200, 4200)])
def test_split_covers_each_column_once_and_stays_inside(lo, hi):
    """Every width from lo to hi cells: exact cover, loads inside; from 125
    cells on the rule finds a split for nearly every width."""
    found = 0
    for n0 in range(lo, hi):
        s = split(n0)
        if s is None:
            continue
        found += 1
        ns, w, nb, xc1 = s
        cover = [0] * (n0 + 1)
        for lane, gx, own in lanes_of_x_face(n0, xc1):
            if own:
                assert 0 <= gx <= n0 and lane <= 61, (n0, s, lane)
                cover[gx] += 1
        # the halo lanes of the x_max half read interior columns
        assert xc1 - 2 >= 0
        for k in range(ns):
            x0 = 28 + k * w
            assert x0 - 2 >= 0 and x0 + 61 <= n0 - 1, (n0, s, k)
            for lane in range(2, 2 + w):
                cover[x0 - 2 + lane] += 1
        assert all(c == 1 for c in cover), (n0, s)
    assert found > 0.95 * (hi - max(lo, 125))


def test_split_of_the_512_grid():
    """512^3: eight interior segments of 60 columns, 5 at x_max."""
    assert split(512) == (8, 60, 5, 508)


def test_narrow_grids_take_the_frame():
    """Below about 100 cells there is no room for a segment between the halves."""
    assert split(90) is None and split(96) is None
    assert split(128) == (2, 38, 25, 104)
