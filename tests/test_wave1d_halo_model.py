"""Host model of the fused 1D pass's tiling: how far its halos must reach.

A numpy model of one pass advances windows of a 1D grid K steps with the
kernel's update order (phase A: E0, the axion current, E1, Mur ghosts; phase
B: B, phi) and neighbours clamped at the window's ends, then keeps each
tile's own cells.  Whole-grid steps with the same formulas are the
reference.  With random fields everywhere (every coupling active), halos of
K + 1 cells reproduce the whole-grid steps exactly, and halos of K cells on
either side do not: B at i reads E1 at i - 1 of the same step, which reads
the axion current there, which reads phi at i - 2; phi at i reads B0^{n+1}
at i + 1, which reads E0 at i + 1, which reads B0^n at i + 2.  This is the
reach the HIP kernel's windows are sized for.
"""
import numpy as np
import pytest

DT, DX, M2, GAX, CG1, BEXT = 0.2985, 0.314, 0.09, 0.02, 0.02, 1.0
CDT = DT / DX
MURC = (DT - DX) / (DT + DX)
EM = ("e0y", "e0z", "e1y", "e1z")
BM = ("b0y", "b0z", "b1y", "b1z")


def random_state(n, seed):
    rng = np.random.default_rng(seed)
    st = {k: rng.normal(size=n) for k in EM}
    st.update({k: rng.normal(size=n + 1) for k in BM})      # nodes 0 .. n (Mur x faces)
    st["pa"], st["pb"] = rng.normal(size=n), rng.normal(size=n)
    st["mg"] = rng.normal(size=(2, 2, 2))                   # Mur ghosts [side][order][y, z]
    return st


def cell_a(e, b, rb, pa, pb, pal, pbl, par, pbr):
    """Phase A at one cell: E0^{n+1/2}, the current, E1^{n+1/2}."""
    ey0, ez0, ey1, ez1 = e
    by0, bz0, by1, bz1 = b
    ny0 = ey0 + (0.0 - CDT * (rb[1] - bz0))
    nz0 = ez0 + (CDT * (rb[0] - by0) - 0.0)
    e1, e2 = 0.5 * (ey0 + ny0), 0.5 * (ez0 + nz0)
    b1, b2 = 0.5 * (by0 + rb[0]) + BEXT, 0.5 * (bz0 + rb[1])
    dtp = (pb - pa) / DT
    gp = (0.5 * (par + pbr) - 0.5 * (pal + pbl)) / (2 * DX)
    c1 = dtp * b1 - e2 * gp
    c2 = dtp * b2 + e1 * gp
    ny1 = ey1 + ((0.0 - CDT * (rb[3] - bz1)) - CG1 * c1)
    nz1 = ez1 + ((CDT * (rb[2] - by1) - 0.0) - CG1 * c2)
    return (ny0, nz0, ny1, nz1)


def mur(mg, side, old, new):
    for o in range(2):
        for c in range(2):
            mg[side, o, c] = old[2 * o + c] + MURC * (new[2 * o + c] - mg[side, o, c])


def b_new(b, e, el):
    """B^{n+1} at a node from E^{n+1/2} at the node's right and left centres."""
    return (b[0] - (0.0 - CDT * (e[1] - el[1])), b[1] - (CDT * (e[0] - el[0]) - 0.0),
            b[2] - (0.0 - CDT * (e[3] - el[3])), b[3] - (CDT * (e[2] - el[2]) - 0.0))


def phi_new(e, b, nb, rbo, rbn, pa, pb, pl, pr):
    bb1 = 0.5 * (0.5 * (b[0] + rbo[0]) + 0.5 * (nb[0] + rbn[0])) + BEXT
    bb2 = 0.5 * (0.5 * (b[1] + rbo[1]) + 0.5 * (nb[1] + rbn[1]))
    sax = GAX * (e[0] * bb1 + e[1] * bb2)
    lap = ((pr - 2 * pb) + pl) / DX ** 2
    return (DT * DT * ((sax - M2 * pb) + lap) + 2 * pb) - pa


def whole_grid_step(st):
    """One step on the whole grid (periodic axion, Mur EM faces)."""
    n = len(st["pa"])
    E = [st[k] for k in EM]
    B = [st[k] for k in BM]
    mg = st["mg"].copy()
    pa, pb = st["pa"], st["pb"]
    ne = [np.empty(n) for _ in range(4)]
    for i in range(n):
        v = cell_a([E[q][i] for q in range(4)], [B[q][i] for q in range(4)], [B[q][i + 1] for q in range(4)],
                   pa[i], pb[i], pa[i - 1], pb[i - 1], pa[(i + 1) % n], pb[(i + 1) % n])
        for q in range(4):
            ne[q][i] = v[q]
    for side, i in ((0, 0), (1, n - 1)):
        mur(mg, side, [E[q][i] for q in range(4)], [ne[q][i] for q in range(4)])
    ghost = [[mg[s, q // 2, q % 2] for q in range(4)] for s in range(2)]
    nbv = [np.empty(n + 1) for _ in range(4)]
    for i in range(n + 1):
        er = [ne[q][i] for q in range(4)] if i < n else ghost[1]
        el = [ne[q][i - 1] for q in range(4)] if i > 0 else ghost[0]
        v = b_new([B[q][i] for q in range(4)], er, el)
        for q in range(4):
            nbv[q][i] = v[q]
    pn = np.empty(n)
    for i in range(n):
        pn[i] = phi_new([ne[0][i], ne[1][i]], [B[0][i], B[1][i]], [nbv[0][i], nbv[1][i]], [B[0][i + 1], B[1][i + 1]],
                        [nbv[0][i + 1], nbv[1][i + 1]], pa[i], pb[i], pb[i - 1], pb[(i + 1) % n])
    out = {k: ne[q] for q, k in enumerate(EM)}
    out.update({k: nbv[q] for q, k in enumerate(BM)})
    out.update(pa=pb, pb=pn, mg=mg)
    return out


def tiled_pass(st, K, own, hl, hr):
    """K steps on windows of own cells plus halos hl, hr (wrapping around the
    periodic axion), clamped neighbours at the window's ends, as the kernel
    does them; each tile keeps its own cells."""
    n = len(st["pa"])
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    for x0 in range(0, n, own):
        ow = min(own, n - x0)
        wn = ow + hl + hr
        g = (x0 - hl + np.arange(wn)) % n
        E = [st[k][g].copy() for k in EM]
        B = [st[k][g].copy() for k in BM]
        bn = [st[k][n] for k in BM]
        mg = st["mg"].copy()
        ph = [st["pa"][g].copy(), st["pb"][g].copy(), np.zeros(wn)]

        def nb(j, d):
            return min(max(j + d, 0), wn - 1)

        for k in range(K):
            qa, qb, qn = k % 3, (k + 1) % 3, (k + 2) % 3
            oldE = [e.copy() for e in E]
            for j in range(wn):
                rb = bn if g[j] == n - 1 else [B[q][nb(j, 1)] for q in range(4)]
                v = cell_a([E[q][j] for q in range(4)], [B[q][j] for q in range(4)], rb, ph[qa][j], ph[qb][j],
                           ph[qa][nb(j, -1)], ph[qb][nb(j, -1)], ph[qa][nb(j, 1)], ph[qb][nb(j, 1)])
                for q in range(4):
                    E[q][j] = v[q]
                for side, c in ((0, 0), (1, n - 1)):
                    if g[j] == c:
                        mur(mg, side, [oldE[q][j] for q in range(4)], v)
            ghost = [[mg[s, q // 2, q % 2] for q in range(4)] for s in range(2)]
            nB = [b.copy() for b in B]
            for j in range(wn):
                el = ghost[0] if g[j] == 0 else [E[q][nb(j, -1)] for q in range(4)]
                v = b_new([B[q][j] for q in range(4)], [E[q][j] for q in range(4)], el)
                for q in range(4):
                    nB[q][j] = v[q]
                if g[j] == n - 1:
                    nbn = b_new(bn, ghost[1], [E[q][j] for q in range(4)])
                    rbo, rbn = bn, nbn
                else:
                    jr = nb(j, 1)
                    rbo = [B[q][jr] for q in range(4)]
                    rbn = b_new(rbo, [E[q][jr] for q in range(4)], [E[q][j] for q in range(4)])
                ph[qn][j] = phi_new([E[0][j], E[1][j]], [B[0][j], B[1][j]], [v[0], v[1]], rbo, rbn, ph[qa][j],
                                    ph[qb][j], ph[qb][nb(j, -1)], ph[qb][nb(j, 1)])
                if g[j] == n - 1:
                    bn_next = nbn
            B = nB
            if (n - 1) in g:
                bn = bn_next
        sl = slice(hl, hl + ow)
        for q, key in enumerate(EM):
            out[key][g[sl]] = E[q][sl]
        for q, key in enumerate(BM):
            out[key][g[sl]] = B[q][sl]
        out["pa"][g[sl]] = ph[K % 3][sl]
        out["pb"][g[sl]] = ph[(K + 1) % 3][sl]
        if 0 in g[sl]:
            out["mg"][0] = mg[0]
        if (n - 1) in g[sl]:
            out["mg"][1] = mg[1]
            for q, key in enumerate(BM):
                out[key][n] = bn[q]
    return out


def mismatch(K, hl, hr, n=84, own=28, seed=3):
    st = random_state(n, seed)
    ref = st
    for _ in range(K):
        ref = whole_grid_step(ref)
    got = tiled_pass(st, K, own, hl, hr)
    return max(float(np.abs(ref[k] - got[k]).max()) for k in EM + BM + ("pa", "pb"))


@pytest.mark.parametrize("K", [2, 5, 9])
def test_halos_of_k_plus_one_are_exact(K):
    assert mismatch(K, K + 1, K + 1) == 0.0


@pytest.mark.parametrize("K", [2, 5, 9])
def test_halos_of_k_are_not_enough_on_either_side(K):
    assert mismatch(K, K, K + 1) > 1e-9
    assert mismatch(K, K + 1, K) > 1e-9
