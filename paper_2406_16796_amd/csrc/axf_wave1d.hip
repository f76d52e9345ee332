// axf_wave1d.hip -- the fused 1D step: several steps per launch (temporal
// blocking).
//
// A workgroup holds a window of cells in LDS, the cells it owns plus a halo
// on either side, and advances it K steps with two barriers per step:
//   phase A: E0^{n+1/2}, the axion current at the centre, E1^{n+1/2} and the
//            Mur ghosts (every read but B^n at i + 1 is the cell's own);
//   phase B: B^{n+1} and phi^{n+3/2} with its ghosts.
// Then it writes back only the cells it owns.  A step reads one cell either
// way, with two longer reaches within the step: B at i reads E1^{n+1/2} at
// i - 1, which reads the axion current at i - 1, which reads phi at i - 2;
// phi at i reads B0^{n+1} at i + 1, which reads E0^{n+1/2} at i + 1, which
// reads B0^n at i + 2.  A chain of dependencies takes at most one of them: the
// first ends in phi, whose own inputs (phi, E0, B0) never read the current,
// and the second in B0, which never reads phi.  So after K steps every value
// at least K + 1 cells inside either end of the window is exact, whatever the
// window's ends held: halos of K + 1 cells.  A grid that fits one window is
// held whole, without halos, its periodic axes wrapping inside the window.
//
// Every value is formed by the unfused kernels' expressions, operand for
// operand, so a pass leaves the same bits as K unfused steps.
//
// The halo of one tile is another tile's own cells: a pass reads the slots of
// step s0 and writes those of step s0 + K, and the two must be distinct
// (wave1d_k_ok).
#include "axf_fused.h"
#include "axf_stencil.h"

#include <stdlib.h>

#include <algorithm>

namespace axf {

namespace {

// the most steps per pass; threads per workgroup
constexpr int kW1Kmax = 16, kW1Threads = 256;

// LDS of a window of W cells
template <typename T, int W>
struct W1Lds {
    T e0y[W], e0z[W], e1y[W], e1z[W];   // E^{n-1/2}, E^{n+1/2} after phase A
    T b[2][4][W];                        // B0y B0z B1y B1z: B^n in [n & 1]
    T ph[3][W];                          // axion level L in [L % 3]
    T bn[2][4];                          // the same at node n (Mur x_max face)
    T mg[2][2][2];                       // Mur ghosts [side][order][component - 1]
    T ag[2][3];                          // axion ghosts [side][level % 3]
    double inc[2][kW1Kmax + 1];          // laser at the first centre [0] and at the ghost [1], levels s0 ..
};

// the window of tile t: cells gs .. gs + wn - 1 (mod n when it wraps), own
// slots [own0, own1); ring: the window is the whole grid, slot neighbours wrap
struct W1Tile {
    int gs, wn, own0, own1;
    bool wrap, ring;
};

// own cells of a tile (halos of kmax + 1 cells on either side)
__host__ __device__ inline int w1_own(int W, int kmax) { return W - 2 * (kmax + 1); }

__host__ __device__ inline int w1_ntiles(int n, int W, int kmax)
{
    return n <= W ? 1 : (n + w1_own(W, kmax) - 1) / w1_own(W, kmax);
}

__device__ inline W1Tile w1_tile(int n, bool axp, int W, int kmax, int t)
{
    W1Tile g;
    if (n <= W) {
        g.gs = 0;
        g.wn = n;
        g.own0 = 0;
        g.own1 = n;
        g.wrap = false;
        g.ring = true;
        return g;
    }
    const int S = w1_own(W, kmax), x0 = t * S, own = min(S, n - x0), h = kmax + 1;
    g.ring = false;
    if (axp) {
        // a periodic axion couples the two ends: the window runs on around the grid
        g.wrap = true;
        g.gs = x0 - h;
        g.wn = own + 2 * h;
    } else {
        g.wrap = false;
        g.gs = max(0, x0 - h);
        g.wn = min(n, x0 + own + h) - g.gs;
    }
    g.own0 = x0 - g.gs;
    g.own1 = g.own0 + own;
    return g;
}

// (inlined into its kernels, so that `sm` is known to be LDS)
template <typename T, int W>
__device__ __forceinline__ void w1_pass(const RunK<T>& r, int t, long s0, int K, W1Lds<T, W>& sm)
{
    constexpr int KM = kW1Kmax;
    const int n = r.n[0];
    const bool mur = r.mur[0] != 0, axp = r.axbc[0] == AXF_AX_PERIODIC, outflow = r.axbc[0] == AXF_AX_OUTFLOW;
    const W1Tile tg = w1_tile(n, axp, W, KM, t);
    const int tid = threadIdx.x;
    // (gs > -n and gs + w < 2n: one correction wraps a cell index)
    auto gcell = [&](int w) {
        const int g = tg.gs + w;
        return !tg.wrap ? g : (g < 0 ? g + n : (g >= n ? g - n : g));
    };
    auto nbr = [&](int w, int d) {
        const int v = w + d;
        return tg.ring ? (v < 0 ? v + tg.wn : (v >= tg.wn ? v - tg.wn : v)) : min(max(v, 0), tg.wn - 1);
    };
    // the descriptor's coefficients in registers (the loop's stores to device
    // memory would otherwise have them read again every iteration)
    const T half = r.half, cdt = r.cdt[0], inv_dt = r.inv_dt, inv2dx = r.inv2dx[0], inv_dx2 = r.inv_dx2[0];
    const T cg1 = r.cg1, gax = r.gax, m2 = r.m2, dt2 = r.dt2, out_r = r.out_r[0], sdt_max = r.pml_sdt_max;
    const T bx[3] = {r.bext[0], r.bext[1], r.bext[2]};
    const int slab_lo = r.slab_lo, slab_hi = r.slab_hi, pml_n = r.pml_n, las_on = r.las.on, las_pol = r.las.pol;
    const bool pml = r.axbc[0] == AXF_AX_PML;
    const double murc = r.murc[0];
    // bext_at and pml_sdt with those registers (the same operations)
    auto bext = [&](int c, int g) { return (g >= slab_lo && g < slab_hi) ? bx[c] : T(0); };
    auto sdt_at = [&](int g) {
        T sv = T(0);
        if (pml) {
            const int dist = g < n - 1 - g ? g : n - 1 - g;
            if (dist < pml_n) {
                const T q = T(1) - T(dist) / T(pml_n);
                const T sd = sdt_max * q * q * q;
                sv = sd > sv ? sd : sv;
            }
        }
        return sv;
    };

    // the state of step s0
    {
        const int so = em_slot(s0, r.nem), la = phi_slot(s0, r.nph), lb = phi_slot(s0 + 1, r.nph);
        for (int w = tid; w < tg.wn; w += kW1Threads) {
            const int g = gcell(w);
            sm.e0y[w] = r.E0[so][1][g];
            sm.e0z[w] = r.E0[so][2][g];
            sm.e1y[w] = r.E1[so][1][g];
            sm.e1z[w] = r.E1[so][2][g];
            sm.b[0][0][w] = r.B0[so][1][g];
            sm.b[0][1][w] = r.B0[so][2][g];
            sm.b[0][2][w] = r.B1[so][1][g];
            sm.b[0][3][w] = r.B1[so][2][g];
            sm.ph[0][w] = r.phi[la][g];
            sm.ph[1][w] = r.phi[lb][g];
            for (int side = 0; side < 2; side++) {
                if (g != (side ? n - 1 : 0)) continue;
                if (mur)
                    for (int o = 0; o < 2; o++)
                        for (int c = 1; c < 3; c++) sm.mg[side][o][c - 1] = r.murg[o][0][side][c][so][0];
                if (!axp) {
                    sm.ag[side][0] = r.axg[0][side][la][0];
                    sm.ag[side][1] = r.axg[0][side][lb][0];
                }
                if (side == 1 && mur) {
                    sm.bn[0][0] = r.B0[so][1][n];
                    sm.bn[0][1] = r.B0[so][2][n];
                    sm.bn[0][2] = r.B1[so][1][n];
                    sm.bn[0][3] = r.B1[so][2][n];
                }
            }
        }
        // the laser on the x_min face at levels s0 .. s0 + K, as the unfused
        // path tabulates it
        const int w0 = tg.wrap && tg.gs > 0 ? n - tg.gs : -tg.gs;
        if (mur && las_on && w0 >= 0 && w0 < tg.wn && tid <= K) {
            const int c = las_pol, j = 0, k = 0;
            const double y = (c == 1) ? j * r.dx[1] : (j + 0.5) * r.dx[1];
            const double z = (c == 2) ? k * r.dx[2] : (k + 0.5) * r.dx[2];
            const long L = s0 + tid;
            const double tt = (L - 0.5) * r.dt;
            sm.inc[0][tid] = incident(r.las, c, 0.5 * r.dx[0], y, z, tt);
            sm.inc[1][tid] = incident(r.las, c, -0.5 * r.dx[0], y, z, tt);
        }
    }
    __syncthreads();

    const int so2 = em_slot(s0 + K, r.nem), lo2 = phi_slot(s0 + K, r.nph), ln2 = phi_slot(s0 + K + 1, r.nph);
    // where the pass leaves the state of step s0 + K
    T *const oE[4] = {r.E0[so2][1], r.E0[so2][2], r.E1[so2][1], r.E1[so2][2]};
    T *const oB[4] = {r.B0[so2][1], r.B0[so2][2], r.B1[so2][1], r.B1[so2][2]};
    T *const oP0 = r.phi[lo2], *const oP1 = r.phi[ln2];
    T *oM[2][2][2], *oA[2][2];
    for (int side = 0; side < 2; side++) {
        for (int o = 0; o < 2; o++)
            for (int c = 1; c < 3; c++) oM[side][o][c - 1] = mur ? r.murg[o][0][side][c][so2] : nullptr;
        oA[side][0] = axp ? nullptr : r.axg[0][side][lo2];
        oA[side][1] = axp ? nullptr : r.axg[0][side][ln2];
    }
    for (int k = 0; k < K; k++) {
        const int pb = k & 1, qa = k % 3, qb = (k + 1) % 3, qn = (k + 2) % 3;
        const bool last = k == K - 1;
        // ---- phase A: E0, the axion current, E1, Mur ghosts
        for (int w = tid; w < tg.wn; w += kW1Threads) {
            const int g = gcell(w), wl = nbr(w, -1), wr = nbr(w, 1);
            const T by0 = sm.b[pb][0][w], bz0 = sm.b[pb][1][w], by1 = sm.b[pb][2][w], bz1 = sm.b[pb][3][w];
            T rb[4];
            if (mur && g == n - 1)
                for (int q = 0; q < 4; q++) rb[q] = sm.bn[pb][q];
            else
                for (int q = 0; q < 4; q++) rb[q] = sm.b[pb][q][wr];
            const T ey0 = sm.e0y[w], ez0 = sm.e0z[w], ey1 = sm.e1y[w], ez1 = sm.e1z[w];
            // E0^{n+1/2}: curl B0 by forward differences (y: -dBz/dx, z: dBy/dx)
            const T ny0 = ey0 + T(1) * (T(0) - cdt * (rb[1] - bz0));
            const T nz0 = ez0 + T(1) * (cdt * (rb[0] - by0) - T(0));
            // the axion current at the centre: (D_t phi) B0 - E0 x (D phi), E0 the
            // mean of its two levels, B0 the mean of the two nodes, phi^n the mean
            // of the two axion levels
            const T e0 = T(0), e1 = half * (ey0 + ny0), e2 = half * (ez0 + nz0);
            const T b1 = half * (by0 + rb[0]) + bext(1, g), b2 = half * (bz0 + rb[1]) + bext(2, g);
            const T pa = sm.ph[qa][w], pbv = sm.ph[qb][w];
            T pal, pbl, par, pbr;
            if (!axp && g == 0) {
                pal = sm.ag[0][qa];
                pbl = sm.ag[0][qb];
            } else {
                pal = sm.ph[qa][wl];
                pbl = sm.ph[qb][wl];
            }
            if (!axp && g == n - 1) {
                par = sm.ag[1][qa];
                pbr = sm.ag[1][qb];
            } else {
                par = sm.ph[qa][wr];
                pbr = sm.ph[qb][wr];
            }
            const T dtphi = (pbv - pa) * inv_dt;
            const T up = half * (par + pbr), dn = half * (pal + pbl);
            const T gp0 = (up - dn) * inv2dx, gp1 = T(0), gp2 = T(0);
            const T c1 = dtphi * b1 - (e2 * gp0 - e0 * gp2);
            const T c2 = dtphi * b2 - (e0 * gp1 - e1 * gp0);
            // E1^{n+1/2} with the current on the face (the centre itself in 1D)
            const T ny1 = ey1 + T(1) * ((T(0) - cdt * (rb[3] - bz1)) - cg1 * c1);
            const T nz1 = ez1 + T(1) * ((cdt * (rb[2] - by1) - T(0)) - cg1 * c2);
            sm.e0y[w] = ny0;
            sm.e0z[w] = nz0;
            sm.e1y[w] = ny1;
            sm.e1z[w] = nz1;
            if (mur) {
                const T eo[2][2] = {{ey0, ez0}, {ey1, ez1}}, en[2][2] = {{ny0, nz0}, {ny1, nz1}};
                for (int side = 0; side < 2; side++) {
                    if (g != (side ? n - 1 : 0)) continue;
                    for (int o = 0; o < 2; o++)
                        for (int c = 1; c < 3; c++) {
                            double ia_o = 0.0, ia_n = 0.0, ig_o = 0.0, ig_n = 0.0;
                            if (o == 0 && side == 0 && las_on && c == las_pol) {
                                ia_o = sm.inc[0][k];
                                ig_o = sm.inc[1][k];
                                ia_n = sm.inc[0][k + 1];
                                ig_n = sm.inc[1][k + 1];
                            }
                            T& gh = sm.mg[side][o][c - 1];
                            gh = (T)mur_core(murc, (double)eo[o][c - 1], (double)en[o][c - 1], (double)gh, ia_o, ia_n,
                                             ig_o, ig_n);
                            if (last && w >= tg.own0 && w < tg.own1) oM[side][o][c - 1][0] = gh;
                        }
                }
            }
            if (last && w >= tg.own0 && w < tg.own1) {
                oE[0][g] = ny0;
                oE[1][g] = nz0;
                oE[2][g] = ny1;
                oE[3][g] = nz1;
            }
        }
        __syncthreads();
        // ---- phase B: B, the axion and its ghosts
        for (int w = tid; w < tg.wn; w += kW1Threads) {
            const int g = gcell(w), wl = nbr(w, -1), wr = nbr(w, 1);
            const T ey0 = sm.e0y[w], ez0 = sm.e0z[w], ey1 = sm.e1y[w], ez1 = sm.e1z[w];
            T ly0, lz0, ly1, lz1;     // E^{n+1/2} at i - 1 (the Mur ghost left of cell 0)
            if (mur && g == 0) {
                ly0 = sm.mg[0][0][0];
                lz0 = sm.mg[0][0][1];
                ly1 = sm.mg[0][1][0];
                lz1 = sm.mg[0][1][1];
            } else {
                ly0 = sm.e0y[wl];
                lz0 = sm.e0z[wl];
                ly1 = sm.e1y[wl];
                lz1 = sm.e1z[wl];
            }
            const T by0 = sm.b[pb][0][w], bz0 = sm.b[pb][1][w], by1 = sm.b[pb][2][w], bz1 = sm.b[pb][3][w];
            // B^{n+1}: curl E by backward differences
            const T nby0 = by0 - (T(0) - cdt * (ez0 - lz0));
            const T nbz0 = bz0 - (cdt * (ey0 - ly0) - T(0));
            const T nby1 = by1 - (T(0) - cdt * (ez1 - lz1));
            const T nbz1 = bz1 - (cdt * (ey1 - ly1) - T(0));
            sm.b[pb ^ 1][0][w] = nby0;
            sm.b[pb ^ 1][1][w] = nbz0;
            sm.b[pb ^ 1][2][w] = nby1;
            sm.b[pb ^ 1][3][w] = nbz1;
            // B0 at node i + 1, B^n and B^{n+1} (the latter formed as its own
            // update forms it; at node n from the Mur ghost right of cell n - 1)
            T ry0o, rz0o, ry0n, rz0n;
            if (mur && g == n - 1) {
                const T gy0 = sm.mg[1][0][0], gz0 = sm.mg[1][0][1], gy1 = sm.mg[1][1][0], gz1 = sm.mg[1][1][1];
                ry0o = sm.bn[pb][0];
                rz0o = sm.bn[pb][1];
                ry0n = ry0o - (T(0) - cdt * (gz0 - ez0));
                rz0n = rz0o - (cdt * (gy0 - ey0) - T(0));
                const T ry1n = sm.bn[pb][2] - (T(0) - cdt * (gz1 - ez1));
                const T rz1n = sm.bn[pb][3] - (cdt * (gy1 - ey1) - T(0));
                sm.bn[pb ^ 1][0] = ry0n;
                sm.bn[pb ^ 1][1] = rz0n;
                sm.bn[pb ^ 1][2] = ry1n;
                sm.bn[pb ^ 1][3] = rz1n;
                if (last && w >= tg.own0 && w < tg.own1) {
                    oB[0][n] = ry0n;
                    oB[1][n] = rz0n;
                    oB[2][n] = ry1n;
                    oB[3][n] = rz1n;
                }
            } else {
                ry0o = sm.b[pb][0][wr];
                rz0o = sm.b[pb][1][wr];
                ry0n = ry0o - (T(0) - cdt * (sm.e0z[wr] - ez0));
                rz0n = rz0o - (cdt * (sm.e0y[wr] - ey0) - T(0));
            }
            // phi^{n+3/2}: source g E0^{n+1/2}.B0^{n+1/2} at the centre
            const T eb0 = T(0), eb1 = ey0, eb2 = ez0;
            const T bb0 = half * (T(0) + T(0)) + bext(0, g);
            const T bb1 = half * (half * (by0 + ry0o) + half * (nby0 + ry0n)) + bext(1, g);
            const T bb2 = half * (half * (bz0 + rz0o) + half * (nbz0 + rz0n)) + bext(2, g);
            const T sax = gax * (eb0 * bb0 + eb1 * bb1 + eb2 * bb2);
            const T pa = sm.ph[qa][w], pbv = sm.ph[qb][w];
            const T pl = (!axp && g == 0) ? sm.ag[0][qb] : sm.ph[qb][wl];
            const T pr = (!axp && g == n - 1) ? sm.ag[1][qb] : sm.ph[qb][wr];
            T lap = T(0);
            lap += ((pr - T(2) * pbv) + pl) * inv_dx2;
            const T sdt = sdt_at(g);
            const T x = dt2 * ((sax - m2 * pbv) + lap) - sdt * sdt * pbv;
            T pn = ((x + sdt * pa) + T(2) * pbv) - pa;
            if (sdt != T(0)) pn = pn / (T(1) + sdt);
            sm.ph[qn][w] = pn;
            const bool own = last && w >= tg.own0 && w < tg.own1;
            if (!axp) {
                for (int side = 0; side < 2; side++) {
                    if (g != (side ? n - 1 : 0)) continue;
                    T gv;
                    if (outflow) {
                        // one-way wave and Klein-Gordon at the ghost (Sec. II.D, outflow)
                        const T gb = sm.ag[side][qb], ga = sm.ag[side][qa], rr = out_r;
                        const T xx = (((T(-2) * gb + T(2) * ga) - dt2 * (sax - m2 * gb)) + rr * pbv -
                                      rr * rr * (pbv - T(2) * gb)) / (rr + rr * rr);
                        gv = ga + rr * (pbv - xx);
                    } else {
                        gv = pn;
                    }
                    sm.ag[side][qn] = gv;
                    if (own) {
                        oA[side][0][0] = sm.ag[side][qb];
                        oA[side][1][0] = gv;
                    }
                }
            }
            if (own) {
                oB[0][g] = nby0;
                oB[1][g] = nbz0;
                oB[2][g] = nby1;
                oB[3][g] = nbz1;
                oP0[g] = pbv;
                oP1[g] = pn;
            }
        }
        __syncthreads();
    }
}

template <typename T, int W>
__global__ void __launch_bounds__(kW1Threads) k_wave1d(const RunK<T> *__restrict__ rp, long s0, int K)
{
    __shared__ W1Lds<T, W> sm;
    w1_pass<T, W>(*rp, blockIdx.x, s0, K, sm);
}

template <typename T, int W>
__global__ void __launch_bounds__(kW1Threads) kb_wave1d(const BItem *__restrict__ it, int nrun, long s, int K)
{
    __shared__ W1Lds<T, W> sm;
    const long b = blockIdx.x;
    const int q = find_item<kWave1>(it, nrun, b);
    const RunK<T>& r = *uniform_desc<RunK<T>>(it[q].rk);
    w1_pass<T, W>(r, (int)(b - it[q].blk[kWave1]), it[q].step0 + s, K, sm);
}

}  // namespace

int wave1d_window(bool batched)
{
    // measured (3000 steps; one run of 4096 or 65536 cells, and the 256 1D runs of
    // the 512-run scan in one batch): windows of 256 / 512 / 1024 cells take
    // 7.3 / 10.0 / 16.4 ms for the single FP32 runs (one wavefront per SIMD
    // works through a cell's chain of updates: a step costs the same whatever
    // the grid) and give 91.9 / 110.0 / 65.0 Gcell/s over the batch
    static const int env = [] {
        const char *e = getenv("AXF_W1_WIN");
        const int v = e ? atoi(e) : 0;
        return v == 256 || v == 512 || v == 1024 ? v : 0;
    }();
    return env ? env : (batched ? 512 : 256);
}

bool wave1d_k_ok(int k, int nem, int nph)
{
    const int kp = k % nph;
    return k >= 2 && k % nem != 0 && kp != 0 && kp != 1 && kp != nph - 1;
}

template <typename T>
int wave1d_kmax() { return kW1Kmax; }

int wave1d_pick(long free, int kmax, int nem, int nph)
{
    const int top = (int)std::min<long>(free, kmax);
    int any = 0;
    for (int k = top; k >= 2; k--) {
        if (!wave1d_k_ok(k, nem, nph)) continue;
        if (free - k != 1) return k;       // a remainder of one step would take the unfused kernels
        if (!any) any = k;
    }
    return any;
}

template <typename T>
long wave1d_tiles(const RunK<T>& h, int win) { return w1_ntiles(h.n[0], win, kW1Kmax); }

template <typename T>
hipError_t launch_wave1d(const RunK<T> *rk, const RunK<T>& h, long step, int K, int win, hipStream_t st)
{
    if (h.D != 1 || K < 2 || K > kW1Kmax || !wave1d_k_ok(K, h.nem, h.nph)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)wave1d_tiles(h, win));
    switch (win) {
    case 256: hipLaunchKernelGGL((k_wave1d<T, 256>), grid, dim3(kW1Threads), 0, st, rk, step, K); break;
    case 512: hipLaunchKernelGGL((k_wave1d<T, 512>), grid, dim3(kW1Threads), 0, st, rk, step, K); break;
    default: hipLaunchKernelGGL((k_wave1d<T, 1024>), grid, dim3(kW1Threads), 0, st, rk, step, K); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wave1d_batch(const BItem *it, const BItem *host, int n, long s, int K, int win, hipStream_t st)
{
    if (K < 2 || K > kW1Kmax) return hipErrorInvalidValue;
    const long blocks = host[n].blk[kWave1];
    if (blocks == 0) return hipSuccess;
    const dim3 grid((unsigned)blocks);
    switch (win) {
    case 256: hipLaunchKernelGGL((kb_wave1d<T, 256>), grid, dim3(kW1Threads), 0, st, it, n, s, K); break;
    case 512: hipLaunchKernelGGL((kb_wave1d<T, 512>), grid, dim3(kW1Threads), 0, st, it, n, s, K); break;
    default: hipLaunchKernelGGL((kb_wave1d<T, 1024>), grid, dim3(kW1Threads), 0, st, it, n, s, K); break;
    }
    return hipGetLastError();
}

template int wave1d_kmax<float>();
template int wave1d_kmax<double>();
template long wave1d_tiles<float>(const RunK<float>&, int);
template long wave1d_tiles<double>(const RunK<double>&, int);
template hipError_t launch_wave1d<float>(const RunK<float> *, const RunK<float>&, long, int, int, hipStream_t);
template hipError_t launch_wave1d<double>(const RunK<double> *, const RunK<double>&, long, int, int, hipStream_t);
template hipError_t launch_wave1d_batch<float>(const BItem *, const BItem *, int, long, int, int, hipStream_t);
template hipError_t launch_wave1d_batch<double>(const BItem *, const BItem *, int, long, int, int, hipStream_t);

}  // namespace axf
