// axf_stencil.h -- point stencils of the axion-coupled Yee step (device).
//
// Layout (Sec. II.C, the averaging formulas fix it): phi at cell centres
// (i+1/2, j+1/2, k+1/2); E_c on the faces normal to c, i.e. nodal along c and
// centred along the other axes; B_c on the edges along c, i.e. centred along c
// and nodal along the other axes.  Array index (i, j, k) of every component
// refers to those positions; along a Mur axis the nodal extent is n + 1.
//
// Time levels (leapfrog form of the half-step sequence of Sec. II.C):
//   E^{n+1/2} = E^{n-1/2} + dt (curl B^n - g S^n)          (order 1 only: -g S)
//   B^{n+1}   = B^n - dt curl E^{n+1/2}
//   phi^{n+3/2} from phi^{n+1/2}, phi^{n-1/2} and g E0^{n+1/2}.B0^{n+1/2}
// with S^n = (D_t phi)^n B0^n - E0^n x (D phi)^n formed at the two cell centres
// next to an E face and averaged onto it, E0^n the mean of E0^{n-+1/2}, phi^n the
// mean of the two axion levels, B0^{n+1/2} the mean of B0^n and B0^{n+1}.
#pragma once

#include "axf_internal.h"

namespace axf {

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ long lin(const RunK<T>& r, int i, int j, int k) { return i + j * r.sx + k * r.sy; }

template <typename T>
__device__ __forceinline__ long stride_of(const RunK<T>& r, int d) { return d == 0 ? 1 : (d == 1 ? r.sx : r.sy); }

// Linear offset of the neighbour at coordinate v + s along axis d (EM arrays):
// periodic axes wrap, Mur axes index straight (the caller stays in range).
template <typename T>
__device__ __forceinline__ long em_step(const RunK<T>& r, int d, int v, int s)
{
    int w = v + s;
    if (!r.mur[d]) w = wrapi(w, r.n[d]);
    return (long)(w - v) * stride_of(r, d);
}

// face index of the ghost planes normal to axis d: (coord_b * nn[a] + coord_a), a < b the other axes
template <typename R>
__device__ __forceinline__ long face_index(const R& r, int d, int i, int j, int k)
{
    return d == 0 ? (long)k * r.nn[1] + j : (d == 1 ? (long)k * r.nn[0] + i : (long)j * r.nn[0] + i);
}

__device__ __forceinline__ int coord(int d, int i, int j, int k) { return d == 0 ? i : (d == 1 ? j : k); }

template <int D, int O> __device__ __forceinline__ constexpr bool actE(int c) { return O == 0 ? actE0<D>(c) : actE1<D>(c); }
template <int D, int O> __device__ __forceinline__ constexpr bool actB(int c) { return O == 0 ? actB0<D>(c) : actB1<D>(c); }

template <int D, int O, typename T>
__device__ __forceinline__ T ldB(T *const *B, int c, long id) { return actB<D, O>(c) ? B[c][id] : T(0); }

// dt * (curl B)_c at the E_c point (i,j,k): forward differences
template <int D, int O, typename T>
__device__ __forceinline__ T curl_B(const RunK<T>& r, T *const *B, int c, int i, int j, int k, long id)
{
    T a = T(0), b = T(0);
    if (c == 0) {
        if (D >= 2 && actB<D, O>(2)) a = r.cdt[1] * (B[2][id + em_step(r, 1, j, 1)] - B[2][id]);
        if (D >= 3 && actB<D, O>(1)) b = r.cdt[2] * (B[1][id + em_step(r, 2, k, 1)] - B[1][id]);
    } else if (c == 1) {
        if (D >= 3 && actB<D, O>(0)) a = r.cdt[2] * (B[0][id + em_step(r, 2, k, 1)] - B[0][id]);
        if (actB<D, O>(2)) b = r.cdt[0] * (B[2][id + em_step(r, 0, i, 1)] - B[2][id]);
    } else {
        if (actB<D, O>(1)) a = r.cdt[0] * (B[1][id + em_step(r, 0, i, 1)] - B[1][id]);
        if (D >= 2 && actB<D, O>(0)) b = r.cdt[1] * (B[0][id + em_step(r, 1, j, 1)] - B[0][id]);
    }
    return a - b;
}

// E_c of order O in slot `slot` at (i,j,k) with coordinate v replacing the one
// along axis dd (E_c centred along dd): Mur ghosts outside [0, n), wrap if periodic.
template <int D, int O, typename T>
__device__ __forceinline__ T E_at(const RunK<T>& r, int slot, int mslot, int c, int dd, int v, int i, int j, int k)
{
    if (!actE<D, O>(c)) return T(0);
    T *const *E = O == 0 ? r.E0[slot] : r.E1[slot];
    if (!r.mur[dd]) {
        v = wrapi(v, r.n[dd]);
    } else if (v < 0 || v >= r.n[dd]) {
        int side = v < 0 ? 0 : 1;
        return r.murg[O][dd][side][c][mslot][face_index(r, dd, i, j, k)];
    }
    int ii = dd == 0 ? v : i, jj = dd == 1 ? v : j, kk = dd == 2 ? v : k;
    return E[c][lin(r, ii, jj, kk)];
}

// dt * (curl E)_c at the B_c point (i,j,k): backward differences, ghosts at Mur faces
template <int D, int O, typename T>
__device__ __forceinline__ T curl_E(const RunK<T>& r, int slot, int mslot, int c, int i, int j, int k)
{
    T a = T(0), b = T(0);
    if (c == 0) {
        if (D >= 2 && actE<D, O>(2))
            a = r.cdt[1] * (E_at<D, O>(r, slot, mslot, 2, 1, j, i, j, k) - E_at<D, O>(r, slot, mslot, 2, 1, j - 1, i, j, k));
        if (D >= 3 && actE<D, O>(1))
            b = r.cdt[2] * (E_at<D, O>(r, slot, mslot, 1, 2, k, i, j, k) - E_at<D, O>(r, slot, mslot, 1, 2, k - 1, i, j, k));
    } else if (c == 1) {
        if (D >= 3 && actE<D, O>(0))
            a = r.cdt[2] * (E_at<D, O>(r, slot, mslot, 0, 2, k, i, j, k) - E_at<D, O>(r, slot, mslot, 0, 2, k - 1, i, j, k));
        if (actE<D, O>(2))
            b = r.cdt[0] * (E_at<D, O>(r, slot, mslot, 2, 0, i, i, j, k) - E_at<D, O>(r, slot, mslot, 2, 0, i - 1, i, j, k));
    } else {
        if (actE<D, O>(1))
            a = r.cdt[0] * (E_at<D, O>(r, slot, mslot, 1, 0, i, i, j, k) - E_at<D, O>(r, slot, mslot, 1, 0, i - 1, i, j, k));
        if (D >= 2 && actE<D, O>(0))
            b = r.cdt[1] * (E_at<D, O>(r, slot, mslot, 0, 1, j, i, j, k) - E_at<D, O>(r, slot, mslot, 0, 1, j - 1, i, j, k));
    }
    return a - b;
}

// phi of a level (array ph, ghost slot gs) at the centre shifted by s along axis d
template <typename T>
__device__ __forceinline__ T phi_nb(const RunK<T>& r, const T *ph, int gs, int d, int s, int i, int j, int k, long id)
{
    int v = coord(d, i, j, k), w = v + s;
    if (r.axbc[d] == AXF_AX_PERIODIC) {
        w = wrapi(w, r.n[d]);
    } else if (w < 0 || w >= r.n[d]) {
        return r.axg[d][w < 0 ? 0 : 1][gs][face_index(r, d, i, j, k)];
    }
    return ph[id + (long)(w - v) * stride_of(r, d)];
}

// B_c averaged to the cell centre from 4 edge points (2 along each other
// active axis), pairs summed first; degenerate axes contribute the point itself.
template <int D, int O, typename T>
__device__ __forceinline__ T centre_B(const RunK<T>& r, T *const *B, int c, int i, int j, int k, long id)
{
    if (!actB<D, O>(c)) return T(0);
    const int a = c == 0 ? 1 : 0, b = c == 2 ? 1 : 2;
    const T *p = B[c];
    const bool ua = a < D, ub = b < D;
    if (!ua && !ub) return p[id];
    long oa = ua ? em_step(r, a, coord(a, i, j, k), 1) : 0;
    long ob = ub ? em_step(r, b, coord(b, i, j, k), 1) : 0;
    if (!ub) return r.half * (p[id] + p[id + oa]);
    return T(0.25) * ((p[id] + p[id + oa]) + (p[id + ob] + p[id + oa + ob]));
}

// E_c (value array pair averaged when two slots given) averaged to the centre along c
template <int D, typename T>
__device__ __forceinline__ T centre_E(const RunK<T>& r, const T *p, int c, int i, int j, int k, long id)
{
    if (c >= D) return p[id];
    return r.half * (p[id] + p[id + em_step(r, c, coord(c, i, j, k), 1)]);
}

template <typename R>
__device__ __forceinline__ auto bext_at(const R& r, int c, int i) -> decltype(r.half)
{
    using T = decltype(r.half);
    return (i >= r.slab_lo && i < r.slab_hi) ? r.bext[c] : T(0);
}

// sigma * dt of the PML layer at a cell: max over PML axes of
// sigma_max dt (1 - i/N)^3, i counted from the outermost cell (Sec. III.A)
template <int D, typename R>
__device__ __forceinline__ auto pml_sdt(const R& r, int i, int j, int k) -> decltype(r.half)
{
    using T = decltype(r.half);
    T s = T(0);
#pragma unroll
    for (int d = 0; d < D; d++) {
        if (r.axbc[d] != AXF_AX_PML) continue;
        int v = coord(d, i, j, k);
        int dist = v < r.n[d] - 1 - v ? v : r.n[d] - 1 - v;
        if (dist < r.pml_n) {
            T q = T(1) - T(dist) / T(r.pml_n);
            T sd = r.pml_sdt_max * q * q * q;
            s = sd > s ? sd : s;
        }
    }
    return s;
}

// First-order Mur update of one tangential E ghost (FP64) from the adjacent
// point's E^{n-1/2} and E^{n+1/2} and the ghost's old value, with the laser
// values of the per-level table on the x_min face (the unfused path's formula)
// The Mur formula itself on the scattered parts (E minus the laser's value
// at the adjacent point (ia) and at the ghost (ig), old and new levels)
__device__ __forceinline__ double mur_core(double murc, double e_old, double e_new, double g_old, double ia_o,
                                           double ia_n, double ig_o, double ig_n)
{
    double sa_o = e_old - ia_o, sa_n = e_new - ia_n, sg_o = g_old - ig_o;
    double sg_n = sa_o + murc * (sa_n - sg_o);
    return sg_n + ig_n;
}

template <typename T>
__device__ __forceinline__ T mur_update_rk(const RunK<T>& r, int O, int c, int d, int side, double e_old, double e_new,
                                           double g_old, long fidx, long step)
{
    double ia_o = 0.0, ia_n = 0.0, ig_o = 0.0, ig_n = 0.0;
    if (O == 0 && d == 0 && side == 0 && r.las.on && c == r.las.pol) {
        const long lo = (step % r.inc_k1) * 2 * r.inc_face, ln = ((step + 1) % r.inc_k1) * 2 * r.inc_face;
        ia_o = r.inc[lo + fidx];
        ig_o = r.inc[lo + r.inc_face + fidx];
        ia_n = r.inc[ln + fidx];
        ig_n = r.inc[ln + r.inc_face + fidx];
    }
    return (T)mur_core(r.murc[d], e_old, e_new, g_old, ia_o, ia_n, ig_o, ig_n);
}

// ----------------------------------------------------------- analytic inputs

// Laser field component comp (1: y, 2: z) at (x, y, z, t): sin^2-ramped CW or
// Gaussian envelope in t - x, paraxial Gaussian beam profile at the entry plane.
__device__ __noinline__ double incident(const Laser& L, int comp, double x, double y, double z, double t)
{
    if (!L.on || comp != L.pol) return 0.0;
    double tau = t - x, env;
    if (L.env == AXF_ENV_CW) {
        if (tau <= 0.0) env = 0.0;
        else if (tau < L.ramp_t) { double s = sin(0.5 * M_PI * tau / L.ramp_t); env = s * s; }
        else env = 1.0;
    } else {
        double u = (tau - L.t_center) / L.tau0;
        env = exp(-u * u);
    }
    double amp = 1.0, dph = 0.0;
    if (L.q > 0 && L.waist > 0.0) {
        double r2 = 0.0;
        r2 += (y - L.y_c) * (y - L.y_c);
        if (L.q > 1) r2 += (z - L.z_c) * (z - L.z_c);
        double xi = x - L.x_focus;
        double w2 = L.waist * L.waist * (1.0 + (xi / L.zr) * (xi / L.zr));
        amp = pow(L.waist * L.waist / w2, 0.25 * L.q) * exp(-r2 / w2);
        dph = -0.5 * L.omega * r2 * xi / (xi * xi + L.zr * L.zr) + 0.5 * L.q * atan(xi / L.zr);
    }
    return L.e_amp * amp * env * sin(L.omega * tau + dph + L.cep);
}

__device__ inline double packet_value(const Packet& P, int D, double x, double y, double z, double t)
{
    if (!P.on) return 0.0;
    double eta = x - P.x0 - P.dir * t, r2 = 0.0;
    if (D >= 2) r2 += (y - P.y0) * (y - P.y0);
    if (D >= 3) r2 += (z - P.z0) * (z - P.z0);
    return P.amp * exp(-(eta * eta + r2) / (P.w * P.w)) * sin(P.k * eta);
}

}  // namespace axf
