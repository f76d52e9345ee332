// axf_plain.hip -- the unfused step: one kernel per update phase of the
// leapfrog form (E0, axion current C, E1, Mur ghosts, B, axion), plus the
// initial state, the co-timed -> leapfrog conversion and the diagnostics.
// Every thread owns one storage index (i,j,k) and reads its neighbours from
// global memory.  These kernels are the correctness baseline of the fused path.
#include "axf_stencil.h"
#include "axf_kernels.h"

#include <mutex>

namespace axf {

// storage index p -> (i, j, k); 32-bit divisions (a few instructions, not
// the long 64-bit expansion) whenever the grid's point count fits in them
template <typename T>
__device__ __forceinline__ bool decompose(const RunK<T>& r, long p, int& i, int& j, int& k)
{
    if (p >= r.npts) return false;
    if (r.npts <= 0xffffffffL) {
        const unsigned up = (unsigned)p, n0 = (unsigned)r.nn[0], n1 = (unsigned)r.nn[1];
        const unsigned q = up / n0;
        i = (int)(up - q * n0);
        k = (int)(q / n1);
        j = (int)(q - (unsigned)k * n1);
        return true;
    }
    long q = p / r.nn[0];
    i = (int)(p - q * r.nn[0]);
    k = (int)(q / r.nn[1]);
    j = (int)(q - (long)k * r.nn[1]);
    return true;
}

template <int D, typename T>
__device__ __forceinline__ bool in_E(const RunK<T>& r, int c, int i, int j, int k)
{
    return i < (c == 0 ? r.nn[0] : r.n[0]) && j < (c == 1 ? r.nn[1] : r.n[1]) && k < (c == 2 ? r.nn[2] : r.n[2]);
}

template <int D, typename T>
__device__ __forceinline__ bool in_B(const RunK<T>& r, int c, int i, int j, int k)
{
    return i < (c != 0 ? r.nn[0] : r.n[0]) && j < (c != 1 ? r.nn[1] : r.n[1]) && k < (c != 2 ? r.nn[2] : r.n[2]);
}

template <typename T>
__device__ __forceinline__ bool in_cell(const RunK<T>& r, int i, int j, int k)
{
    return i < r.n[0] && j < r.n[1] && k < r.n[2];
}

// E0_out = E0_in + scale * dt (curl B0 - j0)   (scale 1: step; -1/2: backward
// half step; j0 only with particles, stored as dt j0)
template <int D, typename T>
__device__ __forceinline__ void e0_at(const RunK<T>& r, int i, int j, int k, int s_in, int s_b, int s_out, T scale)
{
    long id = lin(r, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (!actE0<D>(c) || !in_E<D>(r, c, i, j, k)) continue;
        T rhs = curl_B<D, 0>(r, r.B0[s_b], c, i, j, k, id);
        if (r.J[0][c]) rhs = rhs - r.J[0][c][id];
        r.E0[s_out][c][id] = r.E0[s_in][c][id] + scale * rhs;
    }
}

template <int D, typename T>
__device__ __forceinline__ void e0_body(const RunK<T>& r, long bx, int s_in, int s_b, int s_out, T scale)
{
    int i, j, k;
    if (!decompose(r, bx * 256 + threadIdx.x, i, j, k)) return;
    e0_at<D, T>(r, i, j, k, s_in, s_b, s_out, scale);
}

// C = (D_t phi) B0 - E0 x (D phi) at every centre for the integer time between
// axion slots (a, b); E0 = mean of slots (e_m, e_p), or slot e_m alone if cotimed.
template <int D, typename T>
__device__ __forceinline__ void c_at(const RunK<T>& r, int i, int j, int k, int pa, int pb, int e_m, int e_p, int s_b, int cotimed)
{
    if (!in_cell(r, i, j, k)) return;
    long id = lin(r, i, j, k);
    T e[3], b[3], gp[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        e[c] = T(0);
        if (actE0<D>(c)) {
            const T *m = r.E0[e_m][c], *p = r.E0[e_p][c];
            long o = c < D ? em_step(r, c, coord(c, i, j, k), 1) : 0;
            T lo = cotimed ? m[id] : r.half * (m[id] + p[id]);
            T hi = cotimed ? m[id + o] : r.half * (m[id + o] + p[id + o]);
            e[c] = c < D ? r.half * (lo + hi) : lo;
        }
        b[c] = centre_B<D, 0>(r, r.B0[s_b], c, i, j, k, id) + bext_at(r, c, i);
    }
    const T *A = r.phi[pa], *Bp = r.phi[pb];
    T dtphi = (Bp[id] - A[id]) * r.inv_dt;
#pragma unroll
    for (int d = 0; d < D; d++) {
        T up = r.half * (phi_nb(r, A, pa, d, 1, i, j, k, id) + phi_nb(r, Bp, pb, d, 1, i, j, k, id));
        T dn = r.half * (phi_nb(r, A, pa, d, -1, i, j, k, id) + phi_nb(r, Bp, pb, d, -1, i, j, k, id));
        gp[d] = (up - dn) * r.inv2dx[d];
    }
    r.C[0][id] = dtphi * b[0] - (e[1] * gp[2] - e[2] * gp[1]);
    r.C[1][id] = dtphi * b[1] - (e[2] * gp[0] - e[0] * gp[2]);
    r.C[2][id] = dtphi * b[2] - (e[0] * gp[1] - e[1] * gp[0]);
}

template <int D, typename T>
__device__ __forceinline__ void c_body(const RunK<T>& r, long bx, int pa, int pb, int e_m, int e_p, int s_b, int cotimed)
{
    int i, j, k;
    if (!decompose(r, bx * 256 + threadIdx.x, i, j, k)) return;
    c_at<D, T>(r, i, j, k, pa, pb, e_m, e_p, s_b, cotimed);
}

// E0 update and the axion current C in one launch: the E0^{n+1/2} values the
// C formula needs at the next face along each axis are recomputed, not read
template <int D, typename T>
__device__ __forceinline__ void e0c_at(const RunK<T>& r, int i, int j, int k, long step)
{
    const long id = lin(r, i, j, k);
    const int so = em_slot(step, r.nem), sn = em_slot(step + 1, r.nem), la = phi_slot(step, r.nph), lb = phi_slot(step + 1, r.nph);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (!actE0<D>(c) || !in_E<D>(r, c, i, j, k)) continue;
        r.E0[sn][c][id] = e0new_at<D, T>(r, so, c, i, j, k);
    }
    if (!in_cell(r, i, j, k)) return;
    T e[3], b[3], gp[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        e[c] = T(0);
        if (actE0<D>(c)) {
            const T *m = r.E0[so][c];
            const long o = c < D ? em_step(r, c, coord(c, i, j, k), 1) : 0;
            const T p0 = e0new_at<D, T>(r, so, c, i, j, k);
            T p1 = p0;
            if (c < D) {
                int i1 = i, j1 = j, k1 = k;
                coord_up(r, c, i1, j1, k1);
                p1 = e0new_at<D, T>(r, so, c, i1, j1, k1);
            }
            T lo = r.half * (m[id] + p0);
            T hi = r.half * (m[id + o] + p1);
            e[c] = c < D ? r.half * (lo + hi) : lo;
        }
        b[c] = centre_B<D, 0>(r, r.B0[so], c, i, j, k, id) + bext_at(r, c, i);
    }
    const T *A = r.phi[la], *Bp = r.phi[lb];
    T dtphi = (Bp[id] - A[id]) * r.inv_dt;
#pragma unroll
    for (int d = 0; d < D; d++) {
        T up = r.half * (phi_nb(r, A, la, d, 1, i, j, k, id) + phi_nb(r, Bp, lb, d, 1, i, j, k, id));
        T dn = r.half * (phi_nb(r, A, la, d, -1, i, j, k, id) + phi_nb(r, Bp, lb, d, -1, i, j, k, id));
        gp[d] = (up - dn) * r.inv2dx[d];
    }
    r.C[0][id] = dtphi * b[0] - (e[1] * gp[2] - e[2] * gp[1]);
    r.C[1][id] = dtphi * b[1] - (e[2] * gp[0] - e[0] * gp[2]);
    r.C[2][id] = dtphi * b[2] - (e[0] * gp[1] - e[1] * gp[0]);
}

// e0c_at on a walk up the z planes of one column: the z component of
// E0^{n+1/2} one plane up, which this plane's current needs, is the next
// plane's own value (the one it stores and averages): kept in `ez_up` (valid
// when `have`) instead of being computed again.  The same expressions as
// e0c_at, so the same bits.
template <int D, typename T>
__device__ __forceinline__ void e0c_walk_at(const RunK<T>& r, int i, int j, int k, long step, T& ez_up, bool& have)
{
    const long id = lin(r, i, j, k);
    const int so = em_slot(step, r.nem), sn = em_slot(step + 1, r.nem), la = phi_slot(step, r.nph), lb = phi_slot(step + 1, r.nph);
    T own[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (!actE0<D>(c) || !in_E<D>(r, c, i, j, k)) continue;
        own[c] = (D == 3 && c == 2 && have) ? ez_up : e0new_at<D, T>(r, so, c, i, j, k);
        r.E0[sn][c][id] = own[c];
    }
    have = false;
    // (a point of the current is a face point of every component, so own[]
    // holds all three below)
    if (!in_cell(r, i, j, k)) return;
    T e[3], b[3], gp[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        e[c] = T(0);
        if (actE0<D>(c)) {
            const T *m = r.E0[so][c];
            const long o = c < D ? em_step(r, c, coord(c, i, j, k), 1) : 0;
            const T p0 = own[c];
            T p1 = p0;
            if (c < D) {
                int i1 = i, j1 = j, k1 = k;
                coord_up(r, c, i1, j1, k1);
                p1 = e0new_at<D, T>(r, so, c, i1, j1, k1);
                if (c == 2) {
                    ez_up = p1;
                    have = true;
                }
            }
            T lo = r.half * (m[id] + p0);
            T hi = r.half * (m[id + o] + p1);
            e[c] = c < D ? r.half * (lo + hi) : lo;
        }
        b[c] = centre_B<D, 0>(r, r.B0[so], c, i, j, k, id) + bext_at(r, c, i);
    }
    const T *A = r.phi[la], *Bp = r.phi[lb];
    T dtphi = (Bp[id] - A[id]) * r.inv_dt;
#pragma unroll
    for (int d = 0; d < D; d++) {
        T up = r.half * (phi_nb(r, A, la, d, 1, i, j, k, id) + phi_nb(r, Bp, lb, d, 1, i, j, k, id));
        T dn = r.half * (phi_nb(r, A, la, d, -1, i, j, k, id) + phi_nb(r, Bp, lb, d, -1, i, j, k, id));
        gp[d] = (up - dn) * r.inv2dx[d];
    }
    r.C[0][id] = dtphi * b[0] - (e[1] * gp[2] - e[2] * gp[1]);
    r.C[1][id] = dtphi * b[1] - (e[2] * gp[0] - e[0] * gp[2]);
    r.C[2][id] = dtphi * b[2] - (e[0] * gp[1] - e[1] * gp[0]);
}

template <int D, typename T>
__device__ __forceinline__ void e0c_body(const RunK<T>& r, long bx, long step)
{
    int i, j, k;
    if (!decompose(r, bx * 256 + threadIdx.x, i, j, k)) return;
    e0c_at<D, T>(r, i, j, k, step);
}

// axion current on the E_c face: mean of C_c at the two adjacent centres (one
// interior centre on a Mur face, wrap on a periodic axis)
template <int D, typename T>
__device__ __forceinline__ T face_S(const RunK<T>& r, int c, int i, int j, int k, long id)
{
    const T *C = r.C[c];
    if (c >= D) return C[id];
    int v = coord(c, i, j, k), lo = v - 1, hi = v;
    if (r.mur[c]) {
        lo = lo < 0 ? 0 : lo;
        hi = hi > r.n[c] - 1 ? r.n[c] - 1 : hi;
    } else {
        lo = wrapi(lo, r.n[c]);
    }
    long st = stride_of(r, c);
    return r.half * (C[id + (long)(lo - v) * st] + C[id + (long)(hi - v) * st]);
}

// E1_out = E1_in + scale * dt (curl B1 - j1 - g1 S)   (j1 only with particles)
template <int D, typename T>
__device__ __forceinline__ void e1_at(const RunK<T>& r, int i, int j, int k, int s_in, int s_b, int s_out, T scale)
{
    long id = lin(r, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (!actE1<D>(c) || !in_E<D>(r, c, i, j, k)) continue;
        T rhs;
        if (r.J[1][c])
            rhs = (curl_B<D, 1>(r, r.B1[s_b], c, i, j, k, id) - r.J[1][c][id]) - r.cg1 * face_S<D>(r, c, i, j, k, id);
        else
            rhs = curl_B<D, 1>(r, r.B1[s_b], c, i, j, k, id) - r.cg1 * face_S<D>(r, c, i, j, k, id);
        r.E1[s_out][c][id] = r.E1[s_in][c][id] + scale * rhs;
    }
}

template <int D, typename T>
__device__ __forceinline__ void e1_body(const RunK<T>& r, long bx, int s_in, int s_b, int s_out, T scale)
{
    int i, j, k;
    if (!decompose(r, bx * 256 + threadIdx.x, i, j, k)) return;
    e1_at<D, T>(r, i, j, k, s_in, s_b, s_out, scale);
}

// First-order Mur for the tangential E ghost half a cell outside a Mur face, on
// the scattered part E - E_inc (E_inc nonzero for E0 on the x_min face):
// ghost^{n+1/2} = inc_g^{n+1/2} + s_a^{n-1/2} + c_M (s_a^{n+1/2} - s_g^{n-1/2}),
// c_M = (dt - dx)/(dt + dx), s = scattered part, a = adjacent interior centre.
template <int D, int O, typename T>
__device__ __forceinline__ void mur_point(const RunK<T>& r, long step, int d, int side, int c, int ia, int ib)
{
    if (!actE<D, O>(c)) return;
    const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
    int id3[3];
    id3[d] = side ? r.n[d] - 1 : 0;
    id3[a] = ia;
    id3[b] = ib;
    // E_c is nodal along c and centred along the other face axis
    for (int e = 0; e < 3; e++) {
        if (e == d) continue;
        int ext = (e == c) ? r.nn[e] : r.n[e];
        if (id3[e] >= ext) return;
    }
    const int s_old = em_slot(step, r.nem), s_new = em_slot(step + 1, r.nem);
    long id = lin(r, id3[0], id3[1], id3[2]);
    long f = face_index(r, d, id3[0], id3[1], id3[2]);
    T *const *Eo = O == 0 ? r.E0[s_old] : r.E1[s_old];
    T *const *En = O == 0 ? r.E0[s_new] : r.E1[s_new];
    double e_old = (double)Eo[c][id], e_new = (double)En[c][id];
    double g_old = (double)r.murg[O][d][side][c][s_old][f];
    double ia_o = 0.0, ia_n = 0.0, ig_o = 0.0, ig_n = 0.0;
    if (O == r.las.order && d == 0 && side == 0 && r.las.on && c == r.las.pol) {
        const long lo = (step % r.inc_k1) * 2 * r.inc_face, ln = ((step + 1) % r.inc_k1) * 2 * r.inc_face;
        ia_o = r.inc[lo + f];
        ig_o = r.inc[lo + r.inc_face + f];
        ia_n = r.inc[ln + f];
        ig_n = r.inc[ln + r.inc_face + f];
        if (O == 1) {
            // the first-order fields are stored divided by s_1
            const double is1 = 1.0 / r.s_1;
            ia_o *= is1;
            ig_o *= is1;
            ia_n *= is1;
            ig_n *= is1;
        }
    }
    double sa_o = e_old - ia_o, sa_n = e_new - ia_n, sg_o = g_old - ig_o;
    double sg_n = sa_o + r.murc[d] * (sa_n - sg_o);
    r.murg[O][d][side][c][s_new][f] = (T)(sg_n + ig_n);
}

template <int D, typename T>
__device__ __forceinline__ void mur_body(const RunK<T>& r, long bx, long step)
{
    const int d = blockIdx.y >> 1, side = blockIdx.y & 1;
    if (d >= D || !r.mur[d]) return;
    const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
    long p = bx * 256 + threadIdx.x;
    long na = r.nn[a], nb = r.nn[b];
    if (p >= na * nb) return;
    int ia = (int)(p % na), ib = (int)(p / na);
#pragma unroll
    for (int q = 0; q < 2; q++) {
        int c = q == 0 ? a : b;
        mur_point<D, 0>(r, step, d, side, c, ia, ib);
        mur_point<D, 1>(r, step, d, side, c, ia, ib);
    }
}

// laser field at the x_min face for time levels L0 .. L0 + nlev - 1 (t = (L - 1/2) dt),
// at the first interior centre and at the ghost centre, into slot L mod inc_k1
template <int D, typename T>
__device__ __forceinline__ void inc_fill_body(const RunK<T>& r, long bx, long L0, int nlev)
{
    long p = bx * 256 + threadIdx.x;
    if (p >= r.inc_face) return;
    const int c = r.las.pol;
    int j = (int)(p % r.nn[1]), k = (int)(p / r.nn[1]);
    double y = (c == 1) ? j * r.dx[1] : (j + 0.5) * r.dx[1];
    double z = (c == 2) ? k * r.dx[2] : (k + 0.5) * r.dx[2];
    for (int q = 0; q < nlev; q++) {
        long L = L0 + q;
        double t = (L - 0.5) * r.dt;
        long base = (L % r.inc_k1) * 2 * r.inc_face;
        r.inc[base + p] = incident(r.las, c, 0.5 * r.dx[0], y, z, t);
        r.inc[base + r.inc_face + p] = incident(r.las, c, -0.5 * r.dx[0], y, z, t);
    }
}

// Mur ghost slot 0 at t = -dt/2: the incident field on the x_min face, zero elsewhere
template <int D, typename T>
__global__ void k_mur_init(const RunK<T> *__restrict__ rp)
{
    const RunK<T>& r = *rp;
    const int d = blockIdx.y >> 1, side = blockIdx.y & 1;
    if (d >= D || !r.mur[d]) return;
    const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
    long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long na = r.nn[a], nb = r.nn[b];
    if (p >= na * nb) return;
    int ia = (int)(p % na), ib = (int)(p / na);
    for (int q = 0; q < 2; q++) {
        int c = q == 0 ? a : b;
        for (int o = 0; o < 2; o++) {
            T *g = r.murg[o][d][side][c][0];
            if (!g) continue;
            double v = 0.0;
            if (o == r.las.order && d == 0 && side == 0 && r.las.on) {
                int id3[3];
                id3[0] = 0; id3[a] = ia; id3[b] = ib;
                double y = (c == 1) ? id3[1] * r.dx[1] : (id3[1] + 0.5) * r.dx[1];
                double z = (c == 2) ? id3[2] * r.dx[2] : (id3[2] + 0.5) * r.dx[2];
                v = incident(r.las, c, -0.5 * r.dx[0], y, z, -0.5 * r.dt) / (o == 1 ? r.s_1 : 1.0);
            }
            g[p] = (T)v;
        }
    }
}

// B^{n+1} = B^n - dt curl E^{n+1/2}, both orders, old slot -> new slot
template <int D, typename T>
__device__ __forceinline__ void b_at(const RunK<T>& r, int i, int j, int k, long step)
{
    long id = lin(r, i, j, k);
    const int so = em_slot(step, r.nem), sn = em_slot(step + 1, r.nem);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (!in_B<D>(r, c, i, j, k)) continue;
        if (actB0<D>(c))
            r.B0[sn][c][id] = r.B0[so][c][id] - curl_E<D, 0>(r, sn, sn, c, i, j, k);
        if (actB1<D>(c))
            r.B1[sn][c][id] = r.B1[so][c][id] - curl_E<D, 1>(r, sn, sn, c, i, j, k);
    }
}

template <int D, typename T>
__device__ __forceinline__ void b_body(const RunK<T>& r, long bx, long step)
{
    int i, j, k;
    if (!decompose(r, bx * 256 + threadIdx.x, i, j, k)) return;
    b_at<D, T>(r, i, j, k, step);
}

// coordinates one step up along axis d (wrapped on a periodic axis)
template <typename T>
__device__ __forceinline__ void coord_up(const RunK<T>& r, int d, int& i, int& j, int& k)
{
    int& v = d == 0 ? i : (d == 1 ? j : k);
    v += 1;
    if (!r.mur[d]) v = wrapi(v, r.n[d]);
}

// E0^{n+1/2} at face point (i,j,k): the expression the E0 update stores
template <int D, typename T>
__device__ __forceinline__ T e0new_at(const RunK<T>& r, int so, int c, int i, int j, int k)
{
    const long id = lin(r, i, j, k);
    return r.E0[so][c][id] + T(1) * curl_B<D, 0>(r, r.B0[so], c, i, j, k, id);
}

// phi^{n+3/2}: leapfrog of the Klein-Gordon equation with source g E0.B0 at
// t_{n+1/2} (Sec. II.C, eq. update_axion), in the damped form of the PML
// layer (Sec. II.D) where sigma > 0, then the ghosts of the new level.
template <int D, typename T>
__device__ __forceinline__ void phi_at(const RunK<T>& r, int i, int j, int k, long step)
{
    if (!in_cell(r, i, j, k)) return;
    long id = lin(r, i, j, k);
    const int so = em_slot(step, r.nem), sn = em_slot(step + 1, r.nem);
    const int la = phi_slot(step, r.nph), lb = phi_slot(step + 1, r.nph), ln = phi_slot(step + 2, r.nph);
    T e[3], b[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        e[c] = actE0<D>(c) ? centre_E<D>(r, r.E0[sn][c], c, i, j, k, id) : T(0);
        T bo = centre_B<D, 0>(r, r.B0[so], c, i, j, k, id);
        T bn = centre_B<D, 0>(r, r.B0[sn], c, i, j, k, id);
        b[c] = r.half * (bo + bn) + bext_at(r, c, i);
    }
    T sax = r.gax * (e[0] * b[0] + e[1] * b[1] + e[2] * b[2]);
    const T *A = r.phi[la], *Bp = r.phi[lb];
    T pa = A[id], pb = Bp[id];
    T lap = T(0);
#pragma unroll
    for (int d = 0; d < D; d++)
        lap += ((phi_nb(r, Bp, lb, d, 1, i, j, k, id) - T(2) * pb) + phi_nb(r, Bp, lb, d, -1, i, j, k, id)) * r.inv_dx2[d];
    T sdt = pml_sdt<D>(r, i, j, k);
    T x = r.dt2 * ((sax - r.m2 * pb) + lap) - sdt * sdt * pb;
    // outside the damping layer the divisor is exactly 1: skip the division
    T pn = ((x + sdt * pa) + T(2) * pb) - pa;
    if (sdt != T(0)) pn = pn / (T(1) + sdt);
    r.phi[ln][id] = pn;
#pragma unroll
    for (int d = 0; d < D; d++) {
        if (r.axbc[d] == AXF_AX_PERIODIC) continue;
        int v = coord(d, i, j, k);
        for (int side = 0; side < 2; side++) {
            if (v != (side ? r.n[d] - 1 : 0)) continue;
            long f = face_index(r, d, i, j, k);
            T g;
            if (r.axbc[d] == AXF_AX_OUTFLOW) {
                // one-way wave and Klein-Gordon at the ghost (Sec. II.D, outflow)
                T gb = r.axg[d][side][lb][f], ga = r.axg[d][side][la][f], rr = r.out_r[d];
                T xx = (((T(-2) * gb + T(2) * ga) - r.dt2 * (sax - r.m2 * gb)) + rr * pb - rr * rr * (pb - T(2) * gb))
                       / (rr + rr * rr);
                g = ga + rr * (pb - xx);
            } else {
                g = pn;
            }
            r.axg[d][side][ln][f] = g;
        }
    }
}

template <int D, typename T>
__device__ __forceinline__ void phi_body(const RunK<T>& r, long bx, long step)
{
    int i, j, k;
    if (!decompose(r, bx * 256 + threadIdx.x, i, j, k)) return;
    phi_at<D, T>(r, i, j, k, step);
}

// initial axion levels at t = -dt/2 (slot 0) and +dt/2 (slot 1) from the packet,
// with their ghosts (outflow: the packet at the ghost centre; others: copies)
template <int D, typename T>
__global__ void __launch_bounds__(256) k_init_phi(const RunK<T> *__restrict__ rp)
{
    const RunK<T>& r = *rp;
    int i, j, k;
    if (!decompose(r, blockIdx.x * (long)blockDim.x + threadIdx.x, i, j, k)) return;
    if (!in_cell(r, i, j, k)) return;
    long id = lin(r, i, j, k);
    double x = (i + 0.5) * r.dx[0], y = (j + 0.5) * r.dx[1], z = (k + 0.5) * r.dx[2];
    double inv = 1.0 / r.s_phi;
    for (int L = 0; L < 2; L++) {
        double t = (L == 0 ? -0.5 : 0.5) * r.dt;
        r.phi[L][id] = (T)(packet_value(r.pk, D, x, y, z, t) * inv);
    }
    for (int d = 0; d < D; d++) {
        if (r.axbc[d] != AXF_AX_OUTFLOW) continue;
        int v = coord(d, i, j, k);
        for (int side = 0; side < 2; side++) {
            if (v != (side ? r.n[d] - 1 : 0)) continue;
            double pos[3] = {x, y, z};
            pos[d] = side ? (r.n[d] + 0.5) * r.dx[d] : -0.5 * r.dx[d];
            long f = face_index(r, d, i, j, k);
            for (int L = 0; L < 2; L++) {
                double t = (L == 0 ? -0.5 : 0.5) * r.dt;
                r.axg[d][side][L][f] = (T)(packet_value(r.pk, D, pos[0], pos[1], pos[2], t) * inv);
            }
        }
    }
}

// reflect / PML ghosts of axion slots 0 and 1 copied from the interior
template <int D, typename T>
__global__ void __launch_bounds__(256) k_copy_ghosts(const RunK<T> *__restrict__ rp, int s0, int s1)
{
    const RunK<T>& r = *rp;
    int i, j, k;
    if (!decompose(r, blockIdx.x * (long)blockDim.x + threadIdx.x, i, j, k)) return;
    if (!in_cell(r, i, j, k)) return;
    long id = lin(r, i, j, k);
    for (int d = 0; d < D; d++) {
        if (r.axbc[d] != AXF_AX_REFLECT && r.axbc[d] != AXF_AX_PML) continue;
        int v = coord(d, i, j, k);
        for (int side = 0; side < 2; side++) {
            if (v != (side ? r.n[d] - 1 : 0)) continue;
            long f = face_index(r, d, i, j, k);
            r.axg[d][side][s0][f] = r.phi[s0][id];
            r.axg[d][side][s1][f] = r.phi[s1][id];
        }
    }
}

// ---------------------------------------------------------------- diagnostics

template <typename T>
__device__ __forceinline__ bool finite_val(T v) { return v == v && v - v == T(0); }

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// block sums of the kDiagSums quantities in a fixed order (deterministic):
// each wave's sum, then the four waves in turn, written to out[q]
__device__ __forceinline__ void block_sums(double v[kDiagSums], double *out)
{
    __shared__ double red[4][kDiagSums];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kDiagSums; q++) {
        double s = wave_sum(v[q]);
        if (lane == 0) red[w][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < kDiagSums) {
        int q = threadIdx.x;
        out[q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
    }
}

// energies at t_n: E^n = mean of the two E slots, B^n = old slot, phi^n = mean
// of the axion levels; H_phi = sum ((D_t phi)^2 + sum_d (D+_d phi)^2 + m^2 phi^2) / 2.
// Sums 4 and 5: x B1z^2 and B1z^2 over the B1z points (on the x nodes, x = i dx),
// whose ratio is the laser centroid of Sec. III.D
template <int D, typename T>
__device__ __forceinline__ void diag_point(const RunK<T>& r, long p, long step, double v[kDiagSums])
{
    int i, j, k;
    if (decompose(r, p, i, j, k)) {
        long id = lin(r, i, j, k);
        const int so = em_slot(step, r.nem), sn = em_slot(step + 1, r.nem);
        const int la = phi_slot(step, r.nph), lb = phi_slot(step + 1, r.nph);
        bool fin = true;
        if (in_cell(r, i, j, k)) {
            const T *A = r.phi[la], *Bp = r.phi[lb];
            double pa = A[id], pb = Bp[id];
            double dtp = (pb - pa) / r.dt, pm = 0.5 * (pa + pb);
            double e = dtp * dtp + r.m2d * pm * pm;
            for (int d = 0; d < D; d++) {
                int vv = coord(d, i, j, k);
                if (r.axbc[d] != AXF_AX_PERIODIC && vv + 1 >= r.n[d]) continue;
                int w = wrapi(vv + 1, r.n[d]);
                long o = (long)(w - vv) * stride_of(r, d);
                double pn = 0.5 * ((double)A[id + o] + (double)Bp[id + o]);
                double gr = (pn - pm) / r.dx[d];
                e += gr * gr;
            }
            v[0] += 0.5 * e;
            fin = fin && finite_val(pa) && finite_val(pb);
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            if (in_E<D>(r, c, i, j, k)) {
                if (actE0<D>(c)) {
                    double ev = 0.5 * ((double)r.E0[so][c][id] + (double)r.E0[sn][c][id]);
                    v[1] += 0.5 * ev * ev;
                    fin = fin && finite_val(ev);
                }
                if (actE1<D>(c)) {
                    double ev = 0.5 * ((double)r.E1[so][c][id] + (double)r.E1[sn][c][id]);
                    v[2] += 0.5 * ev * ev;
                    fin = fin && finite_val(ev);
                }
            }
            if (in_B<D>(r, c, i, j, k)) {
                if (actB0<D>(c)) {
                    double bv = r.B0[so][c][id];
                    v[1] += 0.5 * bv * bv;
                    fin = fin && finite_val(bv);
                }
                if (actB1<D>(c)) {
                    double bv = r.B1[so][c][id];
                    v[2] += 0.5 * bv * bv;
                    fin = fin && finite_val(bv);
                    if (c == 2) {
                        v[4] += (double)i * (double)r.dx[0] * (bv * bv);
                        v[5] += bv * bv;
                    }
                }
            }
        }
        v[3] += fin ? 0.0 : 1.0;
    }
}

template <int D, typename T>
__device__ __forceinline__ void diag_body(const RunK<T>& r, long bx, long step)
{
    double v[kDiagSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    diag_point<D, T>(r, bx * 256 + threadIdx.x, step, v);
    block_sums(v, r.part + bx * kDiagSums);
}

// fixed-order sum of the block partials into record slot `slot`
template <typename T>
__device__ __forceinline__ void diag_fold(const RunK<T>& r, long step, const double *part, int nparts,
                                          axf_diag_record *dst)
{
    double v[kDiagSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // thread t adds partials t, t + 256, t + 512, ... in that order; the
    // loads of eight of them are issued before their additions
    constexpr int kU = 8;
    const int nt = (int)blockDim.x;
    int blk = threadIdx.x;
    for (; blk + (kU - 1) * nt < nparts; blk += kU * nt) {
        double w[kU][kDiagSums];
#pragma unroll
        for (int u = 0; u < kU; u++)
#pragma unroll
            for (int q = 0; q < kDiagSums; q++) w[u][q] = part[(long)(blk + u * nt) * kDiagSums + q];
#pragma unroll
        for (int u = 0; u < kU; u++)
#pragma unroll
            for (int q = 0; q < kDiagSums; q++) v[q] += w[u][q];
    }
    for (; blk < nparts; blk += nt)
#pragma unroll
        for (int q = 0; q < kDiagSums; q++) v[q] += part[(long)blk * kDiagSums + q];
    __shared__ double tot[kDiagSums];
    block_sums(v, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        double dv = 1.0;
        for (int d = 0; d < r.D; d++) dv *= r.dx[d];
        axf_diag_record rec;
        rec.step = step;
        rec.t = step * r.dt;
        rec.h_phi = tot[0] * dv * r.s_phi * r.s_phi;
        rec.h_em0 = tot[1] * dv;
        rec.h_em1 = tot[2] * dv * r.s_1 * r.s_1;
        rec.p_gen = rec.h_em0 > 0.0 ? rec.h_phi / rec.h_em0 : 0.0;
        rec.p_conv = rec.h_phi > 0.0 ? rec.h_em1 / rec.h_phi : 0.0;
        rec.finite = tot[3] == 0.0 ? 1 : 0;
        rec.pad = 0;
        rec.x_laser = tot[5] > 0.0 ? tot[4] / tot[5] : 0.0;
        *dst = rec;
    }
}

template <typename T>
__device__ __forceinline__ void diag_final_body(const RunK<T>& r, long step, int slot)
{
    diag_fold<T>(r, step, r.part, r.diag_blocks, &r.rec[slot]);
}

// ------------------------------------------------------ single-run kernels

template <int D, typename T>
__global__ void __launch_bounds__(256) k_e0(const RunK<T> *__restrict__ rp, int s_in, int s_b, int s_out, T scale)
{
    e0_body<D, T>(*rp, blockIdx.x, s_in, s_b, s_out, scale);
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_c(const RunK<T> *__restrict__ rp, int pa, int pb, int e_m, int e_p, int s_b, int cotimed)
{
    c_body<D, T>(*rp, blockIdx.x, pa, pb, e_m, e_p, s_b, cotimed);
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_e1(const RunK<T> *__restrict__ rp, int s_in, int s_b, int s_out, T scale)
{
    e1_body<D, T>(*rp, blockIdx.x, s_in, s_b, s_out, scale);
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_mur(const RunK<T> *__restrict__ rp, long step)
{
    mur_body<D, T>(*rp, blockIdx.x, step);
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_inc_fill(const RunK<T> *__restrict__ rp, long L0, int nlev)
{
    inc_fill_body<D, T>(*rp, blockIdx.x, L0, nlev);
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_b(const RunK<T> *__restrict__ rp, long step)
{
    b_body<D, T>(*rp, blockIdx.x, step);
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_phi(const RunK<T> *__restrict__ rp, long step)
{
    phi_body<D, T>(*rp, blockIdx.x, step);
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_diag(const RunK<T> *__restrict__ rp, long step)
{
    diag_body<D, T>(*rp, blockIdx.x, step);
}

template <typename T>
__global__ void __launch_bounds__(256) k_diag_final(const RunK<T> *__restrict__ rp, long step, int slot)
{
    diag_final_body<T>(*rp, step, slot);
}

// ------------------------------------------ static diagnostic workspace
// The partials and the record of axf_diag_now_static: kStaticDiagRows rows of
// kDiagSums FP64 sums, then one record.  Every device holds its own copy until
// the process ends; host code reaches it only through the device address that
// static_workspace looks up, never through this name.
static __device__ __align__(256) double scratch[kStaticDiagRows * kDiagSums + kStaticRecDoubles];
static_assert(sizeof(axf_diag_record) <= kStaticRecDoubles * sizeof(double), "record slot too small");
static_assert((kStaticDiagRows * kDiagSums * sizeof(double)) % 256 == 0, "record slot alignment");

// workgroup b folds the 256-point blocks b, b + rows, b + 2 rows, ... in turn
template <int D, typename T>
__global__ void __launch_bounds__(256) k_diag_rows(const RunK<T> *__restrict__ rp, long step, double *part, int rows)
{
    const RunK<T>& r = *rp;
    double v[kDiagSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long bx = blockIdx.x; bx < r.diag_blocks; bx += rows) diag_point<D, T>(r, bx * 256 + threadIdx.x, step, v);
    block_sums(v, part + (long)blockIdx.x * kDiagSums);
}

template <typename T>
__global__ void __launch_bounds__(256) k_diag_rows_final(const RunK<T> *__restrict__ rp, long step,
                                                         const double *part, int rows, axf_diag_record *dst)
{
    diag_fold<T>(*rp, step, part, rows, dst);
}

// merged phase of the semi-fused step: E0 with the axion current
template <int D, typename T>
__global__ void __launch_bounds__(256) k_e0c(const RunK<T> *__restrict__ rp, long step)
{
    e0c_body<D, T>(*rp, blockIdx.x, step);
}

// ------------------------------------------------------ 3D tiled launches
//
// The same point formulas on a tile walk: a workgroup of 64 x 4 threads owns a
// 64 x 4 column tile and walks kTZ consecutive z planes, so the y and z
// neighbours a point reads were just read by its own workgroup (cache hits)
// instead of by a workgroup far away in the launch order.

constexpr int kTX = 64, kTY = 4, kTZ = 4;
enum TilePhase { kTE0C = 0, kTE1, kTB, kTPhi };

// Occupancy in FP32 (measured on 512^3, Gcell/s of the whole step): E0 + the
// axion current held at 96 VGPRs, 5 wavefronts per SIMD instead of 4, no
// spills (16.0 -> 16.3); B at 8 instead of 7, some scalar registers spilled
// to vector lanes (-> 17.2).  The axion update at 7 spills vector registers
// and was slower.
template <int D, typename T, int PH>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && PH == kTE0C ? 5 : (sizeof(T) == 4 && PH == kTB ? 8 : 1))))
k3_tile(const RunK<T> *__restrict__ rp, long step, int tz)
{
    const RunK<T>& r = *rp;
    const int i = blockIdx.x * kTX + (threadIdx.x & (kTX - 1));
    const int j = blockIdx.y * kTY + (threadIdx.x / kTX);
    if (i >= r.nn[0] || j >= r.nn[1]) return;
    const int so = em_slot(step, r.nem), sn = em_slot(step + 1, r.nem);
    const int k0 = blockIdx.z * tz, k1 = min(k0 + tz, r.nn[2]);
    T ez_up = T(0);
    bool have = false;
    for (int k = k0; k < k1; k++) {
        if (PH == kTE0C) e0c_walk_at<D, T>(r, i, j, k, step, ez_up, have);
        else if (PH == kTE1) e1_at<D, T>(r, i, j, k, so, so, sn, T(1));
        else if (PH == kTB) b_at<D, T>(r, i, j, k, step);
        else phi_at<D, T>(r, i, j, k, step);
    }
}

// ---------------------------------------------------------- batched kernels
//
// One launch advances one phase of every active run of a batch group; block b
// belongs to the run found by find_item and runs that run's own body with the
// run's own step counter (step0 + s), so each run's arithmetic and block
// partition are those of its single-run launch.

enum BatchPhase { kPhE0 = 0, kPhC, kPhE0C, kPhE1, kPhB, kPhPhi, kPhDiag };

template <int D, typename T, int PH>
__device__ __forceinline__ void kb_volume_run(const RunK<T> *__restrict__ rp, long bx, long step)
{
    const RunK<T>& r = *rp;
    const int so = em_slot(step, r.nem), sn = em_slot(step + 1, r.nem), la = phi_slot(step, r.nph), lb = phi_slot(step + 1, r.nph);
    if (PH == kPhE0) e0_body<D, T>(r, bx, so, so, sn, T(1));
    else if (PH == kPhC) c_body<D, T>(r, bx, la, lb, so, sn, so, 0);
    else if (PH == kPhE0C) e0c_body<D, T>(r, bx, step);
    else if (PH == kPhE1) e1_body<D, T>(r, bx, so, so, sn, T(1));
    else if (PH == kPhB) b_body<D, T>(r, bx, step);
    else if (PH == kPhPhi) phi_body<D, T>(r, bx, step);
    else diag_body<D, T>(r, bx, step);
}

template <int D, typename T, int PH>
__global__ void __launch_bounds__(256) kb_volume(const BItem *__restrict__ it, int n, long s)
{
    const int i = find_item<kVolume>(it, n, blockIdx.x);
    kb_volume_run<D, T, PH>(uniform_desc<RunK<T>>(it[i].rk), blockIdx.x - it[i].blk[kVolume], it[i].step0 + s);
}

template <int D, typename T>
__device__ __forceinline__ void kb_mur_run(const RunK<T> *__restrict__ rp, long bx, long step)
{
    mur_body<D, T>(*rp, bx, step);
}

template <int D, typename T>
__global__ void __launch_bounds__(256) kb_mur(const BItem *__restrict__ it, int n, long s)
{
    const int i = find_item<kFace>(it, n, blockIdx.x);
    kb_mur_run<D, T>(uniform_desc<RunK<T>>(it[i].rk), blockIdx.x - it[i].blk[kFace], it[i].step0 + s);
}

template <int D, typename T>
__device__ __forceinline__ void kb_inc_run(const RunK<T> *__restrict__ rp, long bx, long L0, int nlev)
{
    inc_fill_body<D, T>(*rp, bx, L0, nlev);
}

template <int D, typename T>
__global__ void __launch_bounds__(256) kb_inc_fill(const BItem *__restrict__ it, int n, long s, int nlev)
{
    const int i = find_item<kLaser>(it, n, blockIdx.x);
    kb_inc_run<D, T>(uniform_desc<RunK<T>>(it[i].rk), blockIdx.x - it[i].blk[kLaser], it[i].step0 + s, nlev);
}

// one block per run: record `ev` of this call goes to slot (rec0 + ev) mod rec_cap
template <typename T>
__global__ void __launch_bounds__(256) kb_diag_final(const BItem *__restrict__ it, long s, long ev)
{
    const BItem& b = it[blockIdx.x];
    const RunK<T>& r = *(const RunK<T> *)b.rk;
    diag_final_body<T>(r, b.step0 + s, (int)((b.rec0 + ev) % r.rec_cap));
}

// ------------------------------------------------------------------ launchers

static inline unsigned nblocks(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <int D, typename T>
void Plain<D, T>::e0(const RunK<T> *rk, const RunK<T>& h, int s_in, int s_b, int s_out, T scale, hipStream_t st)
{
    hipLaunchKernelGGL((k_e0<D, T>), dim3(nblocks(h.npts, 256)), dim3(256), 0, st, rk, s_in, s_b, s_out, scale);
}

template <int D, typename T>
void Plain<D, T>::c(const RunK<T> *rk, const RunK<T>& h, int pa, int pb, int e_m, int e_p, int s_b, int cotimed, hipStream_t st)
{
    hipLaunchKernelGGL((k_c<D, T>), dim3(nblocks(h.npts, 256)), dim3(256), 0, st, rk, pa, pb, e_m, e_p, s_b, cotimed);
}

template <int D, typename T>
void Plain<D, T>::e1(const RunK<T> *rk, const RunK<T>& h, int s_in, int s_b, int s_out, T scale, hipStream_t st)
{
    hipLaunchKernelGGL((k_e1<D, T>), dim3(nblocks(h.npts, 256)), dim3(256), 0, st, rk, s_in, s_b, s_out, scale);
}

template <int D, typename T>
void Plain<D, T>::mur(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st)
{
    long face = 0;
    for (int d = 0; d < D; d++) {
        if (!h.mur[d]) continue;
        int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
        long f = (long)h.nn[a] * h.nn[b];
        face = f > face ? f : face;
    }
    if (face == 0) return;
    hipLaunchKernelGGL((k_mur<D, T>), dim3(nblocks(face, 256), 2 * D), dim3(256), 0, st, rk, step);
}

template <int D, typename T>
void Plain<D, T>::mur_init(const RunK<T> *rk, const RunK<T>& h, hipStream_t st)
{
    long face = 0;
    for (int d = 0; d < D; d++) {
        if (!h.mur[d]) continue;
        int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
        long f = (long)h.nn[a] * h.nn[b];
        face = f > face ? f : face;
    }
    if (face == 0) return;
    hipLaunchKernelGGL((k_mur_init<D, T>), dim3(nblocks(face, 256), 2 * D), dim3(256), 0, st, rk);
}

template <int D, typename T>
void Plain<D, T>::inc_fill(const RunK<T> *rk, const RunK<T>& h, long L0, int nlev, hipStream_t st)
{
    hipLaunchKernelGGL((k_inc_fill<D, T>), dim3(nblocks(h.inc_face, 256)), dim3(256), 0, st, rk, L0, nlev);
}

template <int D, typename T>
void Plain<D, T>::b(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st)
{
    hipLaunchKernelGGL((k_b<D, T>), dim3(nblocks(h.npts, 256)), dim3(256), 0, st, rk, step);
}

template <int D, typename T>
void Plain<D, T>::phi(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st)
{
    hipLaunchKernelGGL((k_phi<D, T>), dim3(nblocks(h.npts, 256)), dim3(256), 0, st, rk, step);
}

template <int D, typename T>
void Plain<D, T>::init_phi(const RunK<T> *rk, const RunK<T>& h, hipStream_t st)
{
    hipLaunchKernelGGL((k_init_phi<D, T>), dim3(nblocks(h.npts, 256)), dim3(256), 0, st, rk);
}

template <int D, typename T>
void Plain<D, T>::copy_ghosts(const RunK<T> *rk, const RunK<T>& h, int s0, int s1, hipStream_t st)
{
    hipLaunchKernelGGL((k_copy_ghosts<D, T>), dim3(nblocks(h.npts, 256)), dim3(256), 0, st, rk, s0, s1);
}

template <int D, typename T>
void Plain<D, T>::diag(const RunK<T> *rk, const RunK<T>& h, long step, int slot, hipStream_t st)
{
    hipLaunchKernelGGL((k_diag<D, T>), dim3(nblocks(h.npts, 256)), dim3(256), 0, st, rk, step);
    hipLaunchKernelGGL((k_diag_final<T>), dim3(1), dim3(256), 0, st, rk, step, slot);
}

template <int D, typename T>
void Plain<D, T>::diag_rows(const RunK<T> *rk, const RunK<T>& h, long step, double *ws, int rows, hipStream_t st)
{
    hipLaunchKernelGGL((k_diag_rows<D, T>), dim3(rows), dim3(256), 0, st, rk, step, ws, rows);
    hipLaunchKernelGGL((k_diag_rows_final<T>), dim3(1), dim3(256), 0, st, rk, step, (const double *)ws, rows,
                       (axf_diag_record *)(ws + kStaticDiagRows * kDiagSums));
}

static std::mutex g_ws_mu;
static double *g_ws_ptr[64];

hipError_t static_workspace(int dev, double **ptr)
{
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_ws_mu);
    if (!g_ws_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ws_ptr[dev] = (double *)p;
    }
    *ptr = g_ws_ptr[dev];
    return hipSuccess;
}

template <int D, typename T>
void Plain<D, T>::e0c(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st)
{
    hipLaunchKernelGGL((k_e0c<D, T>), dim3(nblocks(h.npts, 256)), dim3(256), 0, st, rk, step);
}

template <int D, typename T>
void Plain<D, T>::tiled_step(const RunK<T> *rk, const RunK<T>& h, long step, int tz, hipStream_t st)
{
    if (tz <= 0) tz = kTZ;
    const dim3 grid((unsigned)((h.nn[0] + kTX - 1) / kTX), (unsigned)((h.nn[1] + kTY - 1) / kTY),
                    (unsigned)((h.nn[2] + tz - 1) / tz));
    hipLaunchKernelGGL((k3_tile<D, T, kTE0C>), grid, dim3(256), 0, st, rk, step, tz);
    hipLaunchKernelGGL((k3_tile<D, T, kTE1>), grid, dim3(256), 0, st, rk, step, tz);
    mur(rk, h, step, st);
    hipLaunchKernelGGL((k3_tile<D, T, kTB>), grid, dim3(256), 0, st, rk, step, tz);
    hipLaunchKernelGGL((k3_tile<D, T, kTPhi>), grid, dim3(256), 0, st, rk, step, tz);
}

template <int D, typename T>
void Plain<D, T>::batch_step(const BItem *it, const BItem *host, int n, long s, hipStream_t st)
{
    const unsigned nv = (unsigned)host[n].blk[kVolume], nf = (unsigned)host[n].blk[kFace];
    if (nv == 0) return;
    if (D == 3) {
        // E0 with the axion current in one launch, as in a single 3D run
        hipLaunchKernelGGL((kb_volume<D, T, kPhE0C>), dim3(nv), dim3(256), 0, st, it, n, s);
    } else {
        hipLaunchKernelGGL((kb_volume<D, T, kPhE0>), dim3(nv), dim3(256), 0, st, it, n, s);
        hipLaunchKernelGGL((kb_volume<D, T, kPhC>), dim3(nv), dim3(256), 0, st, it, n, s);
    }
    hipLaunchKernelGGL((kb_volume<D, T, kPhE1>), dim3(nv), dim3(256), 0, st, it, n, s);
    if (nf > 0) hipLaunchKernelGGL((kb_mur<D, T>), dim3(nf, 2 * D), dim3(256), 0, st, it, n, s);
    hipLaunchKernelGGL((kb_volume<D, T, kPhB>), dim3(nv), dim3(256), 0, st, it, n, s);
    hipLaunchKernelGGL((kb_volume<D, T, kPhPhi>), dim3(nv), dim3(256), 0, st, it, n, s);
}

template <int D, typename T>
void Plain<D, T>::batch_inc_fill(const BItem *it, const BItem *host, int n, long s, int nlev, hipStream_t st)
{
    const unsigned nl = (unsigned)host[n].blk[kLaser];
    if (nl > 0) hipLaunchKernelGGL((kb_inc_fill<D, T>), dim3(nl), dim3(256), 0, st, it, n, s, nlev);
}

template <int D, typename T>
void Plain<D, T>::batch_diag(const BItem *it, const BItem *host, int n, long s, long ev, hipStream_t st)
{
    const unsigned nv = (unsigned)host[n].blk[kVolume];
    if (nv == 0) return;
    hipLaunchKernelGGL((kb_volume<D, T, kPhDiag>), dim3(nv), dim3(256), 0, st, it, n, s);
    hipLaunchKernelGGL((kb_diag_final<T>), dim3(n), dim3(256), 0, st, it, s, ev);
}

template struct Plain<1, float>;
template struct Plain<2, float>;
template struct Plain<3, float>;
template struct Plain<1, double>;
template struct Plain<2, double>;
template struct Plain<3, double>;

}  // namespace axf
