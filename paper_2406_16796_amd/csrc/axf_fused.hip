// axf_fused.hip -- the fused step: one launch advances every field of a run by
// one full step, so each cell's state is read once and written once from HBM.
//
// A workgroup owns an in-plane tile (x for 2D; x,y for 3D) and marches along the
// last axis M (y for 2D, z for 3D) over a chunk of planes.  Each plane of each
// input is loaded once (prefetched one iteration ahead into registers) into an
// LDS window of recent planes that covers the tile plus a halo of 3 cells on
// each side.  The intermediate quantities of the step are computed plane by
// plane, each in its own LDS window, lagging the newest loaded plane:
//   S1  E0^{n+1/2} and E0^n at plane t-1        (+ Mur ghosts of E0)
//   S2  axion current C^n at centres, plane t-2
//   S3  B0^{n+1} at plane t-1
//   S4  E1^{n+1/2} at plane t-2                 (+ Mur ghosts of E1)
//   S5  B1^{n+1} at plane t-2
//   S6  phi^{n+3/2} at plane t-2                (+ axion ghosts of the new level)
// The point formulas are the ones of the unfused kernels, written in the same
// operation order, so the two paths agree bit for bit.
#include <stdlib.h>

#include <type_traits>
#include <utility>

#include "axf_fused.h"
#include "axf_stencil.h"

namespace axf {

__device__ __forceinline__ int pmod(int p, int w) { int r = p % w; return r < 0 ? r + w : r; }
__device__ __forceinline__ int imod(int v, int n) { int r = v % n; return r < 0 ? r + n : r; }
// periodic wrap of a coordinate at most one period outside [0, n)
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// dynamic LDS of the fused kernel (accessed through the symbol so that the
// compiler keeps LDS addressing)
extern __shared__ __align__(16) unsigned char axf_smem[];

template <typename T>
__device__ __forceinline__ T *lds() { return reinterpret_cast<T *>(axf_smem); }

// state arrays live in global memory: address them as such, so that their
// loads and stores do not share the LDS counters (generic pointers would)
template <typename T>
__device__ __forceinline__ T gld(const T *p, long i) { return ((const __attribute__((address_space(1))) T *)p)[i]; }
template <typename T>
__device__ __forceinline__ void gst(T *p, long i, T v) { ((__attribute__((address_space(1))) T *)p)[i] = v; }

// Registers-resident view of a run for one step: the two base pointers of the
// uniform layout, the geometry and the coefficients (loaded once per launch,
// so that nothing in the march has to wait on a descriptor load)
template <typename T>
struct KV {
    const char *sb, *fb;       // field arrays / boundary planes
    long as, fs;               // their strides in bytes
    int n[3], nn[3], mur[3], axbc[3];
    long sx, sy;
    T cdt[3], half, inv_dt, inv2dx[3], inv_dx2[3], dt2, m2, gax, cg1, out_r[3], bext[3], pml_sdt_max;
    int slab_lo, slab_hi, pml_n;
    const double *inc;          // laser table on the x_min face (see RunK::inc)
    long inc_face;
    int inc_k1, las_on, las_pol;
    int nem, nph;
    double murc[3];

    __device__ __forceinline__ const T *arr(int q) const { return (const T *)(sb + q * as); }
    __device__ __forceinline__ T *warr(int q) const { return (T *)(sb + q * as); }
    __device__ __forceinline__ const T *face(int q) const { return (const T *)(fb + q * fs); }
    __device__ __forceinline__ T *wface(int q) const { return (T *)(fb + q * fs); }
};

template <typename T>
__device__ __forceinline__ KV<T> make_kv(const RunK<T> *__restrict__ rp)
{
    KV<T> v;
    v.sb = rp->state_base;
    v.fb = rp->face_base;
    v.as = rp->arr_stride;
    v.fs = rp->face_stride;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        v.n[d] = rp->n[d];
        v.nn[d] = rp->nn[d];
        v.mur[d] = rp->mur[d];
        v.axbc[d] = rp->axbc[d];
        v.cdt[d] = rp->cdt[d];
        v.inv2dx[d] = rp->inv2dx[d];
        v.inv_dx2[d] = rp->inv_dx2[d];
        v.out_r[d] = rp->out_r[d];
        v.bext[d] = rp->bext[d];
    }
    v.sx = rp->sx;
    v.sy = rp->sy;
    v.half = rp->half;
    v.inv_dt = rp->inv_dt;
    v.dt2 = rp->dt2;
    v.m2 = rp->m2;
    v.gax = rp->gax;
    v.cg1 = rp->cg1;
    v.pml_sdt_max = rp->pml_sdt_max;
    v.slab_lo = rp->slab_lo;
    v.slab_hi = rp->slab_hi;
    v.pml_n = rp->pml_n;
    v.inc = rp->inc;
    v.inc_face = rp->inc_face;
    v.inc_k1 = rp->inc_k1;
    v.las_on = rp->las.on;
    v.las_pol = rp->las.pol;
    v.nem = rp->nem;
    v.nph = rp->nph;
#pragma unroll
    for (int d = 0; d < 3; d++) v.murc[d] = rp->murc[d];
    return v;
}

template <int D, int TX, int TY, typename T>
struct FK {
    static constexpr int M = D - 1;
    static constexpr int RX = TX + 6, RY = (D == 3 ? TY + 6 : 1), R = RX * RY;
    static constexpr int NT = ((R + 63) / 64) * 64;
    static constexpr int W_B0N = 3, W_PH = 3, W_B1N = 2, W2 = 2;
    static constexpr int nE0 = D == 3 ? 3 : 2, nB0 = D == 3 ? 3 : 1;
    __host__ __device__ static constexpr int iE0(int c) { return c; }                 // 2D: E0x, E0y
    __host__ __device__ static constexpr int iB0(int c) { return D == 3 ? c : 0; }    // 2D: B0z only
    static constexpr int oB0N = 0;
    static constexpr int oPHA = oB0N + nB0 * W_B0N;
    static constexpr int oPHB = oPHA + W_PH;
    static constexpr int oB1N = oPHB + W_PH;
    static constexpr int oE0H = oB1N + 3 * W_B1N;
    static constexpr int oE0N = oE0H + nE0 * W2;
    static constexpr int oC = oE0N + nE0 * W2;
    static constexpr int oB0P = oC + 3 * W2;
    static constexpr int oE1H = oB0P + nB0 * W2;
    static constexpr int NPL = oE1H + 3 * W2;
    static constexpr size_t LDS = (size_t)NPL * R * sizeof(T);
    // in-plane region index shift of a unit step along axis a (a != M)
    __device__ static constexpr int sh(int a) { return a == 0 ? 1 : RX; }
};

// one point's view of the LDS windows
template <int D, int TX, int TY, typename T>
struct Win {
    using K = FK<D, TX, TY, T>;
    int li;   // region index of the point
    // value of window buffer `base` (W planes) at plane p + o[M], in-plane offset o
    __device__ __forceinline__ T at(int base, int W, int p, int o0, int o1, int o2) const
    {
        const int o[3] = {o0, o1, o2};
        int plane = p + o[K::M];
        int idx = li;
#pragma unroll
        for (int a = 0; a < D; a++)
            if (a != K::M) idx += o[a] * K::sh(a);
        return lds<T>()[(base + pmod(plane, W)) * K::R + idx];
    }
    __device__ __forceinline__ T &ref(int base, int W, int p) const { return lds<T>()[(base + pmod(p, W)) * K::R + li]; }
};

// unit offset along axis a as an (o0, o1, o2) triple
#define OFF(a, s) ((a) == 0 ? (s) : 0), ((a) == 1 ? (s) : 0), ((a) == 2 ? (s) : 0)

template <int D, int TX, int TY, typename T>
struct FusedStep {
    using K = FK<D, TX, TY, T>;
    using Wn = Win<D, TX, TY, T>;
    static constexpr int M = K::M;

    // buffers of the quantities (plane-buffer base of component c)
    __device__ static int bB0N(int c) { return K::oB0N + K::iB0(c) * K::W_B0N; }
    __device__ static int bB1N(int c) { return K::oB1N + c * K::W_B1N; }
    __device__ static int bE0H(int c) { return K::oE0H + K::iE0(c) * K::W2; }
    __device__ static int bE0N(int c) { return K::oE0N + K::iE0(c) * K::W2; }
    __device__ static int bC(int c) { return K::oC + c * K::W2; }
    __device__ static int bB0P(int c) { return K::oB0P + K::iB0(c) * K::W2; }
    __device__ static int bE1H(int c) { return K::oE1H + c * K::W2; }

    template <int O>
    __device__ static T B_n(const Wn& w, int c, int p, int o0, int o1, int o2)
    {
        return O == 0 ? w.at(bB0N(c), K::W_B0N, p, o0, o1, o2) : w.at(bB1N(c), K::W_B1N, p, o0, o1, o2);
    }

    // dt (curl B)_c at the E_c point: same terms and order as curl_B of the unfused path
    template <int O>
    __device__ static T curlB(const KV<T>& r, const Wn& w, int c, int p)
    {
        T a = T(0), b = T(0);
        if (c == 0) {
            if (D >= 2 && actB<D, O>(2)) a = r.cdt[1] * (B_n<O>(w, 2, p, OFF(1, 1)) - B_n<O>(w, 2, p, 0, 0, 0));
            if (D >= 3 && actB<D, O>(1)) b = r.cdt[2] * (B_n<O>(w, 1, p, OFF(2, 1)) - B_n<O>(w, 1, p, 0, 0, 0));
        } else if (c == 1) {
            if (D >= 3 && actB<D, O>(0)) a = r.cdt[2] * (B_n<O>(w, 0, p, OFF(2, 1)) - B_n<O>(w, 0, p, 0, 0, 0));
            if (actB<D, O>(2)) b = r.cdt[0] * (B_n<O>(w, 2, p, OFF(0, 1)) - B_n<O>(w, 2, p, 0, 0, 0));
        } else {
            if (actB<D, O>(1)) a = r.cdt[0] * (B_n<O>(w, 1, p, OFF(0, 1)) - B_n<O>(w, 1, p, 0, 0, 0));
            if (D >= 2 && actB<D, O>(0)) b = r.cdt[1] * (B_n<O>(w, 0, p, OFF(1, 1)) - B_n<O>(w, 0, p, 0, 0, 0));
        }
        return a - b;
    }

    template <int O>
    __device__ static T E_h(const Wn& w, int c, int p, int o0, int o1, int o2)
    {
        if (!actE<D, O>(c)) return T(0);
        return O == 0 ? w.at(bE0H(c), K::W2, p, o0, o1, o2) : w.at(bE1H(c), K::W2, p, o0, o1, o2);
    }

    // dt (curl E)_c at the B_c point from E^{n+1/2} (ghosts already in the windows)
    template <int O>
    __device__ static T curlE(const KV<T>& r, const Wn& w, int c, int p)
    {
        T a = T(0), b = T(0);
        if (c == 0) {
            if (D >= 2 && actE<D, O>(2)) a = r.cdt[1] * (E_h<O>(w, 2, p, 0, 0, 0) - E_h<O>(w, 2, p, OFF(1, -1)));
            if (D >= 3 && actE<D, O>(1)) b = r.cdt[2] * (E_h<O>(w, 1, p, 0, 0, 0) - E_h<O>(w, 1, p, OFF(2, -1)));
        } else if (c == 1) {
            if (D >= 3 && actE<D, O>(0)) a = r.cdt[2] * (E_h<O>(w, 0, p, 0, 0, 0) - E_h<O>(w, 0, p, OFF(2, -1)));
            if (actE<D, O>(2)) b = r.cdt[0] * (E_h<O>(w, 2, p, 0, 0, 0) - E_h<O>(w, 2, p, OFF(0, -1)));
        } else {
            if (actE<D, O>(1)) a = r.cdt[0] * (E_h<O>(w, 1, p, 0, 0, 0) - E_h<O>(w, 1, p, OFF(0, -1)));
            if (D >= 2 && actE<D, O>(0)) b = r.cdt[1] * (E_h<O>(w, 0, p, 0, 0, 0) - E_h<O>(w, 0, p, OFF(1, -1)));
        }
        return a - b;
    }

    // 4-point centre average of a B window buffer (same order as centre_B)
    template <int O>
    __device__ static T centreB(const Wn& w, int base, int W, int c, int p)
    {
        if (!actB<D, O>(c)) return T(0);
        const int a = c == 0 ? 1 : 0, b = c == 2 ? 1 : 2;
        const bool ua = a < D, ub = b < D;
        T p00 = w.at(base, W, p, 0, 0, 0);
        if (!ua && !ub) return p00;
        T pa = w.at(base, W, p, OFF(a, 1));
        if (!ub) return T(0.5) * (p00 + pa);
        T pb = w.at(base, W, p, OFF(b, 1));
        T pab = w.at(base, W, p, (a == 0 || b == 0) ? 1 : 0, (a == 1 || b == 1) ? 1 : 0, (a == 2 || b == 2) ? 1 : 0);
        return T(0.25) * ((p00 + pa) + (pb + pab));
    }
};

// ------------------------------------------------------------------ loads

// coordinate v along axis d of an EM array: wrapped on periodic axes, checked
// against the nodal or centred extent on Mur axes
template <typename R>
__device__ __forceinline__ bool em_coord(const R& r, int d, int v, bool nodal, int& w)
{
    if (!r.mur[d]) { w = wrap1(v, r.n[d]); return true; }
    w = v;
    return v >= 0 && v < (nodal ? r.nn[d] : r.n[d]);
}

template <int D, typename R>
__device__ __forceinline__ long lin3(const R& r, int x, int y, int z)
{
    return x + (D >= 2 ? (long)y * r.sx : 0) + (D >= 3 ? (long)z * r.sy : 0);
}

// B_c (nodal along the axes other than c) at global coordinates, 0 outside
template <int D, typename T>
__device__ __forceinline__ T load_B(const KV<T>& r, const T *a, int c, int x, int y, int z)
{
    int wx, wy = 0, wz = 0;
    if (!em_coord(r, 0, x, c != 0, wx)) return T(0);
    if (D >= 2 && !em_coord(r, 1, y, c != 1, wy)) return T(0);
    if (D >= 3 && !em_coord(r, 2, z, c != 2, wz)) return T(0);
    return gld(a, lin3<D>(r, wx, wy, wz));
}

// E_c (nodal along c) at global coordinates, 0 outside
template <int D, typename T>
__device__ __forceinline__ T load_E(const KV<T>& r, const T *a, int c, int x, int y, int z)
{
    int wx, wy = 0, wz = 0;
    if (!em_coord(r, 0, x, c == 0, wx)) return T(0);
    if (D >= 2 && !em_coord(r, 1, y, c == 1, wy)) return T(0);
    if (D >= 3 && !em_coord(r, 2, z, c == 2, wz)) return T(0);
    return gld(a, lin3<D>(r, wx, wy, wz));
}

// phi of axion slot L at centre coordinates; axion ghosts one cell outside
// non-periodic faces; 0 elsewhere outside (each axis handled by a constant
// index so that the view stays in registers)
template <int D, typename T>
__device__ __forceinline__ T load_phi(const KV<T>& r, int L, int x, int y, int z)
{
    int v0 = x, v1 = D >= 2 ? y : 0, v2 = D >= 3 ? z : 0;
    int o0 = 0, o1 = 0, o2 = 0;   // -1 / +1: one cell outside the low / high face; 2: further out
    auto chk = [&](int d, int& v, int& o) __attribute__((always_inline)) {
        if (r.axbc[d] == AXF_AX_PERIODIC) {
            v = wrap1(v, r.n[d]);
        } else if (v < 0 || v >= r.n[d]) {
            o = (v == -1) ? -1 : (v == r.n[d] ? 1 : 2);
        }
    };
    chk(0, v0, o0);
    if (D >= 2) chk(1, v1, o1);
    if (D >= 3) chk(2, v2, o2);
    const int nout = (o0 != 0) + (o1 != 0) + (o2 != 0);
    if (nout > 1 || o0 == 2 || o1 == 2 || o2 == 2) return T(0);
    if (o0) return gld(r.face(q_axg(0, o0 < 0 ? 0 : 1, L)), face_index(r, 0, v0, v1, v2));
    if (D >= 2 && o1) return gld(r.face(q_axg(1, o1 < 0 ? 0 : 1, L)), face_index(r, 1, v0, v1, v2));
    if (D >= 3 && o2) return gld(r.face(q_axg(2, o2 < 0 ? 0 : 1, L)), face_index(r, 2, v0, v1, v2));
    return gld(r.arr(q_phi(r.nem, L)), lin3<D>(r, v0, v1, v2));
}

// Address of a B / E / phi point for an unconditional load: the element
// pointer (a valid location of the same array when the point is outside) and
// whether the value is real.  Loading unconditionally and masking at use keeps
// the prefetch loads in flight together instead of waiting on each branch.
template <int D, typename T>
__device__ __forceinline__ const T *addr_em(const KV<T>& r, const T *a, unsigned nodal, int x, int y, int z, bool& ok)
{
    int wx, wy = 0, wz = 0;
    ok = em_coord(r, 0, x, nodal & 1u, wx);
    if (D >= 2) ok = em_coord(r, 1, y, (nodal >> 1) & 1u, wy) && ok;
    if (D >= 3) ok = em_coord(r, 2, z, (nodal >> 2) & 1u, wz) && ok;
    return a + (ok ? lin3<D>(r, wx, wy, wz) : 0);
}

template <int D, typename T>
__device__ __forceinline__ const T *addr_phi(const KV<T>& r, int L, int x, int y, int z, bool& ok)
{
    int v0 = x, v1 = D >= 2 ? y : 0, v2 = D >= 3 ? z : 0;
    int o0 = 0, o1 = 0, o2 = 0;
    auto chk = [&](int d, int& v, int& o) __attribute__((always_inline)) {
        if (r.axbc[d] == AXF_AX_PERIODIC) {
            v = wrap1(v, r.n[d]);
        } else if (v < 0 || v >= r.n[d]) {
            o = (v == -1) ? -1 : (v == r.n[d] ? 1 : 2);
        }
    };
    chk(0, v0, o0);
    if (D >= 2) chk(1, v1, o1);
    if (D >= 3) chk(2, v2, o2);
    const int nout = (o0 != 0) + (o1 != 0) + (o2 != 0);
    ok = !(nout > 1 || o0 == 2 || o1 == 2 || o2 == 2);
    const T *base = r.arr(q_phi(r.nem, L));
    if (!ok) return base;
    if (o0) return r.face(q_axg(0, o0 < 0 ? 0 : 1, L)) + face_index(r, 0, v0, v1, v2);
    if (D >= 2 && o1) return r.face(q_axg(1, o1 < 0 ? 0 : 1, L)) + face_index(r, 1, v0, v1, v2);
    if (D >= 3 && o2) return r.face(q_axg(2, o2 < 0 ? 0 : 1, L)) + face_index(r, 2, v0, v1, v2);
    return base + lin3<D>(r, v0, v1, v2);
}

// First-order Mur update of one tangential E ghost (FP64), the same formula as
// the unfused path, with the laser values from the per-level table
template <typename T>
__device__ __forceinline__ T mur_update(const KV<T>& r, int O, int c, int d, int side, double e_old, double e_new,
                                        double g_old, long fidx, long step)
{
    double ia_o = 0.0, ia_n = 0.0, ig_o = 0.0, ig_n = 0.0;
    if (O == 0 && d == 0 && side == 0 && r.las_on && c == r.las_pol) {
        const long lo = (step % r.inc_k1) * 2 * r.inc_face, ln = ((step + 1) % r.inc_k1) * 2 * r.inc_face;
        ia_o = r.inc[lo + fidx];
        ig_o = r.inc[lo + r.inc_face + fidx];
        ia_n = r.inc[ln + fidx];
        ig_n = r.inc[ln + r.inc_face + fidx];
    }
    double sa_o = e_old - ia_o, sa_n = e_new - ia_n, sg_o = g_old - ig_o;
    double sg_n = sa_o + r.murc[d] * (sa_n - sg_o);
    return (T)(sg_n + ig_n);
}

// ------------------------------------------------------------------ kernel

template <int D, int TX, int TY, typename T>
__global__ void __launch_bounds__((FK<D, TX, TY, T>::NT))
k_fused(const RunK<T> *__restrict__ rp, long step, int ntx, int nty, int nch, int chunk)
{
    using K = FK<D, TX, TY, T>;
    using S = FusedStep<D, TX, TY, T>;
    using Wn = Win<D, TX, TY, T>;
    constexpr int M = K::M;
    KV<T> r = make_kv(rp);

    // XCD-aware tile order: consecutive workgroups land on different XCDs, so
    // hand each XCD a contiguous run of tiles (neighbours share its L2)
    const int L = (int)xcd_band(blockIdx.x, (long)ntx * nty * nch);
    const int tx = L % ntx, ty = (L / ntx) % nty, ch = L / (ntx * nty);

    const int so = em_slot(step, r.nem), sn = em_slot(step + 1, r.nem);
    const int la = phi_slot(step, r.nph), lb = phi_slot(step + 1, r.nph), ln = phi_slot(step + 2, r.nph);

    // in-plane tile and ownership ranges (the last tile also owns the nodal plane n)
    const int x0 = tx * TX, y0 = ty * TY;
    const int own_x_hi = (tx == ntx - 1) ? r.nn[0] : x0 + TX;
    const int own_y_hi = D == 3 ? ((ty == nty - 1) ? r.nn[1] : y0 + TY) : 1;
    const int c0 = ch * chunk, c1 = (ch == nch - 1) ? r.nn[M] : c0 + chunk;

    const int tid = threadIdx.x;
    const bool live = tid < K::R;
    const int lx = tid % K::RX, ly = tid / K::RX;
    const int rx = lx - 3, ry = D == 3 ? ly - 3 : 0;       // offsets from the tile origin
    const int gx = x0 + rx, gy = D == 3 ? y0 + ry : 0;     // global in-plane coordinates
    const Wn w{live ? tid : 0};

    auto in_rng = [&](int lo, int hi) __attribute__((always_inline)) {
        bool ok = live && rx >= lo && rx < hi;
        if (D == 3) ok = ok && ry >= lo && ry < hi;
        return ok;
    };
    // stage regions (offsets from the tile origin, per in-plane axis)
    const bool rS1 = in_rng(-2, TX + 2), rS2 = in_rng(-2, TX + 1), rS3 = in_rng(0, TX + 2);
    const bool rS4 = in_rng(-1, TX + 1), rS56 = in_rng(0, TX + 1);
    const bool own_inplane = live && gx >= x0 && gx < own_x_hi && (D == 2 || (gy >= y0 && gy < own_y_hi));

    // global coordinates of this thread's point at plane p
    auto X = [&](int p) __attribute__((always_inline)) { return gx; };
    auto Y = [&](int p) __attribute__((always_inline)) { return D == 3 ? gy : p; };
    auto Z = [&](int p) __attribute__((always_inline)) { return D == 3 ? p : 0; };
    // is the point (at plane p) inside the extent of a component nodal along the
    // axes in `nodal` (bit mask)?  periodic axes always are
    auto valid = [&](int p, unsigned nodal) __attribute__((always_inline)) {
        bool ok = true;
        int v[3] = {X(p), Y(p), Z(p)};
#pragma unroll
        for (int d = 0; d < D; d++) {
            if (!r.mur[d]) continue;
            int ext = (nodal >> d & 1) ? r.nn[d] : r.n[d];
            ok = ok && v[d] >= 0 && v[d] < ext;
        }
        return ok;
    };
    auto own_plane = [&](int p) __attribute__((always_inline)) { return p >= c0 && p < c1; };
    auto gindex = [&](int p) __attribute__((always_inline)) {
        int vx = X(p), vy = Y(p), vz = Z(p);
        if (!r.mur[0]) vx = wrap1(vx, r.n[0]);
        if (D >= 2 && !r.mur[1]) vy = wrap1(vy, r.n[1]);
        if (D >= 3 && !r.mur[2]) vz = wrap1(vz, r.n[2]);
        return lin3<D>(r, vx, vy, vz);
    };

    // ---- prefetch registers for one iteration: raw loads plus validity masks
    T pf_b0[3], pf_b1[3], pf_pa, pf_pb, pf_e0m[3], pf_e1m[3];
    unsigned pf_mask = 0;
    T cur_e0m[3], cur_e1m[3];
    auto prefetch = [&](int t) __attribute__((always_inline)) {
        if (!live) return;
        unsigned m = 0;
        bool ok;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            if (!actB0<D>(c)) { pf_b0[c] = T(0); continue; }
            const T *p = addr_em<D>(r, r.arr(q_em(1, so, c)), 7u & ~(1u << c), X(t), Y(t), Z(t), ok);
            pf_b0[c] = gld(p, 0);
            m |= ok ? 1u << c : 0u;
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const T *p = addr_em<D>(r, r.arr(q_em(3, so, c)), 7u & ~(1u << c), X(t - 1), Y(t - 1), Z(t - 1), ok);
            pf_b1[c] = gld(p, 0);
            m |= ok ? 8u << c : 0u;
        }
        {
            const T *p = addr_phi<D>(r, la, X(t - 1), Y(t - 1), Z(t - 1), ok);
            pf_pa = gld(p, 0);
            m |= ok ? 64u : 0u;
            p = addr_phi<D>(r, lb, X(t - 1), Y(t - 1), Z(t - 1), ok);
            pf_pb = gld(p, 0);
            m |= ok ? 128u : 0u;
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            if (!actE0<D>(c)) { pf_e0m[c] = T(0); continue; }
            const T *p = addr_em<D>(r, r.arr(q_em(0, so, c)), 1u << c, X(t - 1), Y(t - 1), Z(t - 1), ok);
            pf_e0m[c] = gld(p, 0);
            m |= (ok && rS1) ? 256u << c : 0u;
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const T *p = addr_em<D>(r, r.arr(q_em(2, so, c)), 1u << c, X(t - 2), Y(t - 2), Z(t - 2), ok);
            pf_e1m[c] = gld(p, 0);
            m |= (ok && rS4) ? 2048u << c : 0u;
        }
        pf_mask = m;
    };
    auto sel = [&](T v, unsigned bit) __attribute__((always_inline)) { return (pf_mask & bit) ? v : T(0); };

    // Mur ghost of E_c of order O at this thread's point of plane pg, across axis
    // d (side 0 at coordinate -1, side 1 at n): from the adjacent interior point
    // (offset (o0,o1,o2), at plane pa in the window) and the old state in HBM
    auto mur_ghost = [&](auto Oc, int c, int d, int side, int pg, int pa, int o0, int o1, int o2, bool write_hist) __attribute__((always_inline)) -> T {
        constexpr int O = decltype(Oc)::value;
        int a0 = X(pg) + o0, a1 = Y(pg) + o1, a2 = Z(pg) + o2;
        if (!r.mur[0]) a0 = wrap1(a0, r.n[0]);
        if (D >= 2 && !r.mur[1]) a1 = wrap1(a1, r.n[1]);
        if (D >= 3 && !r.mur[2]) a2 = wrap1(a2, r.n[2]);
        long fidx = face_index(r, d, a0, a1, a2);
        double e_old = (double)gld(r.arr(q_em(O == 0 ? 0 : 2, so, c)), lin3<D>(r, a0, a1, a2));
        const int i0 = M == 0 ? 0 : o0, i1 = M == 1 ? 0 : o1, i2 = M == 2 ? 0 : o2;
        double e_new = (double)(O == 0 ? w.at(S::bE0H(c), K::W2, pa, i0, i1, i2) : w.at(S::bE1H(c), K::W2, pa, i0, i1, i2));
        double g_old = (double)gld(r.face(q_mur(O, d, side, c, so)), fidx);
        T val = mur_update<T>(r, O, c, d, side, e_old, e_new, g_old, fidx, step);
        if (write_hist) gst(r.wface(q_mur(O, d, side, c, sn)), fidx, val);
        return val;
    };

    // Mur ghosts of order O once E^{n+1/2} of plane p is in its window: ghosts
    // across in-plane axes at plane p; on a Mur march axis the ghost plane -1
    // (while plane 0 is done) and the ghost plane n (from plane n - 1)
    auto ghost_fix = [&](auto Oc, int p) __attribute__((always_inline)) {
        constexpr int O = decltype(Oc)::value;
        if (!(O == 0 ? rS1 : rS4)) return;
        const int v[3] = {X(p), Y(p), Z(p)};
#pragma unroll
        for (int c = 0; c < 3; c++) {
            if (!actE<D, O>(c)) continue;
            const int base = O == 0 ? S::bE0H(c) : S::bE1H(c);
#pragma unroll
            for (int d = 0; d < D; d++) {
                if (d == M || d == c || !r.mur[d]) continue;
                int side = v[d] == -1 ? 0 : (v[d] == r.n[d] ? 1 : -1);
                if (side < 0) continue;
                bool ok = true;
#pragma unroll
                for (int e = 0; e < D; e++) {
                    if (e == d || !r.mur[e]) continue;
                    int ext = (e == c) ? r.nn[e] : r.n[e];
                    ok = ok && v[e] >= 0 && v[e] < ext;
                }
                if (!ok) continue;
                const int sg = side == 0 ? 1 : -1;
                const int ax = d == 0 ? gx + sg : gx, ay = (D == 3 && d == 1) ? gy + sg : gy;
                const bool owner = own_plane(p) && ax >= x0 && ax < own_x_hi && (D == 2 || (ay >= y0 && ay < own_y_hi));
                T val = mur_ghost(Oc, c, d, side, p, p, d == 0 ? sg : 0, d == 1 ? sg : 0, d == 2 ? sg : 0, owner);
                w.ref(base, K::W2, p) = val;
            }
            if (c != M && r.mur[M]) {
                int side = -1, pg = 0, pad = 0;
                if (p == 0) { side = 0; pg = -1; pad = 0; }
                else if (p == r.n[M]) { side = 1; pg = p; pad = p - 1; }
                if (side >= 0) {
                    bool ok = true;
#pragma unroll
                    for (int e = 0; e < D; e++) {
                        if (e == M || !r.mur[e]) continue;
                        int ext = (e == c) ? r.nn[e] : r.n[e];
                        ok = ok && v[e] >= 0 && v[e] < ext;
                    }
                    if (ok) {
                        // the top ghost is owned by the chunk owning the nodal plane n[M]:
                        // only the last chunk marches the first-order plane that far
                        const bool owner = own_inplane && own_plane(side == 1 ? p : pad);
                        const int dm = pad - pg;
                        T val = mur_ghost(Oc, c, M, side, pg, pad, M == 0 ? dm : 0, M == 1 ? dm : 0, M == 2 ? dm : 0, owner);
                        w.ref(base, K::W2, pg) = val;
                    }
                }
            }
        }
    };

    // ---- the march
    const int t_first = c0 - 2, t_last = c1 + 1;
    prefetch(t_first);
    for (int t = t_first; t <= t_last; t++) {
        // keep the array strides opaque to loop-invariant code motion: array
        // addresses are then formed per access from two scalar registers instead
        // of being hoisted into dozens of live 64-bit values
        asm volatile("" : "+s"(r.as), "+s"(r.fs));
        __syncthreads();   // previous iteration done with the slots about to be reused
        if (live) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                if (actB0<D>(c)) w.ref(S::bB0N(c), K::W_B0N, t) = sel(pf_b0[c], 1u << c);
                w.ref(S::bB1N(c), K::W_B1N, t - 1) = sel(pf_b1[c], 8u << c);
                cur_e0m[c] = sel(pf_e0m[c], 256u << c);
                cur_e1m[c] = sel(pf_e1m[c], 2048u << c);
            }
            w.ref(K::oPHA, K::W_PH, t - 1) = sel(pf_pa, 64u);
            w.ref(K::oPHB, K::W_PH, t - 1) = sel(pf_pb, 128u);
        }
        if (t < t_last) prefetch(t + 1);
        __syncthreads();

        // S1: E0^{n+1/2} and E0^n at plane p1 = t - 1
        const int p1 = t - 1;
        if (rS1) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                if (!actE0<D>(c)) continue;
                T eh = T(0), en = T(0);
                if (valid(p1, 1u << c)) {
                    T rhs = S::template curlB<0>(r, w, c, p1);
                    eh = cur_e0m[c] + T(1) * rhs;
                    en = r.half * (cur_e0m[c] + eh);
                    if (own_inplane && own_plane(p1)) gst(r.warr(q_em(0, sn, c)), gindex(p1), eh);
                }
                w.ref(S::bE0H(c), K::W2, p1) = eh;
                w.ref(S::bE0N(c), K::W2, p1) = en;
            }
        }
        __syncthreads();
        ghost_fix(std::integral_constant<int, 0>{}, p1);
        __syncthreads();

        // S2: C^n at the centres of plane p2 = t - 2;  S3: B0^{n+1} at plane p1
        const int p2 = t - 2;
        if (rS2) {
            T C0 = T(0), C1 = T(0), C2 = T(0);
            if (valid(p2, 0u)) {
                T e[3], bb[3], gp[3] = {T(0), T(0), T(0)};
                const int cxg = wrap1(X(p2), r.n[0]);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    e[c] = T(0);
                    if (actE0<D>(c)) {
                        T lo = w.at(S::bE0N(c), K::W2, p2, 0, 0, 0);
                        T hi = w.at(S::bE0N(c), K::W2, p2, OFF(c, 1));
                        e[c] = c < D ? r.half * (lo + hi) : lo;
                    }
                    bb[c] = S::template centreB<0>(w, S::bB0N(c), K::W_B0N, c, p2) + bext_at(r, c, cxg);
                }
                T pa0 = w.at(K::oPHA, K::W_PH, p2, 0, 0, 0), pb0 = w.at(K::oPHB, K::W_PH, p2, 0, 0, 0);
                T dtphi = (pb0 - pa0) * r.inv_dt;
#pragma unroll
                for (int d = 0; d < D; d++) {
                    T up = r.half * (w.at(K::oPHA, K::W_PH, p2, OFF(d, 1)) + w.at(K::oPHB, K::W_PH, p2, OFF(d, 1)));
                    T dn = r.half * (w.at(K::oPHA, K::W_PH, p2, OFF(d, -1)) + w.at(K::oPHB, K::W_PH, p2, OFF(d, -1)));
                    gp[d] = (up - dn) * r.inv2dx[d];
                }
                C0 = dtphi * bb[0] - (e[1] * gp[2] - e[2] * gp[1]);
                C1 = dtphi * bb[1] - (e[2] * gp[0] - e[0] * gp[2]);
                C2 = dtphi * bb[2] - (e[0] * gp[1] - e[1] * gp[0]);
            }
            w.ref(S::bC(0), K::W2, p2) = C0;
            w.ref(S::bC(1), K::W2, p2) = C1;
            w.ref(S::bC(2), K::W2, p2) = C2;
        }
        if (rS3) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                if (!actB0<D>(c)) continue;
                T v = T(0);
                if (valid(p1, 7u & ~(1u << c))) {
                    v = w.at(S::bB0N(c), K::W_B0N, p1, 0, 0, 0) - S::template curlE<0>(r, w, c, p1);
                    if (own_inplane && own_plane(p1)) gst(r.warr(q_em(1, sn, c)), gindex(p1), v);
                }
                w.ref(S::bB0P(c), K::W2, p1) = v;
            }
        }
        __syncthreads();

        // S4: E1^{n+1/2} at plane p2
        if (rS4) {
            const int v[3] = {X(p2), Y(p2), Z(p2)};
#pragma unroll
            for (int c = 0; c < 3; c++) {
                T val = T(0);
                if (valid(p2, 1u << c)) {
                    T Sc;
                    if (c >= D) {
                        Sc = w.at(S::bC(c), K::W2, p2, 0, 0, 0);
                    } else {
                        int lo = -1, hi = 0;
                        if (r.mur[c]) {
                            if (v[c] - 1 < 0) lo = 0;
                            if (v[c] > r.n[c] - 1) hi = -1;
                        }
                        Sc = r.half * (w.at(S::bC(c), K::W2, p2, OFF(c, lo)) + w.at(S::bC(c), K::W2, p2, OFF(c, hi)));
                    }
                    T rhs = S::template curlB<1>(r, w, c, p2) - r.cg1 * Sc;
                    val = cur_e1m[c] + T(1) * rhs;
                    if (own_inplane && own_plane(p2)) gst(r.warr(q_em(2, sn, c)), gindex(p2), val);
                }
                w.ref(S::bE1H(c), K::W2, p2) = val;
            }
        }
        __syncthreads();
        ghost_fix(std::integral_constant<int, 1>{}, p2);
        __syncthreads();

        // S5: B1^{n+1} and S6: phi^{n+3/2} at plane p2 (stored directly)
        if (rS56 && own_inplane && own_plane(p2)) {
            const long gi2 = gindex(p2);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                if (!valid(p2, 7u & ~(1u << c))) continue;
                gst(r.warr(q_em(3, sn, c)), gi2, w.at(S::bB1N(c), K::W_B1N, p2, 0, 0, 0) - S::template curlE<1>(r, w, c, p2));
            }
            if (valid(p2, 0u)) {
                const int gi = wrap1(X(p2), r.n[0]);
                const int gj = D >= 2 ? wrap1(Y(p2), r.n[1]) : 0;
                const int gk = D >= 3 ? wrap1(Z(p2), r.n[2]) : 0;
                T e[3], bb[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    e[c] = T(0);
                    if (actE0<D>(c)) {
                        T q0 = w.at(S::bE0H(c), K::W2, p2, 0, 0, 0);
                        e[c] = c < D ? r.half * (q0 + w.at(S::bE0H(c), K::W2, p2, OFF(c, 1))) : q0;
                    }
                    T bo = S::template centreB<0>(w, S::bB0N(c), K::W_B0N, c, p2);
                    T bn = S::template centreB<0>(w, S::bB0P(c), K::W2, c, p2);
                    bb[c] = r.half * (bo + bn) + bext_at(r, c, gi);
                }
                T sax = r.gax * (e[0] * bb[0] + e[1] * bb[1] + e[2] * bb[2]);
                T pa = w.at(K::oPHA, K::W_PH, p2, 0, 0, 0), pb = w.at(K::oPHB, K::W_PH, p2, 0, 0, 0);
                T lap = T(0);
#pragma unroll
                for (int d = 0; d < D; d++)
                    lap += ((w.at(K::oPHB, K::W_PH, p2, OFF(d, 1)) - T(2) * pb) + w.at(K::oPHB, K::W_PH, p2, OFF(d, -1)))
                           * r.inv_dx2[d];
                T sdt = pml_sdt<D>(r, gi, gj, gk);
                T x = r.dt2 * ((sax - r.m2 * pb) + lap) - sdt * sdt * pb;
                // outside the damping layer the divisor is exactly 1: skip the division
    T pn = ((x + sdt * pa) + T(2) * pb) - pa;
    if (sdt != T(0)) pn = pn / (T(1) + sdt);
                gst(r.warr(q_phi(r.nem, ln)), gi2, pn);
                const int gv[3] = {gi, gj, gk};
#pragma unroll
                for (int d = 0; d < D; d++) {
                    if (r.axbc[d] == AXF_AX_PERIODIC) continue;
#pragma unroll
                    for (int side = 0; side < 2; side++) {
                        if (gv[d] != (side ? r.n[d] - 1 : 0)) continue;
                        long f = face_index(r, d, gi, gj, gk);
                        T gval;
                        if (r.axbc[d] == AXF_AX_OUTFLOW) {
                            T gbv = gld(r.face(q_axg(d, side, lb)), f), gav = gld(r.face(q_axg(d, side, la)), f), rr = r.out_r[d];
                            T xx = (((T(-2) * gbv + T(2) * gav) - r.dt2 * (sax - r.m2 * gbv)) + rr * pb - rr * rr * (pb - T(2) * gbv))
                                   / (rr + rr * rr);
                            gval = gav + rr * (pb - xx);
                        } else {
                            gval = pn;
                        }
                        gst(r.wface(q_axg(d, side, ln)), f, gval);
                    }
                }
            }
        }
    }
}

// ====================================================================== 2D
// Fused 2D step without LDS or barriers: one wavefront owns 64 consecutive x
// columns (59 outputs: 3 halo columns on the low side, 2 on the high side) and
// marches along y through a chunk of rows.  x neighbours come from the
// neighbouring lane (DPP wavefront shifts), y history stays in registers of the
// own lane, so every value of a row is computed once per wavefront.  The point
// formulas and their operation order are those of the unfused kernels.

__device__ __forceinline__ float lane_up(float v)    // value of lane + 1 (0 in the last lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_dn(float v)    // value of lane - 1 (0 in lane 0)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_up(double v)
{
    long long b = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x130, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_dn(double v)
{
    long long b = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x138, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

constexpr int kWaveOut = 59;   // output columns per wavefront (one step per pass)
// prefetch distance (rows ahead) of the interior march, by precision (measured)
template <typename T> struct WavePD { static constexpr int value = sizeof(T) == 8 ? 2 : 3; };

// global load / store at a 32-bit byte offset from a wave-uniform base (every
// array of a run has the same layout, so one offset per row serves them all)
template <typename T>
__device__ __forceinline__ T ldo(const T *base, unsigned boff)
{
    return *(const __attribute__((address_space(1))) T *)((const __attribute__((address_space(1))) char *)base + boff);
}
template <typename T>
__device__ __forceinline__ void sto(T *base, unsigned boff, T v)
{
    *(__attribute__((address_space(1))) T *)((__attribute__((address_space(1))) char *)base + boff) = v;
}

// What the interior of the 2D march needs in registers: the field base and
// stride, the grid and the coefficients.  Everything used only at the domain
// boundary (ghost planes, Mur, laser, PML, outflow) is read from the run
// descriptor where it is needed, so that it does not occupy scalar registers
// for the whole march.
template <typename T>
struct KW {
    const char *sb;
    unsigned as;            // array stride in bytes (12 arrays span < 4 GiB: checked on the host)
    int n[2], nn[2], mur[2], axbc[2];
    int sx;
    T cdt[2], half, inv_dt, inv2dx[2], inv_dx2[2], dt2, m2, gax, cg1;

    __device__ __forceinline__ const T *arr(int q) const { return (const T *)(sb + (size_t)q * as); }
    __device__ __forceinline__ T *warr(int q) const { return (T *)(sb + (size_t)q * as); }
};

template <typename T>
__device__ __forceinline__ KW<T> make_kw(const RunK<T> *__restrict__ rp)
{
    KW<T> v;
    v.sb = rp->state_base;
    v.as = (unsigned)rp->arr_stride;
#pragma unroll
    for (int d = 0; d < 2; d++) {
        v.n[d] = rp->n[d];
        v.nn[d] = rp->nn[d];
        v.mur[d] = rp->mur[d];
        v.axbc[d] = rp->axbc[d];
        v.cdt[d] = rp->cdt[d];
        v.inv2dx[d] = rp->inv2dx[d];
        v.inv_dx2[d] = rp->inv_dx2[d];
    }
    v.sx = (int)rp->sx;
    v.half = rp->half;
    v.inv_dt = rp->inv_dt;
    v.dt2 = rp->dt2;
    v.m2 = rp->m2;
    v.gax = rp->gax;
    v.cg1 = rp->cg1;
    return v;
}

// boundary planes of a run (read from the descriptor at the boundary only)
template <typename T>
__device__ __forceinline__ T *face_of(const RunK<T> *rp, int q) { return (T *)(rp->face_base + q * rp->face_stride); }

// The wavefront of x segment `seg` and row chunk `ch` of one run's step.
// INTERIOR: the wavefront's columns and rows (its halo included) keep clear of
// every face, ghost ring and damping layer, so every point is valid, nothing
// wraps and there are no ghosts to read or write; the point formulas are the
// same, so both variants produce the same bits.
template <typename T, bool INTERIOR, int PD>
__device__ __forceinline__ void wave2d_body(const RunK<T> *__restrict__ rp, long step, int seg, int ch, int nch, int chunk,
                                            int wid = kWaveOut)
{
    KW<T> r = make_kw(rp);
    const int lane = threadIdx.x & 63;
    // (the wavefront kernels advance 2D runs only, which keep kEmSlots E/B
    // slots and kPhiSlots axion slots)
    const int so = em_slot(step, kEmSlots), sn = em_slot(step + 1, kEmSlots);
    const int la = phi_slot(step, kPhiSlots), lb = phi_slot(step + 1, kPhiSlots), ln = phi_slot(step + 2, kPhiSlots);

    const int x0 = seg * wid, gx = x0 - 3 + lane;
    const int own_x_hi = min(x0 + wid, r.nn[0]);
    const bool own_x = lane >= 3 && lane < 3 + wid && gx < own_x_hi;
    const int c0 = ch * chunk, c1 = (ch == nch - 1) ? r.nn[1] : c0 + chunk;
    const int n0 = r.n[0], n1 = r.n[1], nn0 = r.nn[0], nn1 = r.nn[1];
    const bool mx = INTERIOR ? false : r.mur[0], my = INTERIOR ? false : r.mur[1];
    const unsigned es = sizeof(T), sxb = (unsigned)r.sx * es;   // element and row pitch in bytes
    // this lane's column: x validity of nodal / centred EM points (fixed for the
    // march) and the storage column read for them (any valid one when masked)
    const bool inx_n = gx >= 0 && gx < nn0, inx_c = gx >= 0 && gx < n0;
    const bool vx_nod = !mx || inx_n;
    const bool vx_cen = !mx || inx_c;
    const unsigned bx = (unsigned)(mx ? (inx_n ? gx : 0) : wrap1(gx, n0)) * es;
    // the same for phi: wrapped on a periodic axion axis, else the interior or
    // the ghost column one cell outside either face
    const bool axpx = INTERIOR || r.axbc[0] == AXF_AX_PERIODIC, axpy = INTERIOR || r.axbc[1] == AXF_AX_PERIODIC;
    const int xgs = axpx ? -1 : (gx == -1 ? 0 : (gx == n0 ? 1 : -1));
    const bool vpx = axpx || inx_c || xgs >= 0;          // phi exists at this column
    const bool vpx_in = axpx || inx_c;                   // ... and is not a ghost
    const unsigned bxp = (unsigned)(axpx ? wrap1(gx, n0) : (inx_c ? gx : 0)) * es;
    // plane p (wave-uniform): y validity and storage row
    auto vy_nod = [&](int p) __attribute__((always_inline)) { return !my || (p >= 0 && p < nn1); };
    auto vy_cen = [&](int p) __attribute__((always_inline)) { return !my || (p >= 0 && p < n1); };
    auto own_plane = [&](int p) __attribute__((always_inline)) { return p >= c0 && p < c1; };
    // every field array is addressed from one of three wave-uniform bases (the
    // EM slot read, the EM slot written, the axion levels) with a 32-bit byte
    // offset index * as + (row, column); the stride is re-read each iteration
    // (opaque to the compiler) so that the per-array products stay in the loop
    // instead of occupying 22 scalar register pairs for the whole march
    unsigned as_l = r.as;
    const char *const b_rd = r.sb + (size_t)q_em(0, so, 0) * r.as;
    const char *const b_wr = r.sb + (size_t)q_em(0, sn, 0) * r.as;
    const char *const b_ph = r.sb + (size_t)q_phi(kEmSlots, 0) * r.as;
    auto lde = [&](int kind, int c, unsigned o) __attribute__((always_inline)) -> T {
        return ldo((const T *)b_rd, (unsigned)(kind * 3 + c) * as_l + o);
    };
    auto ste = [&](int kind, int c, unsigned o, T v) __attribute__((always_inline)) {
        sto((T *)b_wr, (unsigned)(kind * 3 + c) * as_l + o, v);
    };
    auto ldp = [&](int L, unsigned o) __attribute__((always_inline)) -> T { return ldo((const T *)b_ph, (unsigned)L * as_l + o); };
    auto stp = [&](int L, unsigned o, T v) __attribute__((always_inline)) { sto((T *)b_ph, (unsigned)L * as_l + o, v); };
    auto off = [&](int p) __attribute__((always_inline)) -> unsigned {
        const int row = my ? ((p >= 0 && p < nn1) ? p : 0) : wrap1(p, n1);
        return bx + (unsigned)row * sxb;
    };

    // register windows along y (suffix = planes behind the newest loaded plane t)
    T b0z_2 = 0, b0z_1 = 0, b0z_0 = 0;
    T pa_3 = 0, pa_2 = 0, pa_1 = 0, pb_3 = 0, pb_2 = 0, pb_1 = 0;
    T b1_2[3] = {0, 0, 0}, b1_1[3] = {0, 0, 0};
    T e0h_2[2] = {0, 0}, e0h_1[2] = {0, 0}, e0n_2[2] = {0, 0}, e0n_1[2] = {0, 0};
    T c_3[3] = {0, 0, 0}, c_2[3] = {0, 0, 0};
    T b0p_2 = 0, b0p_1 = 0;
    T e1h_3[3] = {0, 0, 0}, e1h_2[3] = {0, 0, 0};
    // prefetched raw values of plane t (and t-1, t-2) and the wave-uniform y
    // validity they were loaded with, PD iterations ahead of their use; the
    // lane masks are applied at use, so that the loads stay in flight together
    struct Pref {
        T b0z, b1[3], pa, pb, e0m[2], e1m[3];
        bool yn0, yn1, yc1, yn2, yc2, pin, pgh;
    };
    Pref buf[PD];
    auto load_phi = [&](int L, int p) __attribute__((always_inline)) -> T {
        const int ys = axpy ? -1 : (p == -1 ? 0 : (p == n1 ? 1 : -1));
        if (ys >= 0) return ldo((const T *)face_of(rp, q_axg(1, ys, L)), bxp);   // the y ghost row (uniform)
        const int row = axpy ? wrap1(p, n1) : ((p >= 0 && p < n1) ? p : 0);
        if (xgs >= 0) return ldo((const T *)face_of(rp, q_axg(0, xgs, L)), (unsigned)row * es);   // x ghost lanes
        return ldp(L, bxp + (unsigned)row * sxb);
    };
    // Rows below the chunk feed the owned rows only through: B0z from row c0-2,
    // phi from c0-3, E0 from c0-2, B1 from c0-1, E1 from c0-1 (the first owned
    // row c0 needs E1 and B1 one row down, C two rows down, E0^n and B0 along
    // with C, phi one row below that).  Older rows of a field are not loaded.
    auto prefetch = [&](int t, Pref& P) __attribute__((always_inline)) {
        const unsigned o0 = off(t), o1 = off(t - 1), o2 = off(t - 2);
        P.b0z = lde(1, 2, o0);
#pragma unroll
        for (int c = 0; c < 3; c++) P.b1[c] = t - 1 >= c0 - 1 ? lde(3, c, o1) : T(0);
        P.pa = load_phi(la, t - 1);
        P.pb = load_phi(lb, t - 1);
#pragma unroll
        for (int c = 0; c < 2; c++) P.e0m[c] = t - 1 >= c0 - 2 ? lde(0, c, o1) : T(0);
#pragma unroll
        for (int c = 0; c < 3; c++) P.e1m[c] = t - 2 >= c0 - 1 ? lde(2, c, o2) : T(0);
        P.yn0 = vy_nod(t);
        P.yn1 = vy_nod(t - 1);
        P.yc1 = vy_cen(t - 1);
        P.yn2 = vy_nod(t - 2);
        P.yc2 = vy_cen(t - 2);
        const int p = t - 1;
        P.pgh = !axpy && (p == -1 || p == n1);
        P.pin = axpy || (p >= 0 && p < n1);
    };

    // Mur ghost of E_c (order O) of this lane at plane pg from the adjacent
    // interior point (x offset ox, plane pa) whose E^{n+1/2} is e_new
    auto ghost = [&](int O, int c, int d, int side, int pg, int ox, int pa, T e_new, bool owner) __attribute__((always_inline)) -> T {
        int a0 = gx + ox, a1 = pa;
        if (!mx) a0 = wrap1(a0, n0);
        if (!my) a1 = wrap1(a1, n1);
        long fidx = face_index(r, d, a0, a1, 0);
        double e_old = (double)gld(r.arr(q_em(O == 0 ? 0 : 2, so, c)), (long)a0 + (long)a1 * r.sx);
        double g_old = (double)gld((const T *)face_of(rp, q_mur(O, d, side, c, so)), fidx);
        T val = mur_update_rk<T>(*rp, O, c, d, side, e_old, (double)e_new, g_old, fidx, step);
        if (owner) gst(face_of(rp, q_mur(O, d, side, c, sn)), fidx, val);
        return val;
    };

    const T bext0 = bext_at(*rp, 0, wrap1(gx, n0)), bext1 = bext_at(*rp, 1, wrap1(gx, n0));
    const T bext2 = bext_at(*rp, 2, wrap1(gx, n0));
    const int t_first = c0 - 2, t_last = c1 + 1;
#pragma unroll
    for (int k = 0; k < PD; k++)
        if (t_first + k <= t_last) prefetch(t_first + k, buf[k]);
    // the march, unrolled by a multiple of the prefetch distance and of the
    // window lengths (2 and 3) so that every buffer and window has a fixed
    // register home across the unrolled block
    constexpr int U = PD == 1 ? 1 : 6;
    for (int t0 = t_first; t0 <= t_last; t0 += U)
#pragma unroll
    for (int k = 0; k < U; k++) {
        const int t = t0 + k;
        if (t > t_last) break;
        Pref& P = buf[k % PD];
        asm volatile("" : "+s"(as_l));
        // rotate the windows and take in the prefetched planes
        b0z_2 = b0z_1; b0z_1 = b0z_0; b0z_0 = (vx_nod && P.yn0) ? P.b0z : T(0);
        const bool pok = P.pgh ? vpx_in : (vpx && P.pin);
        pa_3 = pa_2; pa_2 = pa_1; pa_1 = pok ? P.pa : T(0);
        pb_3 = pb_2; pb_2 = pb_1; pb_1 = pok ? P.pb : T(0);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            b1_2[c] = b1_1[c];
            c_3[c] = c_2[c];
            e1h_3[c] = e1h_2[c];
        }
        b1_1[0] = (vx_cen && P.yn1) ? P.b1[0] : T(0);   // B1x: centred x, nodal y
        b1_1[1] = (vx_nod && P.yc1) ? P.b1[1] : T(0);   // B1y: nodal x, centred y
        b1_1[2] = (vx_nod && P.yn1) ? P.b1[2] : T(0);   // B1z: nodal x, nodal y
#pragma unroll
        for (int c = 0; c < 2; c++) {
            e0h_2[c] = e0h_1[c];
            e0n_2[c] = e0n_1[c];
        }
        b0p_2 = b0p_1;
        const T e0m[2] = {(vx_nod && P.yc1) ? P.e0m[0] : T(0), (vx_cen && P.yn1) ? P.e0m[1] : T(0)};
        const T e1m[3] = {(vx_nod && P.yc2) ? P.e1m[0] : T(0), (vx_cen && P.yn2) ? P.e1m[1] : T(0),
                          (vx_cen && P.yc2) ? P.e1m[2] : T(0)};
        if (t + PD <= t_last) prefetch(t + PD, P);

        const int p1 = t - 1, p2 = t - 2;
        const unsigned o1 = off(p1), o2 = off(p2);
        // ---- S1: E0^{n+1/2}, E0^n at plane p1 (E0x nodal in x, E0y nodal in y)
        {
            const T up_b0z = lane_up(b0z_1);
            T eh[2] = {T(0), T(0)}, en[2] = {T(0), T(0)};
            if (vx_nod && vy_cen(p1)) {
                T a = r.cdt[1] * (b0z_0 - b0z_1), b = T(0);
                T rhs = a - b;
                eh[0] = e0m[0] + T(1) * rhs;
                en[0] = r.half * (e0m[0] + eh[0]);
            }
            if (vx_cen && vy_nod(p1)) {
                T a = T(0), b = r.cdt[0] * (up_b0z - b0z_1);
                T rhs = a - b;
                eh[1] = e0m[1] + T(1) * rhs;
                en[1] = r.half * (e0m[1] + eh[1]);
            }
            e0h_1[0] = eh[0]; e0h_1[1] = eh[1];
            e0n_1[0] = en[0]; e0n_1[1] = en[1];
            const bool own = own_x && own_plane(p1);
            if (own && vx_nod && vy_cen(p1)) ste(0, 0, o1, eh[0]);
            if (own && vx_cen && vy_nod(p1)) ste(0, 1, o1, eh[1]);
            // Mur ghosts of E0y across x (E0y centred in x)
            const T up_e = lane_up(e0h_1[1]), dn_e = lane_dn(e0h_1[1]);
            if (mx && (gx == -1 || gx == n0) && vy_nod(p1)) {
                const int side = gx == -1 ? 0 : 1, ox = side ? -1 : 1;
                const bool owner = own_plane(p1) && lane + ox >= 3 && lane + ox < 3 + wid && gx + ox < own_x_hi;
                e0h_1[1] = ghost(0, 1, 0, side, p1, ox, p1, side ? dn_e : up_e, owner);
            }
            // Mur ghosts of E0x across y (E0x centred in y): plane -1 from plane 0, plane n1 from n1 - 1
            if (my && vx_nod) {
                if (p1 == 0) e0h_2[0] = ghost(0, 0, 1, 0, -1, 0, 0, e0h_1[0], own_x && own_plane(0));
                else if (p1 == n1) e0h_1[0] = ghost(0, 0, 1, 1, n1, 0, n1 - 1, e0h_2[0], own_x && own_plane(n1 - 1));
            }
        }
        // ---- S2: C^n at the centres of plane p2
        {
            T e[3], bb[3], gp[3];
            const T up_en0 = lane_up(e0n_2[0]);
            const T up_b2 = lane_up(b0z_2), up_b1 = lane_up(b0z_1);
            const T up_pa = lane_up(pa_2), up_pb = lane_up(pb_2), dn_pa = lane_dn(pa_2), dn_pb = lane_dn(pb_2);
            T C0 = T(0), C1 = T(0), C2 = T(0);
            if (vx_cen && vy_cen(p2)) {
                e[0] = r.half * (e0n_2[0] + up_en0);
                e[1] = r.half * (e0n_2[1] + e0n_1[1]);
                e[2] = T(0);
                bb[0] = T(0) + bext0;
                bb[1] = T(0) + bext1;
                bb[2] = T(0.25) * ((b0z_2 + up_b2) + (b0z_1 + up_b1)) + bext2;
                T dtphi = (pb_2 - pa_2) * r.inv_dt;
                {
                    T up = r.half * (up_pa + up_pb), dn = r.half * (dn_pa + dn_pb);
                    gp[0] = (up - dn) * r.inv2dx[0];
                }
                {
                    T up = r.half * (pa_1 + pb_1), dn = r.half * (pa_3 + pb_3);
                    gp[1] = (up - dn) * r.inv2dx[1];
                }
                gp[2] = T(0);
                C0 = dtphi * bb[0] - (e[1] * gp[2] - e[2] * gp[1]);
                C1 = dtphi * bb[1] - (e[2] * gp[0] - e[0] * gp[2]);
                C2 = dtphi * bb[2] - (e[0] * gp[1] - e[1] * gp[0]);
            }
            c_2[0] = C0; c_2[1] = C1; c_2[2] = C2;
        }
        // ---- S3: B0z^{n+1} at plane p1
        {
            const T dn_e0y = lane_dn(e0h_1[1]);
            T v = T(0);
            if (vx_nod && vy_nod(p1)) {
                T a = r.cdt[0] * (e0h_1[1] - dn_e0y), b = r.cdt[1] * (e0h_1[0] - e0h_2[0]);
                v = b0z_1 - (a - b);
                if (own_x && own_plane(p1)) ste(1, 2, o1, v);
            }
            b0p_1 = v;
        }
        // ---- S4: E1^{n+1/2} at plane p2
        {
            const T up_b1z = lane_up(b1_2[2]), up_b1y = lane_up(b1_2[1]);
            const T dn_cx = lane_dn(c_2[0]);
            T v[3] = {T(0), T(0), T(0)};
            const bool own = own_x && own_plane(p2);
            // E1x: nodal x, centred y
            if (vx_nod && vy_cen(p2)) {
                T lo = (mx && gx - 1 < 0) ? c_2[0] : dn_cx;
                T hi = (mx && gx > n0 - 1) ? dn_cx : c_2[0];
                T Sc = r.half * (lo + hi);
                T a = r.cdt[1] * (b1_1[2] - b1_2[2]), b = T(0);
                T rhs = (a - b) - r.cg1 * Sc;
                v[0] = e1m[0] + T(1) * rhs;
                if (own) ste(2, 0, o2, v[0]);
            }
            // E1y: centred x, nodal y
            if (vx_cen && vy_nod(p2)) {
                T lo = (my && p2 - 1 < 0) ? c_2[1] : c_3[1];
                T hi = (my && p2 > n1 - 1) ? c_3[1] : c_2[1];
                T Sc = r.half * (lo + hi);
                T a = T(0), b = r.cdt[0] * (up_b1z - b1_2[2]);
                T rhs = (a - b) - r.cg1 * Sc;
                v[1] = e1m[1] + T(1) * rhs;
                if (own) ste(2, 1, o2, v[1]);
            }
            // E1z: centred x, centred y
            if (vx_cen && vy_cen(p2)) {
                T Sc = c_2[2];
                T a = r.cdt[0] * (up_b1y - b1_2[1]), b = r.cdt[1] * (b1_1[0] - b1_2[0]);
                T rhs = (a - b) - r.cg1 * Sc;
                v[2] = e1m[2] + T(1) * rhs;
                if (own) ste(2, 2, o2, v[2]);
            }
            e1h_2[0] = v[0]; e1h_2[1] = v[1]; e1h_2[2] = v[2];
            // Mur ghosts of E1y, E1z across x; of E1x, E1z across y
            const T up_y = lane_up(e1h_2[1]), dn_y = lane_dn(e1h_2[1]);
            const T up_z = lane_up(e1h_2[2]), dn_z = lane_dn(e1h_2[2]);
            if (mx && (gx == -1 || gx == n0)) {
                const int side = gx == -1 ? 0 : 1, ox = side ? -1 : 1;
                const bool owner = own_plane(p2) && lane + ox >= 3 && lane + ox < 3 + wid && gx + ox < own_x_hi;
                if (vy_nod(p2)) e1h_2[1] = ghost(1, 1, 0, side, p2, ox, p2, side ? dn_y : up_y, owner);
                if (vy_cen(p2)) e1h_2[2] = ghost(1, 2, 0, side, p2, ox, p2, side ? dn_z : up_z, owner);
            }
            if (my) {
                if (p2 == 0) {
                    if (vx_nod) e1h_3[0] = ghost(1, 0, 1, 0, -1, 0, 0, e1h_2[0], own_x && own_plane(0));
                    if (vx_cen) e1h_3[2] = ghost(1, 2, 1, 0, -1, 0, 0, e1h_2[2], own_x && own_plane(0));
                } else if (p2 == n1) {
                    // only the last chunk (which owns the nodal row n1) marches p2 up to n1
                    if (vx_nod) e1h_2[0] = ghost(1, 0, 1, 1, n1, 0, n1 - 1, e1h_3[0], own_x && own_plane(n1));
                    if (vx_cen) e1h_2[2] = ghost(1, 2, 1, 1, n1, 0, n1 - 1, e1h_3[2], own_x && own_plane(n1));
                }
            }
        }
        // ---- S5: B1^{n+1} and S6: phi^{n+3/2} at plane p2
        {
            const T dn_e1z = lane_dn(e1h_2[2]), dn_e1y = lane_dn(e1h_2[1]);
            const T up_e0x = lane_up(e0h_2[0]);
            const T up_b2 = lane_up(b0z_2), up_b1 = lane_up(b0z_1);
            const T up_p2 = lane_up(b0p_2), up_p1 = lane_up(b0p_1);
            const T up_pb = lane_up(pb_2), dn_pb = lane_dn(pb_2);
            if (own_x && own_plane(p2)) {
                // B1x: centred x, nodal y
                if (vx_cen && vy_nod(p2)) {
                    T a = r.cdt[1] * (e1h_2[2] - e1h_3[2]), b = T(0);
                    ste(3, 0, o2, b1_2[0] - (a - b));
                }
                // B1y: nodal x, centred y
                if (vx_nod && vy_cen(p2)) {
                    T a = T(0), b = r.cdt[0] * (e1h_2[2] - dn_e1z);
                    ste(3, 1, o2, b1_2[1] - (a - b));
                }
                // B1z: nodal x, nodal y
                if (vx_nod && vy_nod(p2)) {
                    T a = r.cdt[0] * (e1h_2[1] - dn_e1y), b = r.cdt[1] * (e1h_2[0] - e1h_3[0]);
                    ste(3, 2, o2, b1_2[2] - (a - b));
                }
                if (vx_cen && vy_cen(p2)) {
                    const int gi = wrap1(gx, n0), gj = my ? p2 : wrap1(p2, n1);
                    T e[3], bb[3];
                    e[0] = r.half * (e0h_2[0] + up_e0x);
                    e[1] = r.half * (e0h_2[1] + e0h_1[1]);
                    e[2] = T(0);
                    T bo0 = T(0), bn0 = T(0), bo1 = T(0), bn1 = T(0);
                    T bo2 = T(0.25) * ((b0z_2 + up_b2) + (b0z_1 + up_b1));
                    T bn2 = T(0.25) * ((b0p_2 + up_p2) + (b0p_1 + up_p1));
                    bb[0] = r.half * (bo0 + bn0) + bext0;
                    bb[1] = r.half * (bo1 + bn1) + bext1;
                    bb[2] = r.half * (bo2 + bn2) + bext2;
                    T sax = r.gax * (e[0] * bb[0] + e[1] * bb[1] + e[2] * bb[2]);
                    T pa = pa_2, pb = pb_2;
                    T lap = T(0);
                    lap += ((up_pb - T(2) * pb) + dn_pb) * r.inv_dx2[0];
                    lap += ((pb_1 - T(2) * pb) + pb_3) * r.inv_dx2[1];
                    // (an FP64 interior keeps clear of a damping layer)
                    T sdt = ((!INTERIOR || sizeof(T) == 4) && (r.axbc[0] == AXF_AX_PML || r.axbc[1] == AXF_AX_PML))
                                ? pml_sdt<2>(*rp, gi, gj, 0) : T(0);
                    T x = r.dt2 * ((sax - r.m2 * pb) + lap) - sdt * sdt * pb;
                    T num = ((x + sdt * pa) + T(2) * pb) - pa;
                    T pn = num;
                    if (sdt != T(0)) pn = num / (T(1) + sdt);
                    stp(ln, o2, pn);
                    const int gv[2] = {gi, gj};
#pragma unroll
                    for (int d = 0; d < 2; d++) {
                        if (INTERIOR || r.axbc[d] == AXF_AX_PERIODIC) continue;
#pragma unroll
                        for (int side = 0; side < 2; side++) {
                            if (gv[d] != (side ? r.n[d] - 1 : 0)) continue;
                            long f = face_index(r, d, gi, gj, 0);
                            T gval;
                            if (r.axbc[d] == AXF_AX_OUTFLOW) {
                                T gbv = gld((const T *)face_of(rp, q_axg(d, side, lb)), f);
                                T gav = gld((const T *)face_of(rp, q_axg(d, side, la)), f), rr = rp->out_r[d];
                                T xx = (((T(-2) * gbv + T(2) * gav) - r.dt2 * (sax - r.m2 * gbv)) + rr * pb - rr * rr * (pb - T(2) * gbv))
                                       / (rr + rr * rr);
                                gval = gav + rr * (pb - xx);
                            } else {
                                gval = pn;
                            }
                            gst(face_of(rp, q_axg(d, side, ln)), f, gval);
                        }
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------ several steps per pass
//
// Temporal blocking of the interior march: a wavefront advances its rows NS
// (2, 3 or 4) time steps per pass.  Stage 0 is the one-step pipeline on the
// loaded rows; stage k is the same pipeline one row behind stage k - 1, fed
// from its registers (E, B and the axion level of step n + k) instead of from
// memory, so each row of the state is read once and written once per NS
// steps.  Every stage uses the point formulas of the one-step interior march
// in the same order, so the results are the same bits.

// register windows of one stage along y (suffix = rows behind the newest row t
// of the stage); the outputs of an advance are at rows t - 1 (E0^{n+1/2},
// B0^{n+1}) and t - 2 (E1^{n+1/2}, B1^{n+1}, phi^{n+3/2})
template <typename T>
struct Stage {
    T b0z_2, b0z_1, b0z_0;
    T pa_3, pa_2, pa_1, pb_3, pb_2, pb_1;
    T b1_2[3], b1_1[3];
    T e0h_2[2], e0h_1[2], e0n_2[2], e0n_1[2];
    T c_3[3], c_2[3];
    T b0p_2, b0p_1;
    T e1h_3[3], e1h_2[3];
    T b1n[3], pn;                          // B1^{n+1} and phi^{n+3/2} at row t - 2

    __device__ __forceinline__ void clear()
    {
        b0z_2 = b0z_1 = b0z_0 = T(0);
        pa_3 = pa_2 = pa_1 = pb_3 = pb_2 = pb_1 = T(0);
        b0p_2 = b0p_1 = pn = T(0);
#pragma unroll
        for (int c = 0; c < 3; c++) b1_2[c] = b1_1[c] = c_3[c] = c_2[c] = e1h_3[c] = e1h_2[c] = b1n[c] = T(0);
#pragma unroll
        for (int c = 0; c < 2; c++) e0h_2[c] = e0h_1[c] = e0n_2[c] = e0n_1[c] = T(0);
    }

    // one row of the interior one-step march: take in B0z at row t, B1, the
    // two axion levels and E0 at row t - 1, E1 at row t - 2; S5 and S6 (B1 and
    // phi at t - 2) only when full
    template <typename K>
    __device__ __forceinline__ void advance(const K& r, T bext0, T bext1, T bext2, T in_b0z, const T in_b1[3], T in_pa,
                                            T in_pb, const T e0m[2], const T e1m[3], bool full, bool compute = true,
                                            T sdt = T(0))
    {
        b0z_2 = b0z_1; b0z_1 = b0z_0; b0z_0 = in_b0z;
        pa_3 = pa_2; pa_2 = pa_1; pa_1 = in_pa;
        pb_3 = pb_2; pb_2 = pb_1; pb_1 = in_pb;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            b1_2[c] = b1_1[c];
            c_3[c] = c_2[c];
            e1h_3[c] = e1h_2[c];
            b1_1[c] = in_b1[c];
        }
#pragma unroll
        for (int c = 0; c < 2; c++) {
            e0h_2[c] = e0h_1[c];
            e0n_2[c] = e0n_1[c];
        }
        b0p_2 = b0p_1;
        // (a warm-up row no stored value needs: take the inputs only)
        if (!compute) return;
        // S1: E0^{n+1/2}, E0^n at row t - 1
        {
            const T up_b0z = lane_up(b0z_1);
            T eh[2], en[2];
            {
                T a = r.cdt[1] * (b0z_0 - b0z_1), b = T(0);
                T rhs = a - b;
                eh[0] = e0m[0] + T(1) * rhs;
                en[0] = r.half * (e0m[0] + eh[0]);
            }
            {
                T a = T(0), b = r.cdt[0] * (up_b0z - b0z_1);
                T rhs = a - b;
                eh[1] = e0m[1] + T(1) * rhs;
                en[1] = r.half * (e0m[1] + eh[1]);
            }
            e0h_1[0] = eh[0]; e0h_1[1] = eh[1];
            e0n_1[0] = en[0]; e0n_1[1] = en[1];
        }
        // S2: C^n at the centres of row t - 2
        {
            T e[3], bb[3], gp[3];
            const T up_en0 = lane_up(e0n_2[0]);
            const T up_b2 = lane_up(b0z_2), up_b1 = lane_up(b0z_1);
            const T up_pa = lane_up(pa_2), up_pb = lane_up(pb_2), dn_pa = lane_dn(pa_2), dn_pb = lane_dn(pb_2);
            e[0] = r.half * (e0n_2[0] + up_en0);
            e[1] = r.half * (e0n_2[1] + e0n_1[1]);
            e[2] = T(0);
            bb[0] = T(0) + bext0;
            bb[1] = T(0) + bext1;
            bb[2] = T(0.25) * ((b0z_2 + up_b2) + (b0z_1 + up_b1)) + bext2;
            T dtphi = (pb_2 - pa_2) * r.inv_dt;
            {
                T up = r.half * (up_pa + up_pb), dn = r.half * (dn_pa + dn_pb);
                gp[0] = (up - dn) * r.inv2dx[0];
            }
            {
                T up = r.half * (pa_1 + pb_1), dn = r.half * (pa_3 + pb_3);
                gp[1] = (up - dn) * r.inv2dx[1];
            }
            gp[2] = T(0);
            c_2[0] = dtphi * bb[0] - (e[1] * gp[2] - e[2] * gp[1]);
            c_2[1] = dtphi * bb[1] - (e[2] * gp[0] - e[0] * gp[2]);
            c_2[2] = dtphi * bb[2] - (e[0] * gp[1] - e[1] * gp[0]);
        }
        // S3: B0z^{n+1} at row t - 1
        {
            const T dn_e0y = lane_dn(e0h_1[1]);
            T a = r.cdt[0] * (e0h_1[1] - dn_e0y), b = r.cdt[1] * (e0h_1[0] - e0h_2[0]);
            b0p_1 = b0z_1 - (a - b);
        }
        // S4: E1^{n+1/2} at row t - 2
        {
            const T up_b1z = lane_up(b1_2[2]), up_b1y = lane_up(b1_2[1]);
            const T dn_cx = lane_dn(c_2[0]);
            {
                T Sc = r.half * (dn_cx + c_2[0]);
                T a = r.cdt[1] * (b1_1[2] - b1_2[2]), b = T(0);
                T rhs = (a - b) - r.cg1 * Sc;
                e1h_2[0] = e1m[0] + T(1) * rhs;
            }
            {
                T Sc = r.half * (c_3[1] + c_2[1]);
                T a = T(0), b = r.cdt[0] * (up_b1z - b1_2[2]);
                T rhs = (a - b) - r.cg1 * Sc;
                e1h_2[1] = e1m[1] + T(1) * rhs;
            }
            {
                T Sc = c_2[2];
                T a = r.cdt[0] * (up_b1y - b1_2[1]), b = r.cdt[1] * (b1_1[0] - b1_2[0]);
                T rhs = (a - b) - r.cg1 * Sc;
                e1h_2[2] = e1m[2] + T(1) * rhs;
            }
        }
        if (!full) return;
        // S5: B1^{n+1} and S6: phi^{n+3/2} at row t - 2
        {
            const T dn_e1z = lane_dn(e1h_2[2]), dn_e1y = lane_dn(e1h_2[1]);
            {
                T a = r.cdt[1] * (e1h_2[2] - e1h_3[2]), b = T(0);
                b1n[0] = b1_2[0] - (a - b);
            }
            {
                T a = T(0), b = r.cdt[0] * (e1h_2[2] - dn_e1z);
                b1n[1] = b1_2[1] - (a - b);
            }
            {
                T a = r.cdt[0] * (e1h_2[1] - dn_e1y), b = r.cdt[1] * (e1h_2[0] - e1h_3[0]);
                b1n[2] = b1_2[2] - (a - b);
            }
        }
        {
            const T up_e0x = lane_up(e0h_2[0]);
            const T up_b2 = lane_up(b0z_2), up_b1 = lane_up(b0z_1);
            const T up_p2 = lane_up(b0p_2), up_p1 = lane_up(b0p_1);
            const T up_pb = lane_up(pb_2), dn_pb = lane_dn(pb_2);
            T e[3], bb[3];
            e[0] = r.half * (e0h_2[0] + up_e0x);
            e[1] = r.half * (e0h_2[1] + e0h_1[1]);
            e[2] = T(0);
            T bo0 = T(0), bn0 = T(0), bo1 = T(0), bn1 = T(0);
            T bo2 = T(0.25) * ((b0z_2 + up_b2) + (b0z_1 + up_b1));
            T bn2 = T(0.25) * ((b0p_2 + up_p2) + (b0p_1 + up_p1));
            bb[0] = r.half * (bo0 + bn0) + bext0;
            bb[1] = r.half * (bo1 + bn1) + bext1;
            bb[2] = r.half * (bo2 + bn2) + bext2;
            T sax = r.gax * (e[0] * bb[0] + e[1] * bb[1] + e[2] * bb[2]);
            T pa = pa_2, pb = pb_2;
            T lap = T(0);
            lap += ((up_pb - T(2) * pb) + dn_pb) * r.inv_dx2[0];
            lap += ((pb_1 - T(2) * pb) + pb_3) * r.inv_dx2[1];
            T x = r.dt2 * ((sax - r.m2 * pb) + lap) - sdt * sdt * pb;
            pn = ((x + sdt * pa) + T(2) * pb) - pa;
            if (sdt != T(0)) pn = pn / (T(1) + sdt);
        }
    }
};

// Interior rectangle of the wavefront grid: segments [sx0, sx1) and chunks
// [cy0, cy1) whose columns x0-3 .. x0+60 and rows c0-4 .. c1+1 stay at least
// `margin` cells inside the grid (margin = 1, or the damping-layer thickness on
// a PML axis).
// index of this wavefront in its workgroup, as a wave-uniform value (the
// compiler cannot tell that threadIdx.x / 64 is uniform; everything derived from
// it -- segment, chunk, rows -- then stays in scalar registers and branches)
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

struct WaveSplit {
    int nseg, nch, sx0, sx1, cy0, cy1;
    int wid;                              // output columns per segment
    __host__ __device__ long interior() const { return (long)(sx1 - sx0) * (cy1 - cy0); }
    __host__ __device__ long edge() const { return (long)nseg * nch - interior(); }
};

template <typename R>
__host__ __device__ inline WaveSplit wave2d_split(const R& h, int chunk)
{
    WaveSplit w;
    w.wid = kWaveOut;
    w.nseg = (h.nn[0] + kWaveOut - 1) / kWaveOut;
    w.nch = (h.nn[1] + chunk - 1) / chunk;
    // the damping layer of a PML axis is interior in FP32, where the marches
    // apply it from the run's profile table (4096^2: 106.5 -> 110.9 Gcell/s);
    // in FP64 the damped points cost the interior more than the smaller frame
    // saves (58.0 -> 55.6), and a layer wider than the table stays out too
    using TT = decltype(h.half);
    const bool out = sizeof(TT) == 8 || h.pml_n > kPmlProf;
    const int mxg = 1 + (out && h.axbc[0] == AXF_AX_PML ? h.pml_n : 0);
    const int myg = 1 + (out && h.axbc[1] == AXF_AX_PML ? h.pml_n : 0);
    // x0 = seg * kWaveOut: need x0 - 3 >= mxg and x0 + 60 <= n0 - 1 - mxg
    w.sx0 = (mxg + 3 + kWaveOut - 1) / kWaveOut;
    w.sx1 = (h.n[0] - 1 - mxg - 60) >= 0 ? (h.n[0] - 1 - mxg - 60) / kWaveOut + 1 : 0;
    // c0 = ch * chunk: need c0 - 4 >= myg and c0 + chunk + 1 <= n1 - 1 - myg; the
    // last chunk (which runs to the storage end) is never interior
    w.cy0 = (myg + 4 + chunk - 1) / chunk;
    w.cy1 = (h.n[1] - 2 - myg - chunk) >= 0 ? (h.n[1] - 2 - myg - chunk) / chunk + 1 : 0;
    w.cy1 = w.cy1 < w.nch - 1 ? w.cy1 : w.nch - 1;
    if (w.sx1 <= w.sx0 || w.cy1 <= w.cy0) w.sx0 = w.sx1 = w.cy0 = w.cy1 = 0;
    return w;
}

// segment and chunk of the e-th wavefront of the frame around the interior
__device__ __forceinline__ void wave2d_edge_item(const WaveSplit& w, long e, int& seg, int& ch)
{
    const long below = (long)w.cy0 * w.nseg;                 // chunks under the interior, all segments
    const int ni = w.sx1 - w.sx0, nside = w.nseg - ni;      // segments beside the interior
    const long beside = (long)(w.cy1 - w.cy0) * nside;
    if (e < below) {
        seg = (int)(e % w.nseg);
        ch = (int)(e / w.nseg);
    } else if (e < below + beside) {
        const long q = e - below;
        const int k = (int)(q % nside);
        ch = w.cy0 + (int)(q / nside);
        seg = k < w.sx0 ? k : k + ni;
    } else {
        const long q = e - below - beside;
        seg = (int)(q % w.nseg);
        ch = w.cy1 + (int)(q / w.nseg);
    }
}

template <typename T, int PD>
__global__ void __launch_bounds__(256) k_wave2d_int(const RunK<T> *__restrict__ rp, long step, WaveSplit w, int chunk)
{
    const long gw = xcd_band(blockIdx.x, gridDim.x) * 4L + wave_in_block();
    if (gw >= w.interior()) return;       // whole wavefronts only: no barriers in this kernel
    const int ni = w.sx1 - w.sx0;
    wave2d_body<T, true, PD>(rp, step, w.sx0 + (int)(gw % ni), w.cy0 + (int)(gw / ni), w.nch, chunk);
}

template <typename T>
__global__ void __launch_bounds__(256, 3) k_wave2d(const RunK<T> *__restrict__ rp, long step, WaveSplit w, int chunk)
{
    const long gw = blockIdx.x * 4L + wave_in_block();
    if (gw >= w.edge()) return;
    int seg, ch;
    wave2d_edge_item(w, gw, seg, ch);
    wave2d_body<T, false, 1>(rp, step, seg, ch, w.nch, chunk, w.wid);
}


// The pass.  Stage k is valid on lanes 2k + 1 .. 62 - 2k (each stage's
// stencils lose a lane on either side twice), so the pass owns lanes
// 2 NS - 1 .. 64 - 2 NS: 58 columns per wavefront for two steps, 54 for three,
// 50 for four.
// The boundary frame is NS one-step launches in order on the side stream:
// frame k advances step n + k everywhere but core k, the interior shrunk by
// NS - 1 - k rings (a ring is one segment and one frame chunk), so frame k + 1
// finds step n + k + 1 written next to its region; frame NS - 1 leaves out the
// interior.

// f(integral_constant<int, 0>) .. f(integral_constant<int, N - 1>), in order
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__host__ __device__ constexpr int pass_lane0(int ns) { return 2 * ns - 1; }
__host__ __device__ constexpr int pass_width(int ns) { return 66 - 4 * ns; }

template <int NS>
struct WavePass {
    WaveSplit in;                 // the interior, in pass_width columns and ci-row chunks
    WaveSplit fr[NS];             // frame k (cf-row chunks); its rectangle is core k
    int ci;
    int store_e;                  // also store E of step n + 1 (a record of step n follows)
};

template <int NS, typename R>
__host__ __device__ inline WavePass<NS> wave2d_split_pass(const R& h, int ci, int cf)
{
    WavePass<NS> p;
    p.ci = ci;
    p.store_e = 0;
    WaveSplit& w = p.in;
    const int W = pass_width(NS), lo = pass_lane0(NS);
    w.wid = W;
    w.nseg = (h.nn[0] + W - 1) / W;
    w.nch = (h.nn[1] + ci - 1) / ci;
    // the damping layer of a PML axis is interior in FP32, where the marches
    // apply it from the run's profile table (4096^2: 106.5 -> 110.9 Gcell/s);
    // in FP64 the damped points cost the interior more than the smaller frame
    // saves (58.0 -> 55.6), and a layer wider than the table stays out too
    using TT = decltype(h.half);
    const bool out = sizeof(TT) == 8 || h.pml_n > kPmlProf;
    const int mxg = 1 + (out && h.axbc[0] == AXF_AX_PML ? h.pml_n : 0);
    const int myg = 1 + (out && h.axbc[1] == AXF_AX_PML ? h.pml_n : 0);
    // columns x0 - lo .. x0 - lo + 63 and rows c0 - 3 NS - 1 .. c0 + ci + NS
    // (everything the pass loads or computes) stay at least the margin inside
    w.sx0 = (mxg + lo + W - 1) / W;
    w.sx1 = (h.n[0] - 1 - mxg - (63 - lo)) >= 0 ? (h.n[0] - 1 - mxg - (63 - lo)) / W + 1 : 0;
    w.cy0 = (myg + 3 * NS + 1 + ci - 1) / ci;
    w.cy1 = (h.n[1] - 1 - myg - NS - ci) >= 0 ? (h.n[1] - 1 - myg - NS - ci) / ci + 1 : 0;
    const int nchf = (h.nn[1] + cf - 1) / cf, k = ci / cf;
    // the last frame chunk (which runs to the storage end) is never interior
    if (w.cy1 * k > nchf - 1) w.cy1 = (nchf - 1) / k;
    // the innermost core needs at least one segment and one frame chunk
    const int need = 2 * (NS - 1) + 1;
    if (w.sx1 - w.sx0 < need || (w.cy1 - w.cy0) * k < need) w.sx0 = w.sx1 = w.cy0 = w.cy1 = 0;
    for (int f = 0; f < NS; f++) {
        const int d = w.sx1 > w.sx0 ? NS - 1 - f : 0;
        p.fr[f] = WaveSplit{w.nseg, nchf, w.sx0 + d, w.sx1 - d, w.cy0 * k + d, w.cy1 * k - d, W};
    }
    return p;
}

// What a wavefront of the interior stores besides E/B of step n + NS and the
// axion level n + NS + 1:
//   kCores: the level n + 2 + k in core k (the frames recompute the rest);
//   kCore:  the level n + NS (the older level of the state after the pass);
//   kRing:  every intermediate step n + k + 1 (E/B and the level n + k + 2),
//           so the frame launches of the later steps find it next to them.
enum PassMode { kCores = 0, kCore = 1, kRing = 2 };

// The wavefront of segment `seg` and chunk `ch` of the interior of an NS-step
// pass: reads E/B of step n and the axion levels n, n + 1.
template <typename T, int PD, int NS, int MODE>
__device__ __forceinline__ void wave2d_pass_body(const RunK<T> *__restrict__ rp, long step, const WavePass<NS>& wp,
                                                 int seg, int ch, int cf)
{
    KW<T> r = make_kw(rp);
    constexpr int lo = pass_lane0(NS), W = pass_width(NS);
    const int lane = threadIdx.x & 63;
    const int e_rd = em_slot(step, kEmSlots), e_wr = em_slot(step + NS, kEmSlots);
    const int la = phi_slot(step, kPhiSlots), lb = phi_slot(step + 1, kPhiSlots);
    const int ci = wp.ci;
    const bool store_e = __builtin_amdgcn_readfirstlane(wp.store_e) != 0;
    const int x0 = seg * W, gx = x0 - lo + lane;
    const bool own_x = lane >= lo && lane < lo + W;
    const int c0 = ch * ci, c1 = c0 + ci, cs = c0 - 3 * (NS - 1);   // stage 0 starts as if its chunk began at cs
    const unsigned es = sizeof(T), sxb = (unsigned)r.sx * es;
    const unsigned bx = (unsigned)gx * es;
    unsigned as_l = r.as;
    const char *const b_rd = r.sb + (size_t)q_em(0, e_rd, 0) * r.as;
    const char *const b_wr = r.sb + (size_t)q_em(0, e_wr, 0) * r.as;
    const char *const b_ph = r.sb + (size_t)q_phi(kEmSlots, 0) * r.as;
    auto lde = [&](int kind, int c, unsigned o) __attribute__((always_inline)) -> T {
        return ldo((const T *)b_rd, (unsigned)(kind * 3 + c) * as_l + o);
    };
    auto ste = [&](int kind, int c, unsigned o, T v) __attribute__((always_inline)) {
        sto((T *)b_wr, (unsigned)(kind * 3 + c) * as_l + o, v);
    };
    auto ldp = [&](int L, unsigned o) __attribute__((always_inline)) -> T { return ldo((const T *)b_ph, (unsigned)L * as_l + o); };
    auto stp = [&](int L, unsigned o, T v) __attribute__((always_inline)) { sto((T *)b_ph, (unsigned)L * as_l + o, v); };
    auto off = [&](int p) __attribute__((always_inline)) -> unsigned { return bx + (unsigned)p * sxb; };
    // E/B of the intermediate steps n + 1 .. n + NS - 1 (ring wavefronts)
    auto stm = [&](int k, int kind, int c, unsigned o, T v) __attribute__((always_inline)) {
        const char *b = r.sb + (size_t)q_em(0, em_slot(step + k + 1, kEmSlots), 0) * r.as;
        sto((T *)b, (unsigned)(kind * 3 + c) * as_l + o, v);
    };

    struct Pref {
        T b0z, b1[3], pa, pb, e0m[2], e1m[3];
    };
    Pref buf[PD];
    auto prefetch = [&](int t, Pref& P) __attribute__((always_inline)) {
        const unsigned o0 = off(t), o1 = off(t - 1), o2 = off(t - 2);
        P.b0z = lde(1, 2, o0);
#pragma unroll
        for (int c = 0; c < 3; c++) P.b1[c] = t - 1 >= cs - 1 ? lde(3, c, o1) : T(0);
        P.pa = ldp(la, o1);
        P.pb = ldp(lb, o1);
#pragma unroll
        for (int c = 0; c < 2; c++) P.e0m[c] = t - 1 >= cs - 2 ? lde(0, c, o1) : T(0);
#pragma unroll
        for (int c = 0; c < 3; c++) P.e1m[c] = t - 2 >= cs - 1 ? lde(2, c, o2) : T(0);
    };

    const T bext0 = bext_at(*rp, 0, gx), bext1 = bext_at(*rp, 1, gx), bext2 = bext_at(*rp, 2, gx);
    // sigma dt of the axion damping layer (Sec. II.D) at this column, combined
    // per row with the row's as the unfused kernel combines the axes; the
    // values come from the run's table of the profile (FP32 only: an FP64
    // interior, and a layer wider than the table, keep clear of it)
    constexpr bool kDamp = sizeof(T) == 4;
    const bool pmlx = kDamp && rp->axbc[0] == AXF_AX_PML, pmly = kDamp && rp->axbc[1] == AXF_AX_PML;
    const int pml_n = rp->pml_n, n0c = rp->n[0], n1c = rp->n[1];
    bool lx = false;
    T sdx = T(0);
    if (pmlx && pml_n <= kPmlProf) {
        const int dist = gx < n0c - 1 - gx ? gx : n0c - 1 - gx;
        if (dist < pml_n) {
            sdx = rp->pml_prof[dist];
            lx = true;
        }
    }
    auto sdt_at = [&](int row) __attribute__((always_inline)) -> T {
        T s = T(0);
        if (lx) s = sdx > s ? sdx : s;
        if (pmly && pml_n <= kPmlProf) {
            const int dist = row < n1c - 1 - row ? row : n1c - 1 - row;
            if (dist < pml_n) {
                const T sd = rp->pml_prof[dist];
                s = sd > s ? sd : s;
            }
        }
        return s;
    };
    // core k of an intermediate level: segments and rows of frame k's rectangle
    bool core_x[NS];
    int core_y0[NS], core_y1[NS];
#pragma unroll
    for (int k = 0; k < NS; k++) {
        core_x[k] = seg >= wp.fr[k].sx0 && seg < wp.fr[k].sx1;
        core_y0[k] = wp.fr[k].cy0 * cf;
        core_y1[k] = wp.fr[k].cy1 * cf;
    }
    Stage<T> sg[NS];
#pragma unroll
    for (int k = 0; k < NS; k++) sg[k].clear();
    // Warm-up: the first iteration whose loads a stored value needs, and the
    // first whose arithmetic of stage k does (a backward liveness of the stage
    // formulas over the rows, relative to c0); before those, the stage only
    // takes its inputs.  Peeled at compile time, so the main loop has no
    // per-row branch.
    constexpr int kLoad0 = -2 - NS;
    constexpr int kFirstTab[3][4] = {{-3, 0, 0, 0}, {-4, -2, 1, 0}, {-5, -3, -1, 2}};
    constexpr int kHead = kFirstTab[NS - 2][NS - 1] - kLoad0;
    const int t_first = c0 + kLoad0, t_last = c1 + NS;
    (void)cs;
#pragma unroll
    for (int k = 0; k < PD; k++)
        if (t_first + k <= t_last) prefetch(t_first + k, buf[k]);
    // one iteration; stage k computes when bit k of ACT is set
    auto iter = [&](auto act_c, const int t, Pref& P) __attribute__((always_inline)) {
        constexpr int ACT = decltype(act_c)::value;
        asm volatile("" : "+s"(as_l));
        const T b0z = P.b0z, pa = P.pa, pb = P.pb;
        const T b1[3] = {P.b1[0], P.b1[1], P.b1[2]};
        const T e0m[2] = {P.e0m[0], P.e0m[1]};
        const T e1m[3] = {P.e1m[0], P.e1m[1], P.e1m[2]};
        if (t + PD <= t_last) prefetch(t + PD, P);
        // stage 0: step n on the loaded rows
        sg[0].advance(r, bext0, bext1, bext2, b0z, b1, pa, pb, e0m, e1m, true, (ACT & 1) != 0, sdt_at(t - 2));
        // stage k: step n + k, one row behind stage k - 1, from its registers
        const int qf = t - NS - 1;              // the last stage's E1, B1, phi row
        const bool full = qf >= c0 && qf < c1;
#pragma unroll
        for (int k = 1; k < NS; k++) {
            const Stage<T>& pv = sg[k - 1];
            const T e1in[3] = {pv.e1h_3[0], pv.e1h_3[1], pv.e1h_3[2]};
            const T e0in[2] = {pv.e0h_2[0], pv.e0h_2[1]};
            sg[k].advance(r, bext0, bext1, bext2, pv.b0p_1, pv.b1n, pv.pb_2, pv.pn, e0in, e1in, k < NS - 1 || full,
                          ((ACT >> k) & 1) != 0, sdt_at(t - k - 2));
        }
        // a stage stores only where it computes (a warm-up iteration may
        // already hold a stored row of an early stage: four steps, row c0)
        if (own_x) {
            // intermediate steps n + k + 1 (k < NS - 1): E0, B0z at row
            // t - 1 - k; E1, B1 and the axion level n + k + 2 at row t - 2 - k
#pragma unroll
            for (int k = 0; k < NS - 1; k++) {
                const int q = t - 2 - k;
                if (((ACT >> k) & 1) == 0) continue;
                const bool rows = q >= c0 && q < c1;
                if (MODE == kCores && rows && q >= core_y0[k] && q < core_y1[k] && core_x[k])
                    stp(phi_slot(step + 2 + k, kPhiSlots), off(q), sg[k].pn);
                if (MODE == kCore && k == NS - 2 && rows)
                    stp(phi_slot(step + 2 + k, kPhiSlots), off(q), sg[k].pn);
                // E of step n + 1, which the record of step n averages with
                // E of step n (the ring stores it anyway; in one launch, only
                // core 0 is the interior's alone)
                if (MODE != kRing && k == 0 && store_e) {
                    const int qe = t - 1;
                    const bool in0 = MODE == kCore || core_x[0];
                    if (in0 && qe >= c0 && qe < c1 && (MODE == kCore || (qe >= core_y0[0] && qe < core_y1[0]))) {
                        const unsigned o = off(qe);
                        stm(0, 0, 0, o, sg[0].e0h_1[0]);
                        stm(0, 0, 1, o, sg[0].e0h_1[1]);
                    }
                    if (in0 && rows && (MODE == kCore || (q >= core_y0[0] && q < core_y1[0]))) {
                        const unsigned o = off(q);
#pragma unroll
                        for (int c = 0; c < 3; c++) stm(0, 2, c, o, sg[0].e1h_2[c]);
                    }
                }
                if (MODE == kRing) {
                    const int qe = t - 1 - k;
                    if (qe >= c0 && qe < c1) {
                        const unsigned o = off(qe);
                        stm(k, 0, 0, o, sg[k].e0h_1[0]);
                        stm(k, 0, 1, o, sg[k].e0h_1[1]);
                        stm(k, 1, 2, o, sg[k].b0p_1);
                    }
                    if (rows) {
                        const unsigned o = off(q);
#pragma unroll
                        for (int c = 0; c < 3; c++) stm(k, 2, c, o, sg[k].e1h_2[c]);
#pragma unroll
                        for (int c = 0; c < 3; c++) stm(k, 3, c, o, sg[k].b1n[c]);
                        stp(phi_slot(step + 2 + k, kPhiSlots), o, sg[k].pn);
                    }
                }
            }
            // the last stage: E0, B0z of step n + NS at row t - NS; E1, B1 and
            // the axion level n + NS + 1 at row t - NS - 1
            const Stage<T>& sl = sg[NS - 1];
            const int qe = t - NS;
            constexpr bool last_on = ((ACT >> (NS - 1)) & 1) != 0;
            if (last_on && qe >= c0 && qe < c1) {
                const unsigned o = off(qe);
                ste(0, 0, o, sl.e0h_1[0]);
                ste(0, 1, o, sl.e0h_1[1]);
                ste(1, 2, o, sl.b0p_1);
            }
            if (last_on && full) {
                const unsigned o = off(qf);
#pragma unroll
                for (int c = 0; c < 3; c++) ste(2, c, o, sl.e1h_2[c]);
#pragma unroll
                for (int c = 0; c < 3; c++) ste(3, c, o, sl.b1n[c]);
                stp(phi_slot(step + NS + 1, kPhiSlots), o, sl.pn);
            }
        }
    };
    // the warm-up iterations t_first + h, h < kHead
    static_for<kHead>([&](auto hc) __attribute__((always_inline)) {
        constexpr int h = decltype(hc)::value, t_rel = kLoad0 + h;
        constexpr int act = (t_rel >= kFirstTab[NS - 2][0] ? 1 : 0) | (t_rel >= kFirstTab[NS - 2][1] ? 2 : 0) |
                            (NS >= 3 && t_rel >= kFirstTab[NS - 2][2] ? 4 : 0) |
                            (NS >= 4 && t_rel >= kFirstTab[NS - 2][3] ? 8 : 0);
        iter(std::integral_constant<int, act>{}, t_first + h, buf[h % PD]);
    });
    constexpr int U = PD == 1 ? 1 : 6;
    for (int t0 = t_first + kHead; t0 <= t_last; t0 += U)
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int t = t0 + u;
        if (t > t_last) break;
        iter(std::integral_constant<int, (1 << NS) - 1>{}, t, buf[(u + kHead) % PD]);
    }
}

// the interior in one launch (kCores), or its core (kCore) or its ring
// (kRing): `rc` splits the interior's segments and chunks into the ring, its
// outermost segment and chunk on each side, and the core inside
template <typename T, int PD, int NS, int MODE>
__global__ void __launch_bounds__(256) k_wave2d_pass(const RunK<T> *__restrict__ rp, long step, WavePass<NS> wp, int cf,
                                                     WaveSplit rc)
{
    const long gw = xcd_band(blockIdx.x, gridDim.x) * 4L + wave_in_block();
    int seg, ch;
    if (MODE == kCores) {
        if (gw >= wp.in.interior()) return;
        const int ni = wp.in.sx1 - wp.in.sx0;
        seg = wp.in.sx0 + (int)(gw % ni);
        ch = wp.in.cy0 + (int)(gw / ni);
    } else if (MODE == kCore) {
        if (gw >= rc.interior()) return;
        const int ni = rc.sx1 - rc.sx0;
        seg = wp.in.sx0 + rc.sx0 + (int)(gw % ni);
        ch = wp.in.cy0 + rc.cy0 + (int)(gw / ni);
    } else {
        if (gw >= rc.edge()) return;
        wave2d_edge_item(rc, gw, seg, ch);
        seg += wp.in.sx0;
        ch += wp.in.cy0;
    }
    wave2d_pass_body<T, PD, NS, MODE>(rp, step, wp, seg, ch, cf);
}

// batched: every active run of the table, each with its own step and chunk
template <typename T, bool INTERIOR>
__global__ void __launch_bounds__(256, INTERIOR ? 1 : (sizeof(T) == 4 ? 5 : 3)) kb_wave2d(const BItem *__restrict__ it, int n, long s)
{
    constexpr int K = INTERIOR ? kWaveI : kWave;
    const long b = INTERIOR ? xcd_band(blockIdx.x, gridDim.x) : (long)blockIdx.x;
    const int i = find_item<K>(it, n, b);
    const RunK<T> *rp = uniform_desc<RunK<T>>(it[i].rk);
    const int chunk = it[i].chunk;
    const WaveSplit w = wave2d_split(*rp, chunk);
    const long gw = (b - it[i].blk[K]) * 4L + wave_in_block();
    if (INTERIOR) {
        if (gw >= w.interior()) return;
        const int ni = w.sx1 - w.sx0;
        wave2d_body<T, true, WavePD<T>::value>(rp, it[i].step0 + s, w.sx0 + (int)(gw % ni), w.cy0 + (int)(gw / ni), w.nch, chunk);
    } else {
        if (gw >= w.edge()) return;
        int seg, ch;
        wave2d_edge_item(w, gw, seg, ch);
        wave2d_body<T, false, 1>(rp, it[i].step0 + s, seg, ch, w.nch, chunk);
    }
}

// batched two-step pass: every active run of the table advances steps s and
// s + 1 of the call, each with its own pass shape; KIND selects the interior
// (kPair) or one of the two frame launches (kFrameA: step s, kFrameB: s + 1)
template <typename T, int KIND>
__global__ void __launch_bounds__(256, KIND == kPair ? 1 : (sizeof(T) == 4 ? 5 : 3)) kb_wave2d_pair(const BItem *__restrict__ it, int n, long s)
{
    const long b = KIND == kPair ? xcd_band(blockIdx.x, gridDim.x) : (long)blockIdx.x;
    const int i = find_item<KIND>(it, n, b);
    const RunK<T> *rp = uniform_desc<RunK<T>>(it[i].rk);
    const int cf = it[i].pass_cf;
    const WavePass<2> wp = wave2d_split_pass<2>(*rp, it[i].pass_ci, cf);
    const long gw = (b - it[i].blk[KIND]) * 4L + wave_in_block();
    const long step = it[i].step0 + s;
    if (KIND == kPair) {
        if (gw >= wp.in.interior()) return;
        const int ni = wp.in.sx1 - wp.in.sx0;
        wave2d_pass_body<T, sizeof(T) == 8 ? 3 : 2, 2, kCores>(rp, step, wp, wp.in.sx0 + (int)(gw % ni),
                                                               wp.in.cy0 + (int)(gw / ni), cf);
    } else {
        const WaveSplit& w = wp.fr[KIND == kFrameA ? 0 : 1];
        if (gw >= w.edge()) return;
        int seg, ch;
        wave2d_edge_item(w, gw, seg, ch);
        wave2d_body<T, false, 1>(rp, step + (KIND == kFrameB ? 1 : 0), seg, ch, w.nch, cf, w.wid);
    }
}

template <typename T>
void wave2d_pair_blocks(const RunK<T>& h, int ci, int cf, long *interior, long *frame_a, long *frame_b)
{
    const WavePass<2> wp = wave2d_split_pass<2>(h, ci, cf);
    *interior = (wp.in.interior() + 3) / 4;
    *frame_a = (wp.fr[0].edge() + 3) / 4;
    *frame_b = (wp.fr[1].edge() + 3) / 4;
}
template void wave2d_pair_blocks<float>(const RunK<float>&, int, int, long *, long *, long *);
template void wave2d_pair_blocks<double>(const RunK<double>&, int, int, long *, long *, long *);

template <typename T>
hipError_t launch_wave2d_pair_batch(const BItem *it, const BItem *host, int n, long s, hipStream_t st,
                                    const WaveStreams *ws)
{
    const unsigned ni = (unsigned)host[n].blk[kPair], na = (unsigned)host[n].blk[kFrameA];
    const unsigned nb = (unsigned)host[n].blk[kFrameB];
    const bool fork = ws && ws->side;
    hipStream_t se = st;
    if (fork) {
        hipEventRecord(ws->fork, st);
        hipStreamWaitEvent(ws->side, ws->fork, 0);
        se = ws->side;
    }
    if (na > 0) hipLaunchKernelGGL((kb_wave2d_pair<T, kFrameA>), dim3(na), dim3(256), 0, se, it, n, s);
    if (ni > 0) hipLaunchKernelGGL((kb_wave2d_pair<T, kPair>), dim3(ni), dim3(256), 0, st, it, n, s);
    if (nb > 0) hipLaunchKernelGGL((kb_wave2d_pair<T, kFrameB>), dim3(nb), dim3(256), 0, se, it, n, s);
    if (fork) {
        hipEventRecord(ws->join, ws->side);
        hipStreamWaitEvent(st, ws->join, 0);
    }
    return hipGetLastError();
}
template hipError_t launch_wave2d_pair_batch<float>(const BItem *, const BItem *, int, long, hipStream_t, const WaveStreams *);
template hipError_t launch_wave2d_pair_batch<double>(const BItem *, const BItem *, int, long, hipStream_t, const WaveStreams *);

// batched four-step pass: every active run of the table advances steps s ..
// s + 3 of the call, each with its own pass shape, in the three launches of a
// single run's split pass: KIND selects the interior's core (kQuadCore), its
// ring (kQuadRing, storing the intermediate steps) or the frame around the
// interior (kQuadFrame, launched once per step with the call's step in s)
template <typename T>
__device__ __forceinline__ WaveSplit quad_ring_core(const WavePass<4>& wp)
{
    const int nis = wp.in.sx1 - wp.in.sx0, nic = wp.in.cy1 - wp.in.cy0;
    WaveSplit rc{nis, nic, 1, nis - 1, 1, nic - 1, wp.in.wid};
    if (nis < 3 || nic < 3) rc.sx0 = rc.sx1 = rc.cy0 = rc.cy1 = 0;
    return rc;
}

template <typename T, int KIND>
__global__ void __launch_bounds__(256, KIND == kQuadFrame ? (sizeof(T) == 4 ? 5 : 3) : 1) kb_wave2d_quad(const BItem *__restrict__ it, int n, long s)
{
    const long b = KIND == kQuadFrame ? (long)blockIdx.x : xcd_band(blockIdx.x, gridDim.x);
    const int i = find_item<KIND>(it, n, b);
    const RunK<T> *rp = uniform_desc<RunK<T>>(it[i].rk);
    const int cf = it[i].quad_cf;
    const WavePass<4> wp = wave2d_split_pass<4>(*rp, it[i].quad_ci, cf);
    const long gw = (b - it[i].blk[KIND]) * 4L + wave_in_block();
    const long step = it[i].step0 + s;
    constexpr int PD = sizeof(T) == 8 ? 1 : 2;
    if constexpr (KIND == kQuadFrame) {
        const WaveSplit& w = wp.fr[3];
        if (gw >= w.edge()) return;
        int seg, ch;
        wave2d_edge_item(w, gw, seg, ch);
        wave2d_body<T, false, 1>(rp, step, seg, ch, w.nch, cf, w.wid);
    } else {
        const WaveSplit rc = quad_ring_core<T>(wp);
        int seg, ch;
        if (KIND == kQuadCore) {
            if (gw >= rc.interior()) return;
            const int ni = rc.sx1 - rc.sx0;
            seg = wp.in.sx0 + rc.sx0 + (int)(gw % ni);
            ch = wp.in.cy0 + rc.cy0 + (int)(gw / ni);
            wave2d_pass_body<T, PD, 4, kCore>(rp, step, wp, seg, ch, cf);
        } else {
            if (gw >= rc.edge()) return;
            wave2d_edge_item(rc, gw, seg, ch);
            wave2d_pass_body<T, PD, 4, kRing>(rp, step, wp, seg + wp.in.sx0, ch + wp.in.cy0, cf);
        }
    }
}

template <typename T>
void wave2d_quad_blocks(const RunK<T>& h, int ci, int cf, long blk[3])
{
    const WavePass<4> wp = wave2d_split_pass<4>(h, ci, cf);
    const int nis = wp.in.sx1 - wp.in.sx0, nic = wp.in.cy1 - wp.in.cy0;
    WaveSplit rc{nis, nic, 1, nis - 1, 1, nic - 1, wp.in.wid};
    if (nis < 3 || nic < 3) rc.sx0 = rc.sx1 = rc.cy0 = rc.cy1 = 0;
    blk[0] = (rc.interior() + 3) / 4;
    blk[1] = (rc.edge() + 3) / 4;
    blk[2] = (wp.fr[3].edge() + 3) / 4;
}
template void wave2d_quad_blocks<float>(const RunK<float>&, int, int, long *);
template void wave2d_quad_blocks<double>(const RunK<double>&, int, int, long *);

// the streams of a single run's split pass: the core on `st`, the ring on
// ws->ring, the frame on ws->side (its later steps after the ring has stored
// them)
template <typename T>
hipError_t launch_wave2d_quad_batch(const BItem *it, const BItem *host, int n, long s, hipStream_t st,
                                    const WaveStreams *ws)
{
    if (!ws || !ws->side || !ws->ring || !ws->ring_done) return hipErrorInvalidValue;
    const unsigned nc = (unsigned)host[n].blk[kQuadCore], nr = (unsigned)host[n].blk[kQuadRing];
    const unsigned nf = (unsigned)host[n].blk[kQuadFrame];
    hipEventRecord(ws->fork, st);
    hipStreamWaitEvent(ws->side, ws->fork, 0);
    hipStreamWaitEvent(ws->ring, ws->fork, 0);
    if (nr > 0) hipLaunchKernelGGL((kb_wave2d_quad<T, kQuadRing>), dim3(nr), dim3(256), 0, ws->ring, it, n, s);
    hipEventRecord(ws->ring_done, ws->ring);
    if (nf > 0) hipLaunchKernelGGL((kb_wave2d_quad<T, kQuadFrame>), dim3(nf), dim3(256), 0, ws->side, it, n, s);
    if (nc > 0) hipLaunchKernelGGL((kb_wave2d_quad<T, kQuadCore>), dim3(nc), dim3(256), 0, st, it, n, s);
    hipStreamWaitEvent(ws->side, ws->ring_done, 0);
    for (int f = 1; f < 4; f++)
        if (nf > 0) hipLaunchKernelGGL((kb_wave2d_quad<T, kQuadFrame>), dim3(nf), dim3(256), 0, ws->side, it, n, s + f);
    hipEventRecord(ws->join, ws->side);
    hipStreamWaitEvent(st, ws->join, 0);
    return hipGetLastError();
}
template hipError_t launch_wave2d_quad_batch<float>(const BItem *, const BItem *, int, long, hipStream_t, const WaveStreams *);
template hipError_t launch_wave2d_quad_batch<double>(const BItem *, const BItem *, int, long, hipStream_t, const WaveStreams *);

template <typename T>
void wave2d_blocks(const RunK<T>& h, int chunk, long *edge_blocks, long *interior_blocks)
{
    const WaveSplit w = wave2d_split(h, chunk);
    *edge_blocks = (w.edge() + 3) / 4;
    *interior_blocks = (w.interior() + 3) / 4;
}
template void wave2d_blocks<float>(const RunK<float>&, int, long *, long *);
template void wave2d_blocks<double>(const RunK<double>&, int, long *, long *);

template <typename T>
hipError_t launch_wave2d_batch(const BItem *it, const BItem *host, int n, long s, hipStream_t st,
                               const WaveStreams *ws)
{
    const unsigned ni = (unsigned)host[n].blk[kWaveI], ne = (unsigned)host[n].blk[kWave];
    const bool fork = ws && ws->side && ne > 0 && ni > 0;
    hipStream_t se = st;
    if (fork) {
        hipEventRecord(ws->fork, st);
        hipStreamWaitEvent(ws->side, ws->fork, 0);
        se = ws->side;
    }
    if (ne > 0) hipLaunchKernelGGL((kb_wave2d<T, false>), dim3(ne), dim3(256), 0, se, it, n, s);
    if (ni > 0) hipLaunchKernelGGL((kb_wave2d<T, true>), dim3(ni), dim3(256), 0, st, it, n, s);
    if (fork) {
        hipEventRecord(ws->join, ws->side);
        hipStreamWaitEvent(st, ws->join, 0);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wave2d(const RunK<T> *rk, const RunK<T>& h, long step, int chunk, int pd, hipStream_t st,
                         const WaveStreams *ws)
{
    const WaveSplit w = wave2d_split(h, chunk);
    const unsigned ni = (unsigned)((w.interior() + 3) / 4), ne = (unsigned)((w.edge() + 3) / 4);
    if (pd <= 0) pd = wave2d_default_pd(sizeof(T) == 8, 1);
    // the frame runs beside the interior on the side stream when there is one
    // (the two launches touch disjoint outputs and read only the old slots)
    const bool fork = ws && ws->side && ne > 0 && ni > 0;
    hipStream_t se = st;
    if (fork) {
        hipEventRecord(ws->fork, st);
        hipStreamWaitEvent(ws->side, ws->fork, 0);
        se = ws->side;
    }
    if (ne > 0) hipLaunchKernelGGL((k_wave2d<T>), dim3(ne), dim3(256), 0, se, rk, step, w, chunk);
    if (ni > 0) {
        if (pd <= 1) hipLaunchKernelGGL((k_wave2d_int<T, 1>), dim3(ni), dim3(256), 0, st, rk, step, w, chunk);
        else if (pd == 2) hipLaunchKernelGGL((k_wave2d_int<T, 2>), dim3(ni), dim3(256), 0, st, rk, step, w, chunk);
        else hipLaunchKernelGGL((k_wave2d_int<T, 3>), dim3(ni), dim3(256), 0, st, rk, step, w, chunk);
    }
    if (fork) {
        hipEventRecord(ws->join, ws->side);
        hipStreamWaitEvent(st, ws->join, 0);
    }
    return hipGetLastError();
}

int wave2d_default_pd(bool f64, int ns)
{
    // measured on 4096^2: one step per pass FP32 3, FP64 2; two steps FP32 2,
    // FP64 3; three and four steps FP32 2, FP64 1
    if (ns <= 1) return f64 ? 2 : 3;
    if (ns == 2) return f64 ? 3 : 2;
    return f64 ? 1 : 2;
}

template <typename T, int NS, int MODE>
static void launch_interior(const RunK<T> *rk, long step, const WavePass<NS>& wp, int cf, const WaveSplit& rc,
                            unsigned nb, int pd, hipStream_t st)
{
    if (pd <= 1) hipLaunchKernelGGL((k_wave2d_pass<T, 1, NS, MODE>), dim3(nb), dim3(256), 0, st, rk, step, wp, cf, rc);
    else if (pd == 2) hipLaunchKernelGGL((k_wave2d_pass<T, 2, NS, MODE>), dim3(nb), dim3(256), 0, st, rk, step, wp, cf, rc);
    else hipLaunchKernelGGL((k_wave2d_pass<T, 3, NS, MODE>), dim3(nb), dim3(256), 0, st, rk, step, wp, cf, rc);
}

template <typename T, int NS>
static hipError_t launch_pass_ns(const RunK<T> *rk, const RunK<T>& h, long step, int ci, int cf, int pd, hipStream_t st,
                                 const WaveStreams *ws, bool store_e)
{
    WavePass<NS> wp = wave2d_split_pass<NS>(h, ci, cf);
    wp.store_e = store_e ? 1 : 0;
    if (wp.in.interior() == 0) return hipErrorInvalidValue;
    if (pd <= 0) pd = wave2d_default_pd(sizeof(T) == 8, NS);
    // ring and core of the interior (the core empty when the interior is
    // less than three segments or chunks across)
    const int nis = wp.in.sx1 - wp.in.sx0, nic = wp.in.cy1 - wp.in.cy0;
    WaveSplit rc{nis, nic, 1, nis - 1, 1, nic - 1, wp.in.wid};
    if (nis < 3 || nic < 3) rc.sx0 = rc.sx1 = rc.cy0 = rc.cy1 = 0;
    // (measured on 4096^2 FP32: three steps 93.6 Gcell/s split against 86.1;
    // two steps 70.0 against 72.0, where the frames were cheap already; four
    // steps are taken split)
    const bool split = NS >= 3 && ws && ws->side && ws->ring;
    if (!split) {
        // one interior launch; frame k leaves out core k
        const bool fork = ws && ws->side;
        hipStream_t se = st;
        if (fork) {
            hipEventRecord(ws->fork, st);
            hipStreamWaitEvent(ws->side, ws->fork, 0);
            se = ws->side;
        }
        const unsigned nf0 = (unsigned)((wp.fr[0].edge() + 3) / 4);
        if (nf0 > 0) hipLaunchKernelGGL((k_wave2d<T>), dim3(nf0), dim3(256), 0, se, rk, step, wp.fr[0], cf);
        launch_interior<T, NS, kCores>(rk, step, wp, cf, rc, (unsigned)((wp.in.interior() + 3) / 4), pd, st);
        for (int f = 1; f < NS; f++) {
            const unsigned nf = (unsigned)((wp.fr[f].edge() + 3) / 4);
            if (nf > 0) hipLaunchKernelGGL((k_wave2d<T>), dim3(nf), dim3(256), 0, se, rk, step + f, wp.fr[f], cf);
        }
        if (fork) {
            hipEventRecord(ws->join, ws->side);
            hipStreamWaitEvent(st, ws->join, 0);
        }
        return hipGetLastError();
    }
    // three streams: the core on `st`; the ring on ws->ring; the frame, every
    // launch leaving out just the interior, on ws->side, its steps n + 1 ..
    // after the ring has stored them
    const WaveSplit& fr = wp.fr[NS - 1];
    const unsigned nfr = (unsigned)((fr.edge() + 3) / 4);
    hipEventRecord(ws->fork, st);
    hipStreamWaitEvent(ws->side, ws->fork, 0);
    hipStreamWaitEvent(ws->ring, ws->fork, 0);
    launch_interior<T, NS, kRing>(rk, step, wp, cf, rc, (unsigned)((rc.edge() + 3) / 4), pd, ws->ring);
    hipEventRecord(ws->ring_done, ws->ring);
    if (nfr > 0) hipLaunchKernelGGL((k_wave2d<T>), dim3(nfr), dim3(256), 0, ws->side, rk, step, fr, cf);
    if (rc.interior() > 0)
        launch_interior<T, NS, kCore>(rk, step, wp, cf, rc, (unsigned)((rc.interior() + 3) / 4), pd, st);
    hipStreamWaitEvent(ws->side, ws->ring_done, 0);
    for (int f = 1; f < NS; f++)
        if (nfr > 0) hipLaunchKernelGGL((k_wave2d<T>), dim3(nfr), dim3(256), 0, ws->side, rk, step + f, fr, cf);
    hipEventRecord(ws->join, ws->side);
    hipStreamWaitEvent(st, ws->join, 0);
    return hipGetLastError();
}

template <typename T>
bool wave2d_pass_available(const RunK<T>& h, int ns, int ci, int cf)
{
    if (ci <= 0 || cf <= 0 || ci % cf != 0) return false;
    if (ns == 2) return wave2d_split_pass<2>(h, ci, cf).in.interior() > 0;
    if (ns == 3) return wave2d_split_pass<3>(h, ci, cf).in.interior() > 0;
    if (ns == 4) return wave2d_split_pass<4>(h, ci, cf).in.interior() > 0;
    return false;
}

template <typename T>
hipError_t launch_wave2d_pass(const RunK<T> *rk, const RunK<T>& h, long step, int ns, int ci, int cf, int pd,
                              hipStream_t st, const WaveStreams *ws, bool store_e)
{
    if (ns == 2) return launch_pass_ns<T, 2>(rk, h, step, ci, cf, pd, st, ws, store_e);
    if (ns == 3) return launch_pass_ns<T, 3>(rk, h, step, ci, cf, pd, st, ws, store_e);
    if (ns == 4) return launch_pass_ns<T, 4>(rk, h, step, ci, cf, pd, st, ws, store_e);
    return hipErrorInvalidValue;
}

template bool wave2d_pass_available<float>(const RunK<float>&, int, int, int);
template bool wave2d_pass_available<double>(const RunK<double>&, int, int, int);
template hipError_t launch_wave2d_pass<float>(const RunK<float> *, const RunK<float>&, long, int, int, int, int, hipStream_t, const WaveStreams *, bool);
template hipError_t launch_wave2d_pass<double>(const RunK<double> *, const RunK<double>&, long, int, int, int, int, hipStream_t, const WaveStreams *, bool);
template hipError_t launch_wave2d<float>(const RunK<float> *, const RunK<float>&, long, int, int, hipStream_t, const WaveStreams *);
template hipError_t launch_wave2d<double>(const RunK<double> *, const RunK<double>&, long, int, int, hipStream_t, const WaveStreams *);
template hipError_t launch_wave2d_batch<float>(const BItem *, const BItem *, int, long, hipStream_t, const WaveStreams *);
template hipError_t launch_wave2d_batch<double>(const BItem *, const BItem *, int, long, hipStream_t, const WaveStreams *);

template <int D, int TX, int TY, typename T>
size_t Fused<D, TX, TY, T>::lds_bytes() { return FK<D, TX, TY, T>::LDS; }

template <int D, int TX, int TY, typename T>
int Fused<D, TX, TY, T>::threads() { return FK<D, TX, TY, T>::NT; }

template <int D, int TX, int TY, typename T>
hipError_t Fused<D, TX, TY, T>::launch(const RunK<T> *rk, const RunK<T>& h, long step, int chunk, hipStream_t st)
{
    using K = FK<D, TX, TY, T>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_fused<D, TX, TY, T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)K::LDS);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int M = D - 1;
    int ntx = (h.n[0] + TX - 1) / TX;
    int nty = D == 3 ? (h.n[1] + TY - 1) / TY : 1;
    int nch = (h.nn[M] + chunk - 1) / chunk;
    unsigned nb = (unsigned)(ntx * nty * nch);
    hipLaunchKernelGGL((k_fused<D, TX, TY, T>), dim3(nb), dim3(K::NT), K::LDS, st, rk, step, ntx, nty, nch, chunk);
    return hipGetLastError();
}

template struct Fused<2, 256, 1, float>;
template struct Fused<2, 128, 1, double>;
template struct Fused<3, 32, 6, float>;
template struct Fused<3, 32, 8, float>;
template struct Fused<3, 32, 4, double>;

}  // namespace axf
