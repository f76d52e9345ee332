// axf_march3d.hip -- the one-pass 3D step: one launch advances every field of
// a run by one full step (Sec. II.C, eqs. update_E, update_B and
// update_axion, in the leapfrog form), so that each cell's state is read from
// HBM once and written once.
//
// Geometry.  A wavefront owns one y row of 64 consecutive x columns (column
// gx = x0 - 2 + lane; `wid` <= 60 of them are its own, with two halo columns
// below and two above) and marches along z through a chunk of planes.  A
// workgroup stacks NW such row wavefronts along y: rows y0 - 1 .. y0 + NW - 2,
// of which the NW - 2 inner rows are its own.  x neighbours come from the
// neighbouring lane (DPP shifts), the z history of every quantity stays in
// the lane's registers, and y neighbours are exchanged through LDS with one
// workgroup barrier per plane.
//
// Pipeline.  Iteration i takes in B0 of plane i, both axion levels and E0 of
// plane i - 1, B1 of plane i - 2 and E1 of plane i - 3, and computes
//   S1  E0^{n+1/2}, E0^n at plane i - 1      (+ Mur ghosts of E0)
//   S2  axion current C^n at the cells of plane i - 2
//   S3  B0^{n+1} at plane i - 2
//   S4  E1^{n+1/2} at plane i - 3            (+ Mur ghosts of E1)
//   S5  B1^{n+1} at plane i - 4
//   S6  phi^{n+3/2} at plane i - 4           (+ axion ghosts of the new level)
// Each lag is the smallest with which every value a stage takes from a y
// neighbour was written to LDS in an earlier iteration, i.e. before the
// barrier that ends it:
//   S1 reads B0x, B0z one row up (loaded at lag 0);
//   S2 reads E0^n_y, B0x, B0z one row up and both axion levels on both sides;
//   S3 reads E0x, E0z^{n+1/2} one row down (S1);
//   S4 reads B1x, B1z one row up and C_y one row down (S2);
//   S5 reads E1x, E1z^{n+1/2} one row down (S4);
//   S6 reads E0y^{n+1/2}, B0x^{n+1}, B0z^{n+1} (also one plane up) and phi one
//      row up, phi one row down.
// The two rows outside a workgroup's own rows do part of the work only: the
// lower one (y0 - 1) computes E0, C and E1 (the first own row's B reads E one
// row down), the upper one (y0 + NW - 2) E0 and B0 (the last own row's axion
// update averages B0^{n+1} one row up).  The lowest wavefront also loads the
// axion levels of row y0 - 2 and the highest B0x, B0z of row y0 + NW - 1.
//
// The point formulas are those of the unfused kernels, in the same operation
// order, so the two paths agree bit for bit.
#include "axf_fused.h"
#include "axf_stencil.h"

#ifndef AXF_M3_NW
#define AXF_M3_NW 12
#endif

namespace axf {

namespace m3 {

__device__ __forceinline__ int imodn(int v, int n) { int r = v % n; return r < 0 ? r + n : r; }

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

// global load / store at a 32-bit byte offset from a wave-uniform array base
template <typename T>
__device__ __forceinline__ T ldo(const char *base, unsigned boff)
{
    return *(const __attribute__((address_space(1))) T *)((const __attribute__((address_space(1))) char *)base + boff);
}
template <typename T>
__device__ __forceinline__ void sto(const char *base, unsigned boff, T v)
{
    *(__attribute__((address_space(1))) T *)((__attribute__((address_space(1))) char *)base + boff) = v;
}
// element i of a boundary plane (boundary code only)
template <typename T>
__device__ __forceinline__ T fld(const RunK<T> *rp, int q, long i)
{
    return ((const __attribute__((address_space(1))) T *)(rp->face_base + q * rp->face_stride))[i];
}
template <typename T>
__device__ __forceinline__ void fst(const RunK<T> *rp, int q, long i, T v)
{
    ((__attribute__((address_space(1))) T *)(rp->face_base + q * rp->face_stride))[i] = v;
}

}  // namespace m3

// LDS plan: quantity q keeps K(q) plane slots (the write of iteration i goes
// to slot i mod K; a value is read at most K - 1 iterations after it was
// written), each of R(q) rows of 64 lanes.  B0x and B0z have an extra row on
// top (row NW, loaded by the highest wavefront), the axion levels an extra
// row below (row -1, loaded by the lowest).
template <typename T, int NW>
struct M3Lds {
    enum { B0X, B0Z, PA, PB, B1X, B1Z, E0NY, E0HX, E0HY, E0HZ, CY, B0PX, B0PZ, E1X, E1Z, NQ };
    __host__ __device__ static constexpr int K(int q)
    {
        return (q == B0X || q == B0Z || q == B0PX || q == B0PZ) ? 3 : ((q == PB || q == E0HY) ? 4 : 2);
    }
    __host__ __device__ static constexpr int R(int q) { return (q == B0X || q == B0Z || q == PA || q == PB) ? NW + 1 : NW; }
    __host__ __device__ static constexpr int roff(int q) { return (q == PA || q == PB) ? 1 : 0; }
    struct Tab { int v[NQ + 1]; };
    __host__ __device__ static constexpr Tab tab()
    {
        Tab t{};
        int a = 0;
        for (int q = 0; q < NQ; q++) {
            t.v[q] = a;
            a += K(q) * R(q) * 64;
        }
        t.v[NQ] = a;
        return t;
    }
    static constexpr Tab TAB = tab();
    __host__ __device__ static constexpr int base(int q) { return TAB.v[q]; }
    // one spare row: the lane + 1 reads of lane 63 land in it
    static constexpr int ELEMS = TAB.v[NQ] + 64;
    static constexpr size_t BYTES = (size_t)ELEMS * sizeof(T);
};

extern __shared__ __align__(16) unsigned char m3_smem[];

// Occupancy (FP32): 12 wavefronts per workgroup, one workgroup per CU (the
// LDS plan takes about 118 KiB), 3 wavefronts per SIMD.
//
// Values at positions outside a Mur axis's extents (and the axion values
// beyond the ghost cells) are never read by a point inside them: the curl
// and average stencils of a valid point stay inside the extents, or reach
// a ghost, which is computed (E) or loaded (phi) explicitly, and the current
// on a boundary face averages the one interior centre twice.  So the loads
// and intermediate values are not masked; loads of such positions read a
// valid address, and only the stores check the extents.
template <typename T, int NW>
__global__ void __launch_bounds__(64 * NW) k_march3d(const RunK<T> *__restrict__ rp, long step, M3Geom g)
{
    using LQ = M3Lds<T, NW>;
    constexpr int TY = NW - 2;
    T *const lds = reinterpret_cast<T *>(m3_smem);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));

    // ---- the run's geometry and coefficients
    const int n0 = rp->n[0], n1 = rp->n[1], n2 = rp->n[2];
    const int nn0 = rp->nn[0], nn1 = rp->nn[1], nn2 = rp->nn[2];
    const bool mx = rp->mur[0], my = rp->mur[1], mz = rp->mur[2];
    const bool apx = rp->axbc[0] == AXF_AX_PERIODIC, apy = rp->axbc[1] == AXF_AX_PERIODIC;
    const bool apz = rp->axbc[2] == AXF_AX_PERIODIC;
    constexpr unsigned es = sizeof(T);
    const unsigned sxb = (unsigned)rp->sx * es, syb = (unsigned)rp->sy * es;
    const T cdt0 = rp->cdt[0], cdt1 = rp->cdt[1], cdt2 = rp->cdt[2], half = rp->half, inv_dt = rp->inv_dt;
    const T i2x0 = rp->inv2dx[0], i2x1 = rp->inv2dx[1], i2x2 = rp->inv2dx[2];
    const T idx0 = rp->inv_dx2[0], idx1 = rp->inv_dx2[1], idx2 = rp->inv_dx2[2];
    const T dt2 = rp->dt2, m2 = rp->m2, gax = rp->gax, cg1 = rp->cg1;
    const char *const sb = rp->state_base;
    // array stride in bytes and in units of 256 bytes (arrays are 256-byte
    // aligned and sized; the three components of a kind span < 4 GiB: host check)
    const unsigned as32 = (unsigned)rp->arr_stride;
    unsigned as_l = (unsigned)(rp->arr_stride >> 8);
    const int so = em_slot(step), sn = em_slot(step + 1);
    const int la = phi_slot(step), lb = phi_slot(step + 1), ln = phi_slot(step + 2);

    // ---- this workgroup's segment, row group and plane chunk
    unsigned bq = blockIdx.x;
    const int seg = (int)(bq % (unsigned)g.nseg);
    bq /= (unsigned)g.nseg;
    const int ygr = (int)(bq % (unsigned)g.nyg);
    const int zch = (int)(bq / (unsigned)g.nyg);
    const int x0 = seg * g.wid, gx = x0 - 2 + lane;
    const int y0 = ygr * TY, gy = y0 - 1 + w;
    const int z0 = zch * g.zc, z1 = min(z0 + g.zc, nn2);

    // ---- this lane's column
    const int xs_em = mx ? ((gx >= 0 && gx < nn0) ? gx : 0) : m3::imodn(gx, n0);
    // axion column class: 0 a cell (or a periodic axis), 1 / 2 the ghost below / above, 3 none
    const int xcl = apx ? 0 : ((gx >= 0 && gx < n0) ? 0 : (gx == -1 ? 1 : (gx == n0 ? 2 : 3)));
    const int xs_ph = apx ? m3::imodn(gx, n0) : (xcl == 0 ? gx : 0);
    const unsigned xo_em = (unsigned)xs_em * es, xo_ph = (unsigned)xs_ph * es;
    // own columns: nodal x components store there, centred ones where also gx < n0
    const bool own_x = lane >= 2 && lane < 2 + g.wid && gx < nn0;
    const bool own_xc = own_x && (!mx || gx < n0);
    auto own_lane = [&](int l) __attribute__((always_inline)) { return l >= 2 && l < 2 + g.wid && x0 - 2 + l < nn0; };
    // the segment holds a ghost column of an x face (Mur or axion)
    const bool seg_xb = (mx || !apx) && (x0 - 2 <= -1 || x0 + 61 >= n0);
    const T bext0 = bext_at(*rp, 0, xs_em), bext1 = bext_at(*rp, 1, xs_em), bext2 = bext_at(*rp, 2, xs_em);

    // ---- rows (wave-uniform)
    auto ys_em_of = [&](int y) __attribute__((always_inline)) { return my ? ((y >= 0 && y < nn1) ? y : 0) : m3::imodn(y, n1); };
    auto ycl_of = [&](int y) __attribute__((always_inline)) {
        return apy ? 0 : ((y >= 0 && y < n1) ? 0 : (y == -1 ? 1 : (y == n1 ? 2 : 3)));
    };
    auto ys_ph_of = [&](int y) __attribute__((always_inline)) { return apy ? m3::imodn(y, n1) : (ycl_of(y) == 0 ? y : 0); };
    const int ys_em = ys_em_of(gy);
    const unsigned yo_em = (unsigned)ys_em * sxb;
    const unsigned yo_em_up = (unsigned)ys_em_of(gy + 1) * sxb;     // the top wavefront's extra row
    const int ycl_w = ycl_of(gy), ycl_dn = ycl_of(gy - 1);          // axion row classes of the row and the one below
    const int ys_ph_w = ys_ph_of(gy), ys_ph_dn = ys_ph_of(gy - 1);
    const bool own_y = w >= 1 && w <= TY && gy < nn1;
    const bool yc = !my || gy < n1;                     // an own row is a centred-y point too

    // ---- planes (uniform)
    // a plane index is at most 5 planes outside [0, nn2): one wrap suffices
    auto zs_em = [&](int p) __attribute__((always_inline)) {
        return mz ? ((p >= 0 && p < nn2) ? p : 0) : (p < 0 ? p + n2 : (p >= n2 ? p - n2 : p));
    };
    auto zcl_of = [&](int p) __attribute__((always_inline)) {
        return apz ? 0 : ((p >= 0 && p < n2) ? 0 : (p == -1 ? 1 : (p == n2 ? 2 : 3)));
    };
    auto zs_ph = [&](int p) __attribute__((always_inline)) {
        return apz ? (p < 0 ? p + n2 : (p >= n2 ? p - n2 : p)) : (zcl_of(p) == 0 ? p : 0);
    };
    auto own_p = [&](int p) __attribute__((always_inline)) { return p >= z0 && p < z1; };
    auto zc = [&](int p) __attribute__((always_inline)) { return !mz || p < n2; };   // for an own plane
    auto off_em = [&](int p) __attribute__((always_inline)) -> unsigned { return xo_em + yo_em + (unsigned)zs_em(p) * syb; };

    // ---- arrays: the three components of one kind and slot from one base (the
    // stride is re-read at each stage, opaque to the compiler, so that the
    // bases are formed where they are used instead of holding scalar registers)
    auto abase = [&](int q) __attribute__((always_inline)) { return sb + ((unsigned long long)((unsigned)q * as_l) << 8); };
    auto kb_rd = [&](int kind) __attribute__((always_inline)) { return abase(q_em(kind, so, 0)); };
    auto kb_wr = [&](int kind) __attribute__((always_inline)) { return abase(q_em(kind, sn, 0)); };
    auto arr_ph = [&](int L) __attribute__((always_inline)) { return abase(q_phi(L)); };
    auto ld = [&](const char *kb, int c, unsigned off) __attribute__((always_inline)) -> T { return m3::ldo<T>(kb, (unsigned)c * as32 + off); };
    auto st = [&](const char *kb, int c, unsigned off, T v) __attribute__((always_inline)) { m3::sto<T>(kb, (unsigned)c * as32 + off, v); };

    // ---- LDS
    // slot of the write of iteration i - age for quantities of K slots: kept
    // per iteration (k2[a], k3[a], k4[a] = (i - a) mod K)
    int k2[2] = {0, 1}, k3[3] = {0, 2, 1}, k4[4] = {0, 3, 2, 1};
    auto lslot = [&](int K, int age) __attribute__((always_inline)) { return K == 2 ? k2[age] : (K == 3 ? k3[age] : k4[age]); };
    auto lidx = [&](int q, int age, int row) __attribute__((always_inline)) {
        return LQ::base(q) + (lslot(LQ::K(q), age) * LQ::R(q) + row + LQ::roff(q)) * 64;
    };
    auto lw = [&](int q, int age, int row, T v) __attribute__((always_inline)) { lds[lidx(q, age, row) + lane] = v; };
    auto lr = [&](int q, int age, int row) __attribute__((always_inline)) -> T { return lds[lidx(q, age, row) + lane]; };
    auto lr1 = [&](int q, int age, int row) __attribute__((always_inline)) -> T { return lds[lidx(q, age, row) + lane + 1]; };
    const int wlo = w > 0 ? w - 1 : 0;   // the row below (the lowest wavefront reads its own: never used)

    // ---- axion level L of row y, plane p: the array, or the y / z ghost plane
    // for a ghost row / plane; in segments with x ghost columns also the x
    // ghost plane, which phi_take picks for those columns
    struct PhiRaw { T a, fx; };
    auto phi_load = [&](int L, int ycl, int ys, int p) __attribute__((always_inline)) -> PhiRaw {
        PhiRaw r{T(0), T(0)};
        const int zcl = zcl_of(p), zs = zs_ph(p);
        if (zcl == 1 || zcl == 2) {
            r.a = m3::fld(rp, q_axg(2, zcl - 1, L), (long)ys * nn0 + xs_ph);
        } else if (ycl == 1 || ycl == 2) {
            r.a = m3::fld(rp, q_axg(1, ycl - 1, L), (long)zs * nn0 + xs_ph);
        } else {
            r.a = m3::ldo<T>(arr_ph(L), xo_ph + (unsigned)ys * sxb + (unsigned)zs * syb);
            if (seg_xb && !apx) r.fx = m3::fld(rp, q_axg(0, xcl == 2 ? 1 : 0, L), (long)zs * nn1 + ys);
        }
        return r;
    };
    auto phi_take = [&](const PhiRaw& r, int ycl, int p) __attribute__((always_inline)) -> T {
        if (!(seg_xb && !apx) || ycl != 0 || zcl_of(p) != 0) return r.a;
        return (xcl == 1 || xcl == 2) ? r.fx : r.a;
    };

    // ---- register windows along z (suffix k = plane i - k of iteration i)
    T b0_0[3] = {0, 0, 0}, b0_1[3] = {0, 0, 0}, b0_2[3] = {0, 0, 0};
    T pa_1 = 0, pa_2 = 0, pa_3 = 0, pa_4 = 0;
    T pb_1 = 0, pb_2 = 0, pb_3 = 0, pb_4 = 0, pb_5 = 0;
    T e0n_1[3] = {0, 0, 0}, e0n_2[3] = {0, 0, 0};
    T e0h_1[3] = {0, 0, 0}, e0h_2[3] = {0, 0, 0}, e0h_3[3] = {0, 0, 0}, e0h_4[3] = {0, 0, 0};
    T c_2[3] = {0, 0, 0}, c_3[3] = {0, 0, 0}, c_4z = 0;
    T bo_2[3] = {0, 0, 0}, bo_3[3] = {0, 0, 0}, bo_4[3] = {0, 0, 0};
    T b0p_2[3] = {0, 0, 0}, b0p_3[3] = {0, 0, 0}, b0p_4[3] = {0, 0, 0};
    T b1_2[3] = {0, 0, 0}, b1_3[3] = {0, 0, 0}, b1_4[3] = {0, 0, 0};
    T e1h_3[3] = {0, 0, 0}, e1h_4[3] = {0, 0, 0}, e1h_5[2] = {0, 0};

    // values loaded one iteration ahead
    struct Pre {
        T b0[3], e0[3], b1[3], e1[3], xb0x, xb0z;
        PhiRaw pa, pb, xpa, xpb;
    };
    Pre P;
#pragma unroll
    for (int c = 0; c < 3; c++) P.b0[c] = P.e0[c] = P.b1[c] = P.e1[c] = T(0);
    P.xb0x = P.xb0z = T(0);
    P.pa = P.pb = P.xpa = P.xpb = PhiRaw{T(0), T(0)};
    // first and last iterations of the march, and the iterations each load
    // group and stage is needed in (no owned value depends on the others)
    const int i_first = z0 - 2, i_last = z1 + 3;
    auto prefetch = [&](int i) __attribute__((always_inline)) {
        asm volatile("" : "+s"(as_l));
        if (i <= z1 + 1) {                       // B0 of plane i, axion levels of plane i - 1
            const char *kb = kb_rd(1);
            const unsigned o = off_em(i);
#pragma unroll
            for (int c = 0; c < 3; c++) P.b0[c] = ld(kb, c, o);
            P.pa = phi_load(la, ycl_w, ys_ph_w, i - 1);
            P.pb = phi_load(lb, ycl_w, ys_ph_w, i - 1);
            if (w == NW - 1) {
                const unsigned ox = xo_em + yo_em_up + (unsigned)zs_em(i) * syb;
                P.xb0x = ld(kb, 0, ox);
                P.xb0z = ld(kb, 2, ox);
            }
            if (w == 0) {
                P.xpa = phi_load(la, ycl_dn, ys_ph_dn, i - 1);
                P.xpb = phi_load(lb, ycl_dn, ys_ph_dn, i - 1);
            }
        }
        if (i >= z0 - 1 && i <= z1 + 1) {       // E0^{n-1/2} of plane i - 1
            const char *kb = kb_rd(0);
            const unsigned o = off_em(i - 1);
#pragma unroll
            for (int c = 0; c < 3; c++) P.e0[c] = ld(kb, c, o);
        }
        if (i >= z0 + 1 && i <= z1 + 2) {       // B1 of plane i - 2
            const char *kb = kb_rd(3);
            const unsigned o = off_em(i - 2);
#pragma unroll
            for (int c = 0; c < 3; c++) P.b1[c] = ld(kb, c, o);
        }
        if (i >= z0 + 2 && i <= z1 + 2) {       // E1^{n-1/2} of plane i - 3
            const char *kb = kb_rd(2);
            const unsigned o = off_em(i - 3);
#pragma unroll
            for (int c = 0; c < 3; c++) P.e1[c] = ld(kb, c, o);
        }
    };

    // Mur ghost (order O, component c, axis d, side) of face point fidx from
    // the adjacent point's E^{n-1/2} and E^{n+1/2}
    auto mur = [&](int O, int c, int d, int side, T e_old, T e_new, long fidx) __attribute__((always_inline)) -> T {
        const double g_old = (double)m3::fld(rp, q_mur(O, d, side, c, so), fidx);
        return mur_update_rk<T>(*rp, O, c, d, side, (double)e_old, (double)e_new, g_old, fidx, step);
    };

    prefetch(i_first);
    for (int i = i_first; i <= i_last; i++) {
        // rotate the LDS slots: slot of iteration i for each K (the first
        // iteration's slots are the initial ones)
        if (i > i_first) {
            k2[1] = k2[0]; k2[0] ^= 1;
            k3[2] = k3[1]; k3[1] = k3[0]; k3[0] = k3[0] == 2 ? 0 : k3[0] + 1;
            k4[3] = k4[2]; k4[2] = k4[1]; k4[1] = k4[0]; k4[0] = (k4[0] + 1) & 3;
        }
        // ---- rotate the windows and take in the loads of this iteration
#pragma unroll
        for (int c = 0; c < 3; c++) {
            b0_2[c] = b0_1[c];
            b0_1[c] = b0_0[c];
            e0n_2[c] = e0n_1[c];
            e0h_4[c] = e0h_3[c];
            e0h_3[c] = e0h_2[c];
            e0h_2[c] = e0h_1[c];
            bo_4[c] = bo_3[c];
            bo_3[c] = bo_2[c];
            b0p_4[c] = b0p_3[c];
            b0p_3[c] = b0p_2[c];
            b1_4[c] = b1_3[c];
            b1_3[c] = b1_2[c];
        }
        c_4z = c_3[2];
#pragma unroll
        for (int c = 0; c < 3; c++) c_3[c] = c_2[c];
        e1h_5[0] = e1h_4[0];
        e1h_5[1] = e1h_4[1];
#pragma unroll
        for (int c = 0; c < 3; c++) e1h_4[c] = e1h_3[c];
        pa_4 = pa_3; pa_3 = pa_2; pa_2 = pa_1;
        pb_5 = pb_4; pb_4 = pb_3; pb_3 = pb_2; pb_2 = pb_1;

        const int p1 = i - 1, p2 = i - 2, p3 = i - 3, p4 = i - 4;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            b0_0[c] = P.b0[c];
            b1_2[c] = P.b1[c];
        }
        pa_1 = phi_take(P.pa, ycl_w, p1);
        pb_1 = phi_take(P.pb, ycl_w, p1);
        const T xb0x = P.xb0x, xb0z = P.xb0z;
        T xpa = T(0), xpb = T(0);
        if (w == 0) {
            xpa = phi_take(P.xpa, ycl_dn, p1);
            xpb = phi_take(P.xpb, ycl_dn, p1);
        }
        const T e0o[3] = {P.e0[0], P.e0[1], P.e0[2]};
        const T e1o[3] = {P.e1[0], P.e1[1], P.e1[2]};
        if (i < i_last) prefetch(i + 1);

        // ---- loaded values the neighbouring rows read
        lw(LQ::B0X, 0, w, b0_0[0]);
        lw(LQ::B0Z, 0, w, b0_0[2]);
        lw(LQ::PA, 0, w, pa_1);
        lw(LQ::PB, 0, w, pb_1);
        lw(LQ::B1X, 0, w, b1_2[0]);
        lw(LQ::B1Z, 0, w, b1_2[2]);
        if (w == NW - 1) {
            lw(LQ::B0X, 0, NW, xb0x);
            lw(LQ::B0Z, 0, NW, xb0z);
        }
        if (w == 0) {
            lw(LQ::PA, 0, -1, xpa);
            lw(LQ::PB, 0, -1, xpb);
        }

        // ================================================ S1: E0 at plane p1
        asm volatile("" : "+s"(as_l));
        if (i >= z0 - 1 && i <= z1 + 1) {
            const T b0z_y = lr(LQ::B0Z, 1, w + 1), b0x_y = lr(LQ::B0X, 1, w + 1);
            const T b0z_x = m3::lane_up(b0_1[2]), b0y_x = m3::lane_up(b0_1[1]);
            T eh[3], en[3];
            {
                T a = cdt1 * (b0z_y - b0_1[2]), b = cdt2 * (b0_0[1] - b0_1[1]);
                T rhs = a - b;
                eh[0] = e0o[0] + T(1) * rhs;
            }
            {
                T a = cdt2 * (b0_0[0] - b0_1[0]), b = cdt0 * (b0z_x - b0_1[2]);
                T rhs = a - b;
                eh[1] = e0o[1] + T(1) * rhs;
            }
            {
                T a = cdt0 * (b0y_x - b0_1[1]), b = cdt1 * (b0x_y - b0_1[0]);
                T rhs = a - b;
                eh[2] = e0o[2] + T(1) * rhs;
            }
#pragma unroll
            for (int c = 0; c < 3; c++) en[c] = half * (e0o[c] + eh[c]);
            if (own_y && own_p(p1)) {
                const char *kb = kb_wr(0);
                const unsigned o = off_em(p1);
                if (yc && zc(p1) && own_x) st(kb, 0, o, eh[0]);
                if (zc(p1) && own_xc) st(kb, 1, o, eh[1]);
                if (yc && own_xc) st(kb, 2, o, eh[2]);
            }
            // Mur ghosts across x of E0y (nodal y, centred z) and E0z (centred y, nodal z)
            if (mx && seg_xb) {
                const T up_y = m3::lane_up(eh[1]), dn_y = m3::lane_dn(eh[1]), up_z = m3::lane_up(eh[2]), dn_z = m3::lane_dn(eh[2]);
                const T oup_y = m3::lane_up(e0o[1]), odn_y = m3::lane_dn(e0o[1]);
                const T oup_z = m3::lane_up(e0o[2]), odn_z = m3::lane_dn(e0o[2]);
                if (gx == -1 || gx == n0) {
                    const int side = gx == -1 ? 0 : 1;
                    const bool owner = own_lane(side ? lane - 1 : lane + 1) && own_y && own_p(p1);
                    const long f = (long)zs_em(p1) * nn1 + ys_em;
                    const T vy = mur(0, 1, 0, side, side ? odn_y : oup_y, side ? dn_y : up_y, f);
                    const T vz = mur(0, 2, 0, side, side ? odn_z : oup_z, side ? dn_z : up_z, f);
                    eh[1] = vy;
                    eh[2] = vz;
                    if (owner && zc(p1)) m3::fst(rp, q_mur(0, 0, side, 1, sn), f, vy);
                    if (owner && yc) m3::fst(rp, q_mur(0, 0, side, 2, sn), f, vz);
                }
            }
            // Mur ghosts across z of E0x (nodal x, centred y) and E0y (centred x, nodal y);
            // stored by the chunk of plane 0, or of the nodal plane n2 (which
            // always computes this ghost; the chunk of plane n2 - 1 may not)
            if (mz && (p1 == 0 || p1 == n2)) {
                const int side = p1 == 0 ? 0 : 1;
                const bool owner = own_y && own_p(side ? n2 : 0);
                const long f = (long)ys_em * nn0 + xs_em;
                const char *kb = kb_rd(0);
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    T e_old = side ? ld(kb, c, off_em(n2 - 1)) : e0o[c];
                    T e_new = side ? e0h_2[c] : eh[c];
                    T v = mur(0, c, 2, side, e_old, e_new, f);
                    if (side) eh[c] = v;
                    else e0h_2[c] = v;
                    if (owner && (c == 0 ? yc && own_x : own_xc)) m3::fst(rp, q_mur(0, 2, side, c, sn), f, v);
                }
            }
            // Mur ghosts below the y face of E0x (nodal x, centred z) and E0z
            // (centred x, nodal z): row 0 computes them and puts them in the LDS
            // row below, which the row -1 wavefront leaves to it; the top face's
            // are computed by row n1, where they are used (S3)
            if (my && gy == 0) {
                const bool owner = own_p(p1);
                const long f = (long)zs_em(p1) * nn0 + xs_em;
                const T gxv = mur(0, 0, 1, 0, e0o[0], eh[0], f);
                const T gzv = mur(0, 2, 1, 0, e0o[2], eh[2], f);
                if (owner && zc(p1) && own_x) m3::fst(rp, q_mur(0, 1, 0, 0, sn), f, gxv);
                if (owner && own_xc) m3::fst(rp, q_mur(0, 1, 0, 2, sn), f, gzv);
                lw(LQ::E0HX, 0, w - 1, gxv);
                lw(LQ::E0HZ, 0, w - 1, gzv);
            }
#pragma unroll
            for (int c = 0; c < 3; c++) {
                e0h_1[c] = eh[c];
                e0n_1[c] = en[c];
            }
            lw(LQ::E0NY, 0, w, en[1]);
            lw(LQ::E0HY, 0, w, eh[1]);
            if (!(my && gy == -1)) {
                lw(LQ::E0HX, 0, w, eh[0]);
                lw(LQ::E0HZ, 0, w, eh[2]);
            }
        }

        // ================================================ S2: C at the cells of plane p2
        if (w <= NW - 2 && i >= z0 && i <= z1 + 1) {
            T e[3], bb[3], gp[3], bo[3];
            e[0] = half * (e0n_2[0] + m3::lane_up(e0n_2[0]));
            e[1] = half * (e0n_2[1] + lr(LQ::E0NY, 1, w + 1));
            e[2] = half * (e0n_2[2] + e0n_1[2]);
            const T bxy0 = lr(LQ::B0X, 2, w + 1), bxy1 = lr(LQ::B0X, 1, w + 1);
            const T bzy = lr(LQ::B0Z, 2, w + 1), bzyx = lr1(LQ::B0Z, 2, w + 1);
            bo[0] = T(0.25) * ((b0_2[0] + bxy0) + (b0_1[0] + bxy1));
            bo[1] = T(0.25) * ((b0_2[1] + m3::lane_up(b0_2[1])) + (b0_1[1] + m3::lane_up(b0_1[1])));
            bo[2] = T(0.25) * ((b0_2[2] + m3::lane_up(b0_2[2])) + (bzy + bzyx));
            bb[0] = bo[0] + bext0;
            bb[1] = bo[1] + bext1;
            bb[2] = bo[2] + bext2;
            T dtphi = (pb_2 - pa_2) * inv_dt;
            {
                T up = half * (m3::lane_up(pa_2) + m3::lane_up(pb_2)), dn = half * (m3::lane_dn(pa_2) + m3::lane_dn(pb_2));
                gp[0] = (up - dn) * i2x0;
            }
            {
                T up = half * (lr(LQ::PA, 1, w + 1) + lr(LQ::PB, 1, w + 1));
                T dn = half * (lr(LQ::PA, 1, w - 1) + lr(LQ::PB, 1, w - 1));
                gp[1] = (up - dn) * i2x1;
            }
            {
                T up = half * (pa_1 + pb_1), dn = half * (pa_3 + pb_3);
                gp[2] = (up - dn) * i2x2;
            }
            c_2[0] = dtphi * bb[0] - (e[1] * gp[2] - e[2] * gp[1]);
            c_2[1] = dtphi * bb[1] - (e[2] * gp[0] - e[0] * gp[2]);
            c_2[2] = dtphi * bb[2] - (e[0] * gp[1] - e[1] * gp[0]);
#pragma unroll
            for (int c = 0; c < 3; c++) bo_2[c] = bo[c];
            lw(LQ::CY, 0, w, c_2[1]);
        }

        // ================================================ S3: B0^{n+1} at plane p2
        asm volatile("" : "+s"(as_l));
        if (w >= 1 && i >= z0 + 2 && i <= z1 + 2) {
            const T exm = lr(LQ::E0HX, 1, w - 1), ezm = lr(LQ::E0HZ, 1, w - 1);
            T ex = e0h_2[0], ez = e0h_2[2];
            const bool ownr = own_y && own_p(p2);
            if (my && gy == n1) {
                // the Mur ghosts above the top y face, from row n1 - 1's E0x, E0z
                const long f = (long)zs_em(p2) * nn0 + xs_em;
                const unsigned om = xo_em + (unsigned)(n1 - 1) * sxb + (unsigned)zs_em(p2) * syb;
                const char *kb = kb_rd(0);
                ex = mur(0, 0, 1, 1, ld(kb, 0, om), exm, f);
                ez = mur(0, 2, 1, 1, ld(kb, 2, om), ezm, f);
                if (ownr && zc(p2) && own_x) m3::fst(rp, q_mur(0, 1, 1, 0, sn), f, ex);
                if (ownr && own_xc) m3::fst(rp, q_mur(0, 1, 1, 2, sn), f, ez);
            }
            T v[3];
            {
                T a = cdt1 * (ez - ezm), b = cdt2 * (e0h_2[1] - e0h_3[1]);
                v[0] = b0_2[0] - (a - b);
            }
            {
                T a = cdt2 * (ex - e0h_3[0]), b = cdt0 * (ez - m3::lane_dn(ez));
                v[1] = b0_2[1] - (a - b);
            }
            {
                T a = cdt0 * (e0h_2[1] - m3::lane_dn(e0h_2[1])), b = cdt1 * (ex - exm);
                v[2] = b0_2[2] - (a - b);
            }
            if (ownr) {
                const char *kb = kb_wr(1);
                const unsigned o = off_em(p2);
                if (own_xc) st(kb, 0, o, v[0]);
                if (yc && own_x) st(kb, 1, o, v[1]);
                if (zc(p2) && own_x) st(kb, 2, o, v[2]);
            }
#pragma unroll
            for (int c = 0; c < 3; c++) b0p_2[c] = v[c];
            lw(LQ::B0PX, 0, w, v[0]);
            lw(LQ::B0PZ, 0, w, v[2]);
        }

        // ================================================ S4: E1 at plane p3
        asm volatile("" : "+s"(as_l));
        if (w <= NW - 2 && i >= z0 + 2 && i <= z1 + 2) {
            const T b1z_y = lr(LQ::B1Z, 1, w + 1), b1x_y = lr(LQ::B1X, 1, w + 1);
            const T cym = lr(LQ::CY, 1, wlo);
            const T dn_cx = m3::lane_dn(c_3[0]);
            T eh[3];
            {
                T lo = (mx && gx - 1 < 0) ? c_3[0] : dn_cx;
                T hi = (mx && gx > n0 - 1) ? dn_cx : c_3[0];
                T Sc = half * (lo + hi);
                T a = cdt1 * (b1z_y - b1_3[2]), b = cdt2 * (b1_2[1] - b1_3[1]);
                T rhs = (a - b) - cg1 * Sc;
                eh[0] = e1o[0] + T(1) * rhs;
            }
            {
                T lo = (my && gy - 1 < 0) ? c_3[1] : cym;
                T hi = (my && gy > n1 - 1) ? cym : c_3[1];
                T Sc = half * (lo + hi);
                T a = cdt2 * (b1_2[0] - b1_3[0]), b = cdt0 * (m3::lane_up(b1_3[2]) - b1_3[2]);
                T rhs = (a - b) - cg1 * Sc;
                eh[1] = e1o[1] + T(1) * rhs;
            }
            {
                T lo = (mz && p3 - 1 < 0) ? c_3[2] : c_4z;
                T hi = (mz && p3 > n2 - 1) ? c_4z : c_3[2];
                T Sc = half * (lo + hi);
                T a = cdt0 * (m3::lane_up(b1_3[1]) - b1_3[1]), b = cdt1 * (b1x_y - b1_3[0]);
                T rhs = (a - b) - cg1 * Sc;
                eh[2] = e1o[2] + T(1) * rhs;
            }
            if (own_y && own_p(p3)) {
                const char *kb = kb_wr(2);
                const unsigned o = off_em(p3);
                if (yc && zc(p3) && own_x) st(kb, 0, o, eh[0]);
                if (zc(p3) && own_xc) st(kb, 1, o, eh[1]);
                if (yc && own_xc) st(kb, 2, o, eh[2]);
            }
            if (mx && seg_xb) {
                const T up_y = m3::lane_up(eh[1]), dn_y = m3::lane_dn(eh[1]), up_z = m3::lane_up(eh[2]), dn_z = m3::lane_dn(eh[2]);
                const T oup_y = m3::lane_up(e1o[1]), odn_y = m3::lane_dn(e1o[1]);
                const T oup_z = m3::lane_up(e1o[2]), odn_z = m3::lane_dn(e1o[2]);
                if (gx == -1 || gx == n0) {
                    const int side = gx == -1 ? 0 : 1;
                    const bool owner = own_lane(side ? lane - 1 : lane + 1) && own_y && own_p(p3);
                    const long f = (long)zs_em(p3) * nn1 + ys_em;
                    const T vy = mur(1, 1, 0, side, side ? odn_y : oup_y, side ? dn_y : up_y, f);
                    const T vz = mur(1, 2, 0, side, side ? odn_z : oup_z, side ? dn_z : up_z, f);
                    eh[1] = vy;
                    eh[2] = vz;
                    if (owner && zc(p3)) m3::fst(rp, q_mur(1, 0, side, 1, sn), f, vy);
                    if (owner && yc) m3::fst(rp, q_mur(1, 0, side, 2, sn), f, vz);
                }
            }
            if (mz && (p3 == 0 || p3 == n2)) {
                const int side = p3 == 0 ? 0 : 1;
                const bool owner = own_y && own_p(side ? n2 : 0);
                const long f = (long)ys_em * nn0 + xs_em;
                const char *kb = kb_rd(2);
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    T e_old = side ? ld(kb, c, off_em(n2 - 1)) : e1o[c];
                    T e_new = side ? e1h_4[c] : eh[c];
                    T v = mur(1, c, 2, side, e_old, e_new, f);
                    if (side) eh[c] = v;
                    else e1h_4[c] = v;
                    if (owner && (c == 0 ? yc && own_x : own_xc)) m3::fst(rp, q_mur(1, 2, side, c, sn), f, v);
                }
            }
            if (my && gy == 0) {
                const bool owner = own_p(p3);
                const long f = (long)zs_em(p3) * nn0 + xs_em;
                const T gxv = mur(1, 0, 1, 0, e1o[0], eh[0], f);
                const T gzv = mur(1, 2, 1, 0, e1o[2], eh[2], f);
                if (owner && zc(p3) && own_x) m3::fst(rp, q_mur(1, 1, 0, 0, sn), f, gxv);
                if (owner && own_xc) m3::fst(rp, q_mur(1, 1, 0, 2, sn), f, gzv);
                lw(LQ::E1X, 0, w - 1, gxv);
                lw(LQ::E1Z, 0, w - 1, gzv);
            }
#pragma unroll
            for (int c = 0; c < 3; c++) e1h_3[c] = eh[c];
            if (!(my && gy == -1)) {
                lw(LQ::E1X, 0, w, eh[0]);
                lw(LQ::E1Z, 0, w, eh[2]);
            }
        }

        // ================================================ S5, S6 at plane p4 (own rows)
        asm volatile("" : "+s"(as_l));
        if (own_y && i >= z0 + 4 && i <= z1 + 3) {
            const bool ownp = own_p(p4);
            // ---- S5: B1^{n+1}
            {
                const T exm = lr(LQ::E1X, 1, w - 1), ezm = lr(LQ::E1Z, 1, w - 1);
                T ex = e1h_4[0], ez = e1h_4[2];
                if (my && gy == n1) {
                    const long f = (long)zs_em(p4) * nn0 + xs_em;
                    const unsigned om = xo_em + (unsigned)(n1 - 1) * sxb + (unsigned)zs_em(p4) * syb;
                    const char *kb = kb_rd(2);
                    ex = mur(1, 0, 1, 1, ld(kb, 0, om), exm, f);
                    ez = mur(1, 2, 1, 1, ld(kb, 2, om), ezm, f);
                    if (ownp && zc(p4) && own_x) m3::fst(rp, q_mur(1, 1, 1, 0, sn), f, ex);
                    if (ownp && own_xc) m3::fst(rp, q_mur(1, 1, 1, 2, sn), f, ez);
                }
                T v[3];
                {
                    T a = cdt1 * (ez - ezm), b = cdt2 * (e1h_4[1] - e1h_5[1]);
                    v[0] = b1_4[0] - (a - b);
                }
                {
                    T a = cdt2 * (ex - e1h_5[0]), b = cdt0 * (ez - m3::lane_dn(ez));
                    v[1] = b1_4[1] - (a - b);
                }
                {
                    T a = cdt0 * (e1h_4[1] - m3::lane_dn(e1h_4[1])), b = cdt1 * (ex - exm);
                    v[2] = b1_4[2] - (a - b);
                }
                if (ownp) {
                    const char *kb = kb_wr(3);
                    const unsigned o = off_em(p4);
                    if (own_xc) st(kb, 0, o, v[0]);
                    if (yc && own_x) st(kb, 1, o, v[1]);
                    if (zc(p4) && own_x) st(kb, 2, o, v[2]);
                }
            }
            // ---- S6: phi^{n+3/2} at the cells
            {
                T e[3], bb[3], bn[3];
                e[0] = half * (e0h_4[0] + m3::lane_up(e0h_4[0]));
                e[1] = half * (e0h_4[1] + lr(LQ::E0HY, 3, w + 1));
                e[2] = half * (e0h_4[2] + e0h_3[2]);
                bn[0] = T(0.25) * ((b0p_4[0] + lr(LQ::B0PX, 2, w + 1)) + (b0p_3[0] + lr(LQ::B0PX, 1, w + 1)));
                bn[1] = T(0.25) * ((b0p_4[1] + m3::lane_up(b0p_4[1])) + (b0p_3[1] + m3::lane_up(b0p_3[1])));
                bn[2] = T(0.25) * ((b0p_4[2] + m3::lane_up(b0p_4[2])) + (lr(LQ::B0PZ, 2, w + 1) + lr1(LQ::B0PZ, 2, w + 1)));
                bb[0] = half * (bo_4[0] + bn[0]) + bext0;
                bb[1] = half * (bo_4[1] + bn[1]) + bext1;
                bb[2] = half * (bo_4[2] + bn[2]) + bext2;
                T sax = gax * (e[0] * bb[0] + e[1] * bb[1] + e[2] * bb[2]);
                T pa = pa_4, pb = pb_4;
                T lap = T(0);
                lap += ((m3::lane_up(pb_4) - T(2) * pb) + m3::lane_dn(pb_4)) * idx0;
                lap += ((lr(LQ::PB, 3, w + 1) - T(2) * pb) + lr(LQ::PB, 3, w - 1)) * idx1;
                lap += ((pb_3 - T(2) * pb) + pb_5) * idx2;
                const int gz = zs_em(p4);
                const bool pml = rp->axbc[0] == AXF_AX_PML || rp->axbc[1] == AXF_AX_PML || rp->axbc[2] == AXF_AX_PML;
                T sdt = pml ? pml_sdt<3>(*rp, xs_em, ys_em, gz) : T(0);
                T xq = dt2 * ((sax - m2 * pb) + lap) - sdt * sdt * pb;
                T pn = ((xq + sdt * pa) + T(2) * pb) - pa;
                if (sdt != T(0)) pn = pn / (T(1) + sdt);
                if (ownp && yc && zc(p4) && own_xc) {
                    m3::sto<T>(arr_ph(ln), xo_em + yo_em + (unsigned)gz * syb, pn);
                    // axion ghosts of the new level at the boundary cells
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        if (rp->axbc[d] == AXF_AX_PERIODIC) continue;
                        const int gv = d == 0 ? xs_em : (d == 1 ? ys_em : gz);
#pragma unroll
                        for (int side = 0; side < 2; side++) {
                            if (gv != (side ? rp->n[d] - 1 : 0)) continue;
                            const long f = d == 0 ? (long)gz * nn1 + ys_em : (d == 1 ? (long)gz * nn0 + xs_em : (long)ys_em * nn0 + xs_em);
                            T gval;
                            if (rp->axbc[d] == AXF_AX_OUTFLOW) {
                                T gbv = m3::fld(rp, q_axg(d, side, lb), f), gav = m3::fld(rp, q_axg(d, side, la), f);
                                T rr = rp->out_r[d];
                                T xx = (((T(-2) * gbv + T(2) * gav) - dt2 * (sax - m2 * gbv)) + rr * pb - rr * rr * (pb - T(2) * gbv))
                                       / (rr + rr * rr);
                                gval = gav + rr * (pb - xx);
                            } else {
                                gval = pn;
                            }
                            m3::fst(rp, q_axg(d, side, ln), f, gval);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side

template <typename T> struct March3 { static constexpr int NW = sizeof(T) == 4 ? AXF_M3_NW : 8; };


template <typename T>
static M3Geom march3d_geom(const RunK<T>& h, int zc)
{
    constexpr int TY = March3<T>::NW - 2;
    M3Geom g;
    g.nseg = (h.nn[0] + 59) / 60;
    g.wid = (h.nn[0] + g.nseg - 1) / g.nseg;
    g.nyg = (h.nn[1] + TY - 1) / TY;
    g.zc = zc > 0 ? zc : 64;
    g.nzc = (h.nn[2] + g.zc - 1) / g.zc;
    return g;
}

template <typename T>
bool march3d_available(const RunK<T>& h)
{
    // 32-bit byte offsets within one array
    return h.D == 3 && (unsigned long long)h.arr_stride < (1ull << 32);
}

template <typename T>
long march3d_blocks(const RunK<T>& h, int zc)
{
    M3Geom g = march3d_geom(h, zc);
    return (long)g.nseg * g.nyg * g.nzc;
}

template <typename T>
hipError_t launch_march3d(const RunK<T> *rk, const RunK<T>& h, long step, int zc, hipStream_t st)
{
    constexpr int NW = March3<T>::NW;
    using LQ = M3Lds<T, NW>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_march3d<T, NW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)LQ::BYTES);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const M3Geom g = march3d_geom(h, zc);
    const long nb = (long)g.nseg * g.nyg * g.nzc;
    hipLaunchKernelGGL((k_march3d<T, NW>), dim3((unsigned)nb), dim3(64 * NW), LQ::BYTES, st, rk, step, g);
    return hipGetLastError();
}

template bool march3d_available<float>(const RunK<float>&);
template bool march3d_available<double>(const RunK<double>&);
template long march3d_blocks<float>(const RunK<float>&, int);
template long march3d_blocks<double>(const RunK<double>&, int);
template hipError_t launch_march3d<float>(const RunK<float> *, const RunK<float>&, long, int, hipStream_t);
template hipError_t launch_march3d<double>(const RunK<double> *, const RunK<double>&, long, int, hipStream_t);

}  // namespace axf
