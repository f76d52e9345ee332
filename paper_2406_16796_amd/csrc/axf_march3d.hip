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

#include <stdlib.h>

#include <type_traits>

#ifndef AXF_M3_NW
#define AXF_M3_NW 8
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
// element i of a wave-uniform address through the scalar cache (data the
// launch does not write: old ghost levels, the laser table)
template <typename T>
__device__ __forceinline__ T sld(const char *base, long i)
{
    return ((const __attribute__((address_space(4))) T *)base)[i];
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
        return (q == B0X || q == B0Z || q == B0PX || q == B0PZ || q == PB || q == E0HY) ? 4 : 2;
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

// x-face launch: the face values its rows and planes read, staged in LDS
// behind the quantities' slots when a block starts.  Per plane p in
// [z0 - 6, z1 + 2] and row y in [y0 - 2, y0 + NW - 2] one record of NT values
// of T (the axion ghosts of levels la and lb, the Mur ghosts of E0y, E0z,
// E1y, E1z, each for x_min then x_max) and, in a second array, four doubles
// (the laser table's values at that face point for t_n and t_n+1).  FP32 only:
// beside the FP64 slots the records of a chunk do not fit.
template <typename T, int NW>
struct M3Face {
    static constexpr int NT = 12, ROWS = NW + 1, LAG_LO = 6, LAG_HI = 2;
    static constexpr size_t PLANE = (size_t)ROWS * (NT * sizeof(T) + 4 * sizeof(double));
    static constexpr size_t LDS_MAX = 160 * 1024;
    static constexpr int NP_MAX = M3Lds<T, NW>::BYTES < LDS_MAX ? (int)((LDS_MAX - M3Lds<T, NW>::BYTES) / PLANE) : 0;
    static constexpr bool ON = sizeof(T) == 4;
    // planes staged by a block of chunk [z0, z1)
    __host__ __device__ static constexpr int planes(int z0, int z1) { return z1 - z0 + LAG_LO + LAG_HI + 1; }
    static constexpr size_t bytes(int np) { return M3Lds<T, NW>::BYTES + (size_t)np * PLANE; }
};

extern __shared__ __align__(16) unsigned char m3_smem[];

// first plane of chunk k: chunk 0 is [0, zf), chunks 1 .. nzc - 2 split
// [zf, zend) into pieces of zi planes, chunk nzc - 1 is [zend, nn2)
__host__ __device__ inline int m3_zb(const M3Geom& g, int k)
{
    if (k <= 0) return 0;
    if (k >= g.nzc) return g.nn2;
    if (k == g.nzc - 1) return g.zend;
    return min(g.zf + (k - 1) * g.zi, g.zend);
}

// segment, row group and chunk of block b.  The interior launch (mode 0)
// covers the box of segments [sx0, sx1), row groups [gy0, gy1) and chunks
// 1 .. nzc - 2.  (C) the inner chunks of those row groups in the columns
// outside the interior segments are the x-face launch (mode 1) when g.xb is
// set: one block per row group and chunk, whose wavefronts hold the columns
// of both x faces.  The frame launch (mode 2) takes the rest in segments of
// wid columns: (A) the first and last chunks of every segment and row group,
// (B) the inner chunks of the row groups outside [gy0, gy1), and (C) when
// there is no x-face launch, in which case the interior segments are those of
// the frame's split.
__host__ __device__ inline void m3_block(const M3Geom& g, int mode, unsigned b, int& seg, int& ygr, int& zch)
{
    const unsigned nsx = (unsigned)(g.sx1 - g.sx0), ny = (unsigned)(g.gy1 - g.gy0), nzi = (unsigned)(g.nzc - 2);
    if (mode == 1) {
        // row groups fastest (a block's only neighbours here are along y),
        // with a band of the order per XCD as in the interior launch
        if (g.order & 2) b = (unsigned)xcd_band((long)b, (long)(ny * nzi));
        ygr = g.gy0 + (int)(b % ny);
        seg = 0;
        zch = 1 + (int)(b / ny);
        return;
    }
    if (mode == 0) {
        // order & 2: the hardware deals blocks to the 8 XCDs in turn; give
        // each XCD one contiguous band of the block order instead.
        // order & 1: row groups fastest (the blocks that share halo rows run
        // together) instead of segments fastest.
        const unsigned nb = nsx * ny * nzi;
        if (g.order & 2) b = (unsigned)xcd_band((long)b, (long)nb);
        if (g.order & 1) {
            ygr = g.gy0 + (int)(b % ny);
            const unsigned r = b / ny;
            seg = g.sx0 + (int)(r % nsx);
            zch = 1 + (int)(r / nsx);
        } else {
            seg = g.sx0 + (int)(b % nsx);
            const unsigned r = b / nsx;
            ygr = g.gy0 + (int)(r % ny);
            zch = 1 + (int)(r / ny);
        }
        return;
    }
    const unsigned nseg = (unsigned)g.nseg, nyg = (unsigned)g.nyg;
    const unsigned na = (g.nzc > 1 ? 2u : 1u) * nseg * nyg;
    if (b < na) {
        seg = (int)(b % nseg);
        const unsigned r = b / nseg;
        ygr = (int)(r % nyg);
        zch = r < nyg ? 0 : g.nzc - 1;
        return;
    }
    b -= na;
    const unsigned nfy = nyg - ny, nb = nseg * nfy * nzi;
    if (b < nb) {
        seg = (int)(b % nseg);
        const unsigned r = b / nseg;
        const int k = (int)(r % nfy);
        ygr = k < g.gy0 ? k : g.gy1 + (k - g.gy0);
        zch = 1 + (int)(r / nfy);
        return;
    }
    b -= nb;
    const unsigned nfx = nseg - nsx;
    const int k = (int)(b % nfx);
    seg = k < g.sx0 ? k : g.sx1 + (k - g.sx0);
    const unsigned r = b / nfx;
    ygr = g.gy0 + (int)(r % ny);
    zch = 1 + (int)(r / ny);
}

// Occupancy (FP32): 8 wavefronts per workgroup of up to 256 VGPRs each, two
// wavefronts per SIMD, one workgroup per CU (the LDS plan takes 88 KiB);
// 12 wavefronts (3 per SIMD, 168 VGPRs) spill and were slower.
//
// Values at positions outside a Mur axis's extents (and the axion values
// beyond the ghost cells) are never read by a point inside them: the curl
// and average stencils of a valid point stay inside the extents, or reach
// a ghost, which is computed (E) or loaded (phi) explicitly, and the current
// on a boundary face averages the one interior centre twice.  So the loads
// and intermediate values are not masked; loads of such positions read a
// valid address, and only the stores check the extents.
//
// Registers.  The march is unrolled by four, so that every window along z is
// a ring of two or four registers with a fixed home in each unrolled
// iteration (no copies), and every LDS slot is a compile-time offset.  A
// quantity needed for three planes gets a ring of four, whose spare slot is
// where the loads of the next iteration land.
//
// MODE 0 is the launch over the segments, row groups and plane chunks whose
// columns, rows and planes (halos included) keep clear of every face and do
// not wrap: it has no boundary code.  MODE 1 takes the columns at both x
// faces of a run with Mur x faces and an outflow or reflecting axion x
// boundary, in the row groups and plane chunks of the interior, each
// wavefront holding both faces (lanes 0 .. 31 x_min, 32 .. 63 x_max, each
// half with two halo lanes on its inner side): the code of mode 0 plus the
// faces, whose ghosts every lane computes from its half's face values and
// stores (lanes other than a ghost's to the sink), the face values of both
// faces staged in LDS when the block starts (M3Face), so that it too issues
// the same vector memory instructions in every iteration.  A lane shift across
// lanes 31 / 32 reaches only halo lanes, as lane 0's and lane 63's reach
// nothing.  MODE 2 covers the rest (the frame), every boundary included.
template <typename T, int NW, int MODE>
__global__ void __launch_bounds__(64 * NW) k_march3d(const RunK<T> *__restrict__ rp, long step, M3Geom g)
{
    constexpr bool GEN = MODE == 2, XB = MODE == 1;
    using LQ = M3Lds<T, NW>;
    constexpr int TY = NW - 2;
    T *const lds = reinterpret_cast<T *>(m3_smem);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));

    // ---- the run's geometry and coefficients
    const int n0 = rp->n[0], n1 = rp->n[1], n2 = rp->n[2];
    const int nn0 = rp->nn[0], nn1 = rp->nn[1], nn2 = rp->nn[2];
    const bool mx = XB || (GEN && rp->mur[0]), my = GEN && rp->mur[1], mz = GEN && rp->mur[2];
    const bool apx = XB ? false : (!GEN || rp->axbc[0] == AXF_AX_PERIODIC), apy = !GEN || rp->axbc[1] == AXF_AX_PERIODIC;
    const bool apz = !GEN || rp->axbc[2] == AXF_AX_PERIODIC;
    constexpr unsigned es = sizeof(T);
    const unsigned sxb = (unsigned)rp->sx * es, syb = (unsigned)rp->sy * es;
    const T cdt0 = rp->cdt[0], cdt1 = rp->cdt[1], cdt2 = rp->cdt[2], half = rp->half, inv_dt = rp->inv_dt;
    const T i2x0 = rp->inv2dx[0], i2x1 = rp->inv2dx[1], i2x2 = rp->inv2dx[2];
    const T idx0 = rp->inv_dx2[0], idx1 = rp->inv_dx2[1], idx2 = rp->inv_dx2[2];
    const T dt2 = rp->dt2, m2 = rp->m2, gax = rp->gax, cg1 = rp->cg1;
    const char *const sb = rp->state_base;
    // array stride in units of 256 bytes (arrays are 256-byte aligned and sized)
    const unsigned long long as64 = (unsigned long long)rp->arr_stride;
    unsigned as_l = (unsigned)(rp->arr_stride >> 8);
    const int nem = rp->nem, nph = rp->nph;
    const int so = em_slot(step, nem), sn = em_slot(step + 1, nem);
    const int la = phi_slot(step, nph), lb = phi_slot(step + 1, nph), ln = phi_slot(step + 2, nph);

    // ---- this workgroup's segment, row group and plane chunk
    int seg, ygr, zch;
    m3_block(g, MODE, blockIdx.x, seg, ygr, zch);
    // an interior segment (mode 0) starts at column xi0 + (seg - sx0) wi, a
    // frame segment at seg * wid; an x-face wavefront (mode 1) holds columns
    // -2 .. 29 in lanes 0 .. 31 and xc1 - 2 .. xc1 + 29 in lanes 32 .. 63 (own
    // columns 0 .. xa - 1 in lanes 2 .., xc1 .. nn0 - 1 in lanes 34 .. 61)
    const int x0 = MODE == 0 ? g.xi0 + (seg - g.sx0) * g.wi : seg * g.wid;
    const int wseg = MODE == 0 ? g.wi : g.wid;
    const int gx = XB ? (lane < 32 ? lane - 2 : g.xc1 - 34 + lane) : x0 - 2 + lane;
    const int y0 = ygr * TY, gy = y0 - 1 + w;
    const int z0 = m3_zb(g, zch), z1 = m3_zb(g, zch + 1);

    // ---- this lane's column
    const int xs_em = MODE == 0 ? gx : (mx ? ((gx >= 0 && gx < nn0) ? gx : 0) : m3::imodn(gx, n0));
    // axion column class: 0 a cell (or a periodic axis), 1 / 2 the ghost below / above, 3 none
    const int xcl = apx ? 0 : ((gx >= 0 && gx < n0) ? 0 : (gx == -1 ? 1 : (gx == n0 ? 2 : 3)));
    const int xs_ph = MODE == 0 ? gx : (apx ? m3::imodn(gx, n0) : (xcl == 0 ? gx : 0));
    const unsigned xo_em = (unsigned)xs_em * es, xo_ph = (unsigned)xs_ph * es;
    // own columns: nodal x components store there, centred ones where also gx < n0
    auto own_lane = [&](int l) __attribute__((always_inline)) {
        if constexpr (XB) return l < 32 ? (l >= 2 && l < 2 + g.xa) : (l >= 34 && g.xc1 - 34 + l < nn0);
        return l >= 2 && l < 2 + wseg && x0 - 2 + l < nn0;
    };
    const bool own_x = own_lane(lane);
    const bool own_xc = own_x && (!mx || gx < n0);
    // the segment holds a ghost column of an x face (Mur or axion)
    const bool seg_xb = XB || (GEN && (mx || !apx) && (x0 - 2 <= -1 || x0 + 61 >= n0));
    // the x face of this lane's half of a mode-1 wavefront (0: x_min, 1:
    // x_max) and the column of its ghost
    const int xside = (XB && lane >= 32) ? 1 : 0;
    const int gx_ghost = xside ? n0 : -1;
    // B_ext at this lane's cells (slab along x); formed at use from the slab
    // mask in the interior launch, so that it takes no vector registers
    const bool in_slab = xs_em >= rp->slab_lo && xs_em < rp->slab_hi;
    const T bxs0 = rp->bext[0], bxs1 = rp->bext[1], bxs2 = rp->bext[2];
    T bext0v = T(0), bext1v = T(0), bext2v = T(0);
    if constexpr (GEN) {
        bext0v = in_slab ? bxs0 : T(0);
        bext1v = in_slab ? bxs1 : T(0);
        bext2v = in_slab ? bxs2 : T(0);
    }
    auto bext_c = [&](int c) __attribute__((always_inline)) -> T {
        if constexpr (GEN) return c == 0 ? bext0v : (c == 1 ? bext1v : bext2v);
        return in_slab ? (c == 0 ? bxs0 : (c == 1 ? bxs1 : bxs2)) : T(0);
    };

    // ---- rows (wave-uniform)
    auto ys_em_of = [&](int y) __attribute__((always_inline)) {
        return !GEN ? y : (my ? ((y >= 0 && y < nn1) ? y : 0) : m3::imodn(y, n1));
    };
    auto ycl_of = [&](int y) __attribute__((always_inline)) {
        return apy ? 0 : ((y >= 0 && y < n1) ? 0 : (y == -1 ? 1 : (y == n1 ? 2 : 3)));
    };
    auto ys_ph_of = [&](int y) __attribute__((always_inline)) {
        return !GEN ? y : (apy ? m3::imodn(y, n1) : (ycl_of(y) == 0 ? y : 0));
    };
    const int ys_em = ys_em_of(gy);
    const unsigned yo_em = (unsigned)ys_em * sxb;
    const unsigned yo_em_up = (unsigned)ys_em_of(gy + 1) * sxb;     // the top wavefront's extra row
    const int ycl_w = ycl_of(gy), ycl_dn = ycl_of(gy - 1);          // axion row classes of the row and the one below
    const int ys_ph_w = ys_ph_of(gy), ys_ph_dn = ys_ph_of(gy - 1);
    const bool own_y = w >= 1 && w <= TY && (!GEN || gy < nn1);
    const bool yc = !my || gy < n1;                     // an own row is a centred-y point too

    // ---- planes (uniform); a plane index is at most 5 planes outside [0, nn2): one wrap suffices
    auto zs_em = [&](int p) __attribute__((always_inline)) {
        return !GEN ? p : (mz ? ((p >= 0 && p < nn2) ? p : 0) : (p < 0 ? p + n2 : (p >= n2 ? p - n2 : p)));
    };
    auto zcl_of = [&](int p) __attribute__((always_inline)) {
        return apz ? 0 : ((p >= 0 && p < n2) ? 0 : (p == -1 ? 1 : (p == n2 ? 2 : 3)));
    };
    auto zs_ph = [&](int p) __attribute__((always_inline)) {
        return !GEN ? p : (apz ? (p < 0 ? p + n2 : (p >= n2 ? p - n2 : p)) : (zcl_of(p) == 0 ? p : 0));
    };
    auto own_p = [&](int p) __attribute__((always_inline)) { return p >= z0 && p < z1; };
    auto zc = [&](int p) __attribute__((always_inline)) { return !mz || p < n2; };   // for an own plane
    auto off_em = [&](int p) __attribute__((always_inline)) -> unsigned { return xo_em + yo_em + (unsigned)zs_em(p) * syb; };

    // ---- arrays: component c of a kind and slot has its own base, so that the
    // three share one 32-bit offset (the stride is re-read at each stage, opaque
    // to the compiler, so that the bases are formed where they are used)
    auto abase = [&](int q) __attribute__((always_inline)) { return sb + ((unsigned long long)((unsigned)q * as_l) << 8); };
    auto kb_rd = [&](int kind) __attribute__((always_inline)) { return abase(q_em(kind, so, 0)); };
    auto kb_wr = [&](int kind) __attribute__((always_inline)) { return abase(q_em(kind, sn, 0)); };
    auto arr_ph = [&](int L) __attribute__((always_inline)) { return abase(q_phi(nem, L)); };
    auto ld = [&](const char *kb, int c, unsigned off) __attribute__((always_inline)) -> T { return m3::ldo<T>(kb + c * as64, off); };
    auto st = [&](const char *kb, int c, unsigned off, T v) __attribute__((always_inline)) { m3::sto<T>(kb + c * as64, off, v); };

    int i = z0 - 2;   // the iteration (first: z0 - 2, last: z1 + 3)
    // mode 1: first elements of the laser table's levels of t_n and t_n+1
    const long inc_lv0 = (step % rp->inc_k1) * 2 * rp->inc_face;
    const long inc_lv1 = ((step + 1) % rp->inc_k1) * 2 * rp->inc_face;

    // ---- mode 1: the face values of this block's planes and rows into LDS
    // (planes outside the grid, read only by warm-up iterations whose values
    // no owned point takes, are clamped to it; the rows are inside it)
    using FQ = M3Face<T, NW>;
    const int fz0 = z0 - FQ::LAG_LO, fnp = FQ::planes(z0, z1);
    T *const fst_t = reinterpret_cast<T *>(m3_smem + LQ::BYTES);
    double *const fst_d = reinterpret_cast<double *>(m3_smem + LQ::BYTES + (size_t)fnp * FQ::ROWS * FQ::NT * sizeof(T));
    if constexpr (XB) {
        const bool las = rp->las.on;
        for (int k = (int)threadIdx.x; k < fnp * FQ::ROWS; k += 64 * NW) {
            const int pl = k / FQ::ROWS, r = k - pl * FQ::ROWS;
            int p = fz0 + pl;
            p = p < 0 ? 0 : (p > nn2 - 1 ? nn2 - 1 : p);
            const long f = (long)p * nn1 + (y0 - 2 + r);
            T *const d = fst_t + k * FQ::NT;
#pragma unroll
            for (int sd = 0; sd < 2; sd++) {
                d[0 + sd] = m3::fld(rp, q_axg(0, sd, la), f);
                d[2 + sd] = m3::fld(rp, q_axg(0, sd, lb), f);
                d[4 + sd] = m3::fld(rp, q_mur(0, 0, sd, 1, so), f);
                d[6 + sd] = m3::fld(rp, q_mur(0, 0, sd, 2, so), f);
                d[8 + sd] = m3::fld(rp, q_mur(1, 0, sd, 1, so), f);
                d[10 + sd] = m3::fld(rp, q_mur(1, 0, sd, 2, so), f);
            }
            double *const e = fst_d + k * 4;
            e[0] = las ? rp->inc[inc_lv0 + f] : 0.0;
            e[1] = las ? rp->inc[inc_lv0 + rp->inc_face + f] : 0.0;
            e[2] = las ? rp->inc[inc_lv1 + f] : 0.0;
            e[3] = las ? rp->inc[inc_lv1 + rp->inc_face + f] : 0.0;
        }
        __syncthreads();
    }
    // record of plane p, row y - (y0 - 2)
    auto frec = [&](int p, int r) __attribute__((always_inline)) { return (p - fz0) * FQ::ROWS + r; };

    // ---- LDS: row w + d of quantity q at slot s (a compile-time value in
    // each unrolled iteration)
    const int lrow = w * 64 + lane;
    auto lidx = [&](int q, int s, int d) __attribute__((always_inline)) {
        return lrow + LQ::base(q) + (s * LQ::R(q) + d + LQ::roff(q)) * 64;
    };
    const int wlo = w > 0 ? -1 : 0;   // the row below (the lowest wavefront reads its own: never used)
    // Interior launch: every iteration issues the same memory instructions
    // (loads of clamped planes, all stages, every store), so that the compiler
    // can count the loads still in flight exactly and never waits for the
    // stores; a point this wavefront does not own is stored to the array's sink.
    const unsigned sink_o = (unsigned)rp->arr_sink + (((blockIdx.x * NW + (unsigned)w) & 127u) * 64u + (unsigned)lane) * es;
    auto act = [&](int lo, int hi) __attribute__((always_inline)) { return !GEN || (i >= lo && i <= hi); };
    auto clampz = [&](int p, int lo, int hi) __attribute__((always_inline)) { return GEN ? p : (p < lo ? lo : (p > hi ? hi : p)); };
    // rows read one up / one down by the stages of every wavefront (interior
    // launch): clamped to the workgroup, where an edge wavefront's value is never used
    const int dn1 = (!GEN && w == 0) ? 0 : -1;
    const int up1 = (!GEN && w == NW - 1) ? 0 : 1;

    // ---- axion level L of a row of class ycl and storage row ys, plane p: the
    // array, or the y / z ghost plane for a ghost row / plane; in segments with
    // x ghost columns also the x ghost plane, which phi_take picks for those columns
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
            if constexpr (XB) r.fx = fst_t[frec(zs, ys - (y0 - 2)) * FQ::NT + (L == lb ? 2 : 0) + xside];
            else if (seg_xb && !apx) r.fx = m3::fld(rp, q_axg(0, xcl == 2 ? 1 : 0, L), (long)zs * nn1 + ys);
        }
        return r;
    };
    auto phi_take = [&](const PhiRaw& r, int ycl, int p) __attribute__((always_inline)) -> T {
        if (!(seg_xb && !apx) || ycl != 0 || zcl_of(p) != 0) return r.a;
        return (xcl == 1 || xcl == 2) ? r.fx : r.a;
    };

    // ---- windows along z.  Rings of four are indexed by (t - i_first) mod 4,
    // t the iteration that took the value in (loads) or computed it; rings of
    // two likewise mod 2.
    //   b0r: B0 of plane t            b1r: B1 of plane t - 2
    //   e0r: E0^{n-1/2} of plane t - 1 e1r: E1^{n-1/2} of plane t - 3
    //   e0hr: E0^{n+1/2} of plane t - 1, e0nr: E0^n of plane t - 1
    //   cxy, cz: C of plane t - 2 (x, y in a ring of two, z in a ring of four)
    //   bor: B0^n averaged to the centres of plane t - 2 (the current's)
    //   b0pr: B0^{n+1} of plane t - 2   e1hr: E1^{n+1/2} of plane t - 3
    T b0r[4][3], b1r[4][3], e0r[2][3], e1r[2][3], e0hr[4][3], e0nr[2][3], cxy[2][2], cz[4], bor[4][3], b0pr[4][3],
        e1hr[4][3];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        cz[k] = T(0);
#pragma unroll
        for (int c = 0; c < 3; c++) b0r[k][c] = b1r[k][c] = e0hr[k][c] = bor[k][c] = b0pr[k][c] = e1hr[k][c] = T(0);
    }
#pragma unroll
    for (int k = 0; k < 2; k++) {
        cxy[k][0] = cxy[k][1] = T(0);
#pragma unroll
        for (int c = 0; c < 3; c++) e0r[k][c] = e1r[k][c] = e0nr[k][c] = T(0);
    }
    // the axion levels (planes i - 1 .. i - 4 and i - 1 .. i - 5) and the
    // loads of the next iteration's axion levels and extra rows
    T pa_1 = 0, pa_2 = 0, pa_3 = 0, pa_4 = 0;
    T pb_1 = 0, pb_2 = 0, pb_3 = 0, pb_4 = 0, pb_5 = 0;
    PhiRaw Ppa{T(0), T(0)}, Ppb{T(0), T(0)};
    T Pxb0x = T(0), Pxb0z = T(0);      // B0x, B0z of the row above (the highest wavefront)
    T Pxpa = T(0), Pxpb = T(0);        // both axion levels of the row below (the lowest)
    T Pxpa_f = T(0), Pxpb_f = T(0);    // ... their x ghost values (frame launch)
    // FP32 issues the loads of iteration t two iterations ahead, into one of
    // two staging sets (by the parity of t), and moves them into the windows
    // when t begins: an iteration then waits only for the loads, and the
    // stores before them, issued two iterations earlier.  FP64 has no
    // registers to spare and loads one iteration ahead straight into the
    // windows.
    constexpr int PD = sizeof(T) == 4 ? 2 : 1;
    struct Stage {
        T b0[3], e0[3], b1[3], e1[3];
        PhiRaw pa, pb;
        T xb0x, xb0z, xpa, xpb, xpa_f, xpb_f;
    };
    Stage stg[PD];
#pragma unroll
    for (int k = 0; k < PD; k++) {
#pragma unroll
        for (int c = 0; c < 3; c++) stg[k].b0[c] = stg[k].e0[c] = stg[k].b1[c] = stg[k].e1[c] = T(0);
        stg[k].pa = stg[k].pb = PhiRaw{T(0), T(0)};
        stg[k].xb0x = stg[k].xb0z = stg[k].xpa = stg[k].xpb = stg[k].xpa_f = stg[k].xpb_f = T(0);
    }

    // first and last iterations of the march, and the iterations each load
    // group and stage is needed in (no owned value depends on the others)
    const int i_first = z0 - 2, i_last = z1 + 3;
    // the loads taken in by iteration t: into its ring slots (Sc = the slot
    // of t mod 4) or, two iterations ahead, into staging set Sc mod 2
    auto prefetch = [&](int t, auto Sc) __attribute__((always_inline)) {
        constexpr int S4 = decltype(Sc)::value & 3, S2 = decltype(Sc)::value & 1;
        T (&db0)[3] = PD == 2 ? stg[S2 % PD].b0 : b0r[S4];
        T (&de0)[3] = PD == 2 ? stg[S2 % PD].e0 : e0r[S2];
        T (&db1)[3] = PD == 2 ? stg[S2 % PD].b1 : b1r[S4];
        T (&de1)[3] = PD == 2 ? stg[S2 % PD].e1 : e1r[S2];
        PhiRaw &dpa = PD == 2 ? stg[S2 % PD].pa : Ppa;
        PhiRaw &dpb = PD == 2 ? stg[S2 % PD].pb : Ppb;
        T &dxb0x = PD == 2 ? stg[S2 % PD].xb0x : Pxb0x;
        T &dxb0z = PD == 2 ? stg[S2 % PD].xb0z : Pxb0z;
        T &dxpa = PD == 2 ? stg[S2 % PD].xpa : Pxpa;
        T &dxpb = PD == 2 ? stg[S2 % PD].xpb : Pxpb;
        T &dxpa_f = PD == 2 ? stg[S2 % PD].xpa_f : Pxpa_f;
        T &dxpb_f = PD == 2 ? stg[S2 % PD].xpb_f : Pxpb_f;
        asm volatile("" : "+s"(as_l));
        auto need = [&](int lo, int hi) __attribute__((always_inline)) { return !GEN || (t >= lo && t <= hi); };
        if (need(-(1 << 30), z1 + 1)) {          // B0 of plane t, axion levels of plane t - 1
            const char *kb = kb_rd(1);
            const int pz = clampz(t, z0 - 2, z1 + 1), pp = clampz(t - 1, z0 - 3, z1);
            const unsigned o = off_em(pz);
#pragma unroll
            for (int c = 0; c < 3; c++) db0[c] = ld(kb, c, o);
            dpa = phi_load(la, ycl_w, ys_ph_w, pp);
            dpb = phi_load(lb, ycl_w, ys_ph_w, pp);
            if (!GEN || w == NW - 1) {       // (every wavefront of the interior launch loads the extra rows)
                const unsigned ox = xo_em + yo_em_up + (unsigned)zs_em(pz) * syb;
                dxb0x = ld(kb, 0, ox);
                dxb0z = ld(kb, 2, ox);
            }
            if (!GEN || w == 0) {
                const PhiRaw ra = phi_load(la, ycl_dn, ys_ph_dn, pp), rb = phi_load(lb, ycl_dn, ys_ph_dn, pp);
                dxpa = ra.a;
                dxpb = rb.a;
                dxpa_f = ra.fx;
                dxpb_f = rb.fx;
            }
        }
        if (need(z0 - 1, z1 + 1)) {              // E0^{n-1/2} of plane t - 1
            const char *kb = kb_rd(0);
            const unsigned o = off_em(clampz(t - 1, z0 - 2, z1));
#pragma unroll
            for (int c = 0; c < 3; c++) de0[c] = ld(kb, c, o);
        }
        if (need(z0 + 1, z1 + 2)) {              // B1 of plane t - 2
            const char *kb = kb_rd(3);
            const unsigned o = off_em(clampz(t - 2, z0 - 1, z1));
#pragma unroll
            for (int c = 0; c < 3; c++) db1[c] = ld(kb, c, o);
        }
        if (need(z0 + 2, z1 + 2)) {              // E1^{n-1/2} of plane t - 3
            const char *kb = kb_rd(2);
            const unsigned o = off_em(clampz(t - 3, z0 - 1, z1 - 1));
#pragma unroll
            for (int c = 0; c < 3; c++) de1[c] = ld(kb, c, o);
        }
    };

    // Mur ghost (order O, component c, axis d, side) of face point fidx from
    // the adjacent point's E^{n-1/2} and E^{n+1/2}
    auto mur = [&](int O, int c, int d, int side, T e_old, T e_new, long fidx) __attribute__((always_inline)) -> T {
        const double g_old = (double)m3::fld(rp, q_mur(O, d, side, c, so), fidx);
        return mur_update_rk<T>(*rp, O, c, d, side, (double)e_old, (double)e_new, g_old, fidx, step);
    };
    // mode 1: face plane q; a store of element f of it by the lanes that own
    // it, to the sink by the others
    auto face = [&](int q) __attribute__((always_inline)) { return rp->face_base + (size_t)q * rp->face_stride; };
    auto fstx = [&](bool owner, int q, long f, T v) __attribute__((always_inline)) {
        T *const p = owner ? (T *)face(q) + f : (T *)(abase(0) + sink_o);
        *(__attribute__((address_space(1))) T *)p = v;
    };
    // mode 1: the Mur ghost of order O, component c on the x face of this
    // lane's half in this wavefront's row of plane p, from the adjacent
    // point's E^{n-1/2}, E^{n+1/2}; the old ghost and the laser values come
    // from the block's staged face records, and the x_max half takes no laser
    auto mur_x = [&](int O, int c, T e_old, T e_new, int p) __attribute__((always_inline)) -> T {
        const int k = frec(p, w + 1);
        const double g_old = (double)fst_t[k * FQ::NT + 4 + 4 * O + 2 * (c - 1) + xside];
        double ia_o = 0.0, ia_n = 0.0, ig_o = 0.0, ig_n = 0.0;
        if (O == 0) {
            const bool tab = rp->las.on && c == rp->las.pol;
            const bool use = tab && xside == 0;
            const double a0 = fst_d[k * 4 + 0], a1 = fst_d[k * 4 + 1];
            const double a2 = fst_d[k * 4 + 2], a3 = fst_d[k * 4 + 3];
            ia_o = use ? a0 : 0.0;
            ig_o = use ? a1 : 0.0;
            ia_n = use ? a2 : 0.0;
            ig_n = use ? a3 : 0.0;
        }
        return (T)mur_core(rp->murc[0], (double)e_old, (double)e_new, g_old, ia_o, ia_n, ig_o, ig_n);
    };

    auto iter = [&](auto Jc) __attribute__((always_inline)) {
        constexpr int J = decltype(Jc)::value;
        // ring slots of the values taken in / computed k iterations ago
        constexpr int Q0 = J & 3, Q1 = (J + 3) & 3, Q2 = (J + 2) & 3, Q3 = (J + 1) & 3;
        constexpr int H0 = J & 1, H1 = (J + 1) & 1;
        // LDS slot of the write of k iterations ago, K slots
        constexpr int L20 = J & 1, L21 = (J + 1) & 1;
        constexpr int L40 = J & 3, L41 = (J + 3) & 3, L42 = (J + 2) & 3, L43 = (J + 1) & 3;
        auto LW = [&](int q, int s, int d, T v) __attribute__((always_inline)) { lds[lidx(q, s, d)] = v; };
        auto LR = [&](int q, int s, int d) __attribute__((always_inline)) -> T { return lds[lidx(q, s, d)]; };
        auto LR1 = [&](int q, int s, int d) __attribute__((always_inline)) -> T { return lds[lidx(q, s, d) + 1]; };
        auto LRm = [&](int q, int s, int d) __attribute__((always_inline)) -> T { return lds[lidx(q, s, d) - 1]; };

        // ---- FP32: move this iteration's staged loads into the windows
        if constexpr (PD == 2) {
            const Stage &sg = stg[J & 1];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                b0r[Q0][c] = sg.b0[c];
                e0r[H0][c] = sg.e0[c];
                b1r[Q0][c] = sg.b1[c];
                e1r[H0][c] = sg.e1[c];
            }
            Ppa = sg.pa;
            Ppb = sg.pb;
            Pxb0x = sg.xb0x;
            Pxb0z = sg.xb0z;
            Pxpa = sg.xpa;
            Pxpb = sg.xpb;
            Pxpa_f = sg.xpa_f;
            Pxpb_f = sg.xpb_f;
        }
        // ---- take in the axion levels and extra rows, then load for iteration i + PD
        // the axion levels of this row: the interior launch keeps planes i - 3,
        // i - 4 of the older level and i - 5 of the newer in registers and reads
        // the others from its own LDS row (the two reads below take the slots
        // written two and four iterations ago before this iteration reuses them)
        if constexpr (!GEN) {
            pa_4 = pa_3;
            pa_3 = LR(LQ::PA, L20, 0);
            pb_5 = LR(LQ::PB, L40, 0);
        } else {
            pa_4 = pa_3; pa_3 = pa_2; pa_2 = pa_1;
            pb_5 = pb_4; pb_4 = pb_3; pb_3 = pb_2; pb_2 = pb_1;
        }
        const int p1 = i - 1, p2 = i - 2, p3 = i - 3, p4 = i - 4;
        pa_1 = phi_take(Ppa, ycl_w, p1);
        pb_1 = phi_take(Ppb, ycl_w, p1);
        if (w == 0) {
            LW(LQ::PA, L20, -1, phi_take(PhiRaw{Pxpa, Pxpa_f}, ycl_dn, p1));
            LW(LQ::PB, L40, -1, phi_take(PhiRaw{Pxpb, Pxpb_f}, ycl_dn, p1));
        }
        LW(LQ::PA, L20, 0, pa_1);
        LW(LQ::PB, L40, 0, pb_1);
        LW(LQ::B0X, L40, 0, b0r[Q0][0]);
        LW(LQ::B0Z, L40, 0, b0r[Q0][2]);
        if (w == NW - 1) {
            LW(LQ::B0X, L40, 1, Pxb0x);
            LW(LQ::B0Z, L40, 1, Pxb0z);
        }
        if (!GEN || i + PD <= i_last) prefetch(i + PD, std::integral_constant<int, (J + PD) & 3>{});

        // ---- loaded values the neighbouring rows read
        LW(LQ::B1X, L20, 0, b1r[Q0][0]);
        LW(LQ::B1Z, L20, 0, b1r[Q0][2]);

        // ================================================ S1: E0 at plane p1
        asm volatile("" : "+s"(as_l));
        if (act(z0 - 1, z1 + 1)) {
            const T *b0_0 = b0r[Q0], *b0_1 = b0r[Q1];
            const T *e0o = e0r[H0];
            const T b0z_y = LR(LQ::B0Z, L41, 1), b0x_y = LR(LQ::B0X, L41, 1);
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
            if constexpr (XB) {
                // the Mur ghosts across x of E0y and E0z
                const T up_y = m3::lane_up(eh[1]), dn_y = m3::lane_dn(eh[1]), up_z = m3::lane_up(eh[2]), dn_z = m3::lane_dn(eh[2]);
                const T oup_y = m3::lane_up(e0o[1]), odn_y = m3::lane_dn(e0o[1]);
                const T oup_z = m3::lane_up(e0o[2]), odn_z = m3::lane_dn(e0o[2]);
                const long f = (long)zs_em(p1) * nn1 + ys_em;
                const T vy = mur_x(0, 1, xside ? odn_y : oup_y, xside ? dn_y : up_y, p1);
                const T vz = mur_x(0, 2, xside ? odn_z : oup_z, xside ? dn_z : up_z, p1);
                const bool isg = gx == gx_ghost;
                const bool owner = isg && own_lane(xside ? lane - 1 : lane + 1) && own_y && own_p(p1);
                eh[1] = isg ? vy : eh[1];
                eh[2] = isg ? vz : eh[2];
                fstx(owner, q_mur(0, 0, xside, 1, sn), f, vy);
                fstx(owner, q_mur(0, 0, xside, 2, sn), f, vz);
            }
            if constexpr (!GEN) {
                const bool ow = own_y && own_p(p1);
                const unsigned on = (own_x && ow) ? off_em(p1) : sink_o;
                const unsigned oc = XB ? ((own_xc && ow) ? off_em(p1) : sink_o) : on;
                const char *kb = kb_wr(0);
                st(kb, 0, on, eh[0]);
                st(kb, 1, oc, eh[1]);
                st(kb, 2, oc, eh[2]);
            } else if (own_y && own_p(p1)) {
                const char *kb = kb_wr(0);
                const unsigned o = off_em(p1);
                if (yc && zc(p1) && own_x) st(kb, 0, o, eh[0]);
                if (zc(p1) && own_xc) st(kb, 1, o, eh[1]);
                if (yc && own_xc) st(kb, 2, o, eh[2]);
            }
            // Mur ghosts across x of E0y (nodal y, centred z) and E0z (centred y, nodal z)
            if (GEN && mx && seg_xb) {
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
                    T e_new = side ? e0hr[Q1][c] : eh[c];
                    T v = mur(0, c, 2, side, e_old, e_new, f);
                    if (side) eh[c] = v;
                    else e0hr[Q1][c] = v;
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
                LW(LQ::E0HX, L20, -1, gxv);
                LW(LQ::E0HZ, L20, -1, gzv);
            }
#pragma unroll
            for (int c = 0; c < 3; c++) {
                e0hr[Q0][c] = eh[c];
                e0nr[H0][c] = en[c];
            }
            LW(LQ::E0NY, L20, 0, en[1]);
            LW(LQ::E0HY, L40, 0, eh[1]);
            if (!(my && gy == -1)) {
                LW(LQ::E0HX, L20, 0, eh[0]);
                LW(LQ::E0HZ, L20, 0, eh[2]);
            }
        }

        // ================================================ S2: C at the cells of plane p2
        if ((!GEN || w <= NW - 2) && act(z0, z1 + 1)) {
            const T *b0_1 = b0r[Q1], *b0_2 = b0r[Q2];
            const T *e0n_1 = e0nr[H0], *e0n_2 = e0nr[H1];
            T e[3], bb[3], gp[3], bo[3];
            e[0] = half * (e0n_2[0] + m3::lane_up(e0n_2[0]));
            e[1] = half * (e0n_2[1] + LR(LQ::E0NY, L21, up1));
            e[2] = half * (e0n_2[2] + e0n_1[2]);
            const T bxy0 = LR(LQ::B0X, L42, 1), bxy1 = LR(LQ::B0X, L41, 1);
            const T bzy = LR(LQ::B0Z, L42, 1), bzyx = LR1(LQ::B0Z, L42, 1);
            bo[0] = T(0.25) * ((b0_2[0] + bxy0) + (b0_1[0] + bxy1));
            bo[1] = T(0.25) * ((b0_2[1] + m3::lane_up(b0_2[1])) + (b0_1[1] + m3::lane_up(b0_1[1])));
            bo[2] = T(0.25) * ((b0_2[2] + m3::lane_up(b0_2[2])) + (bzy + bzyx));
            bb[0] = bo[0] + bext_c(0);
            bb[1] = bo[1] + bext_c(1);
            bb[2] = bo[2] + bext_c(2);
            T qa2, qb2, qb3, upa2, upb2, dna2, dnb2;
            if constexpr (!GEN) {
                qa2 = LR(LQ::PA, L21, 0);
                qb2 = LR(LQ::PB, L41, 0);
                qb3 = LR(LQ::PB, L42, 0);
                upa2 = LR1(LQ::PA, L21, 0);
                upb2 = LR1(LQ::PB, L41, 0);
                dna2 = LRm(LQ::PA, L21, 0);
                dnb2 = LRm(LQ::PB, L41, 0);
            } else {
                qa2 = pa_2;
                qb2 = pb_2;
                qb3 = pb_3;
                upa2 = m3::lane_up(pa_2);
                upb2 = m3::lane_up(pb_2);
                dna2 = m3::lane_dn(pa_2);
                dnb2 = m3::lane_dn(pb_2);
            }
            T dtphi = (qb2 - qa2) * inv_dt;
            {
                T up = half * (upa2 + upb2), dn = half * (dna2 + dnb2);
                gp[0] = (up - dn) * i2x0;
            }
            {
                T up = half * (LR(LQ::PA, L21, up1) + LR(LQ::PB, L41, up1));
                T dn = half * (LR(LQ::PA, L21, -1) + LR(LQ::PB, L41, -1));
                gp[1] = (up - dn) * i2x1;
            }
            {
                T up = half * (pa_1 + pb_1), dn = half * (pa_3 + qb3);
                gp[2] = (up - dn) * i2x2;
            }
            cxy[H0][0] = dtphi * bb[0] - (e[1] * gp[2] - e[2] * gp[1]);
            cxy[H0][1] = dtphi * bb[1] - (e[2] * gp[0] - e[0] * gp[2]);
            cz[Q0] = dtphi * bb[2] - (e[0] * gp[1] - e[1] * gp[0]);
#pragma unroll
            for (int c = 0; c < 3; c++) bor[Q0][c] = bo[c];
            LW(LQ::CY, L20, 0, cxy[H0][1]);
        }

        // ================================================ S3: B0^{n+1} at plane p2
        asm volatile("" : "+s"(as_l));
        if ((!GEN || w >= 1) && act(z0 + 2, z1 + 2)) {
            const T *b0_2 = b0r[Q2];
            const T exm = LR(LQ::E0HX, L21, dn1), ezm = LR(LQ::E0HZ, L21, dn1);
            // E0^{n+1/2} of this row at planes p2 and p2 - 1 (the interior launch
            // reads the copies its own row wrote to LDS instead of keeping them)
            T e2[3], e3x, e3y, dn_ez, dn_e2y;
            if constexpr (!GEN) {
                e2[0] = LR(LQ::E0HX, L21, 0);
                e2[1] = LR(LQ::E0HY, L41, 0);
                e2[2] = LR(LQ::E0HZ, L21, 0);
                e3x = e0hr[Q2][0];
                e3y = LR(LQ::E0HY, L42, 0);
                dn_ez = LRm(LQ::E0HZ, L21, 0);
                dn_e2y = LRm(LQ::E0HY, L41, 0);
            } else {
                e2[0] = e0hr[Q1][0];
                e2[1] = e0hr[Q1][1];
                e2[2] = e0hr[Q1][2];
                e3x = e0hr[Q2][0];
                e3y = e0hr[Q2][1];
            }
            T ex = e2[0], ez = e2[2];
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
            if constexpr (GEN) {
                dn_ez = m3::lane_dn(ez);
                dn_e2y = m3::lane_dn(e2[1]);
            }
            T v[3];
            {
                T a = cdt1 * (ez - ezm), b = cdt2 * (e2[1] - e3y);
                v[0] = b0_2[0] - (a - b);
            }
            {
                T a = cdt2 * (ex - e3x), b = cdt0 * (ez - dn_ez);
                v[1] = b0_2[1] - (a - b);
            }
            {
                T a = cdt0 * (e2[1] - dn_e2y), b = cdt1 * (ex - exm);
                v[2] = b0_2[2] - (a - b);
            }
            if constexpr (!GEN) {
                const unsigned on = (own_x && ownr) ? off_em(p2) : sink_o;
                const unsigned oc = XB ? ((own_xc && ownr) ? off_em(p2) : sink_o) : on;
                const char *kb = kb_wr(1);
                st(kb, 0, oc, v[0]);
                st(kb, 1, on, v[1]);
                st(kb, 2, on, v[2]);
            } else if (ownr) {
                const char *kb = kb_wr(1);
                const unsigned o = off_em(p2);
                if (own_xc) st(kb, 0, o, v[0]);
                if (yc && own_x) st(kb, 1, o, v[1]);
                if (zc(p2) && own_x) st(kb, 2, o, v[2]);
            }
#pragma unroll
            for (int c = 0; c < 3; c++) b0pr[Q0][c] = v[c];
            LW(LQ::B0PX, L40, 0, v[0]);
            LW(LQ::B0PZ, L40, 0, v[2]);
        }

        // ================================================ S4: E1 at plane p3
        asm volatile("" : "+s"(as_l));
        if ((!GEN || w <= NW - 2) && act(z0 + 2, z1 + 2)) {
            const T *b1_2 = b1r[Q0], *b1_3 = b1r[Q1];
            const T *e1o = e1r[H0];
            const T *c_3 = cxy[H1];
            const T c3z = cz[Q1], c_4z = cz[Q2];
            const T b1z_y = LR(LQ::B1Z, L21, up1), b1x_y = LR(LQ::B1X, L21, up1);
            const T cym = LR(LQ::CY, L21, wlo);
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
                T lo = (mz && p3 - 1 < 0) ? c3z : c_4z;
                T hi = (mz && p3 > n2 - 1) ? c_4z : c3z;
                T Sc = half * (lo + hi);
                T a = cdt0 * (m3::lane_up(b1_3[1]) - b1_3[1]), b = cdt1 * (b1x_y - b1_3[0]);
                T rhs = (a - b) - cg1 * Sc;
                eh[2] = e1o[2] + T(1) * rhs;
            }
            if constexpr (XB) {
                const T up_y = m3::lane_up(eh[1]), dn_y = m3::lane_dn(eh[1]), up_z = m3::lane_up(eh[2]), dn_z = m3::lane_dn(eh[2]);
                const T oup_y = m3::lane_up(e1o[1]), odn_y = m3::lane_dn(e1o[1]);
                const T oup_z = m3::lane_up(e1o[2]), odn_z = m3::lane_dn(e1o[2]);
                const long f = (long)zs_em(p3) * nn1 + ys_em;
                const T vy = mur_x(1, 1, xside ? odn_y : oup_y, xside ? dn_y : up_y, p3);
                const T vz = mur_x(1, 2, xside ? odn_z : oup_z, xside ? dn_z : up_z, p3);
                const bool isg = gx == gx_ghost;
                const bool owner = isg && own_lane(xside ? lane - 1 : lane + 1) && own_y && own_p(p3);
                eh[1] = isg ? vy : eh[1];
                eh[2] = isg ? vz : eh[2];
                fstx(owner, q_mur(1, 0, xside, 1, sn), f, vy);
                fstx(owner, q_mur(1, 0, xside, 2, sn), f, vz);
            }
            if constexpr (!GEN) {
                const bool ow = own_y && own_p(p3);
                const unsigned on = (own_x && ow) ? off_em(p3) : sink_o;
                const unsigned oc = XB ? ((own_xc && ow) ? off_em(p3) : sink_o) : on;
                const char *kb = kb_wr(2);
                st(kb, 0, on, eh[0]);
                st(kb, 1, oc, eh[1]);
                st(kb, 2, oc, eh[2]);
            } else if (own_y && own_p(p3)) {
                const char *kb = kb_wr(2);
                const unsigned o = off_em(p3);
                if (yc && zc(p3) && own_x) st(kb, 0, o, eh[0]);
                if (zc(p3) && own_xc) st(kb, 1, o, eh[1]);
                if (yc && own_xc) st(kb, 2, o, eh[2]);
            }
            if (GEN && mx && seg_xb) {
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
                    T e_new = side ? e1hr[Q1][c] : eh[c];
                    T v = mur(1, c, 2, side, e_old, e_new, f);
                    if (side) eh[c] = v;
                    else e1hr[Q1][c] = v;
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
                LW(LQ::E1X, L20, -1, gxv);
                LW(LQ::E1Z, L20, -1, gzv);
            }
#pragma unroll
            for (int c = 0; c < 3; c++) e1hr[Q0][c] = eh[c];
            if (!(my && gy == -1)) {
                LW(LQ::E1X, L20, 0, eh[0]);
                LW(LQ::E1Z, L20, 0, eh[2]);
            }
        }

        // ================================================ S5, S6 at plane p4 (own rows)
        asm volatile("" : "+s"(as_l));
        if ((!GEN || own_y) && act(z0 + 4, z1 + 3)) {
            const bool ownp = own_p(p4);
            // ---- S5: B1^{n+1}
            {
                const T *e1h_4 = e1hr[Q1], *e1h_5 = e1hr[Q2], *b1_4 = b1r[Q2];
                const T exm = LR(LQ::E1X, L21, dn1), ezm = LR(LQ::E1Z, L21, dn1);
                T ex, ez, dn_ez;
                if constexpr (!GEN) {
                    ex = LR(LQ::E1X, L21, 0);
                    ez = LR(LQ::E1Z, L21, 0);
                    dn_ez = LRm(LQ::E1Z, L21, 0);
                } else {
                    ex = e1h_4[0];
                    ez = e1h_4[2];
                }
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
                if constexpr (GEN) dn_ez = m3::lane_dn(ez);
                {
                    T a = cdt2 * (ex - e1h_5[0]), b = cdt0 * (ez - dn_ez);
                    v[1] = b1_4[1] - (a - b);
                }
                {
                    T a = cdt0 * (e1h_4[1] - m3::lane_dn(e1h_4[1])), b = cdt1 * (ex - exm);
                    v[2] = b1_4[2] - (a - b);
                }
                if constexpr (!GEN) {
                    const unsigned on = (own_x && own_y && ownp) ? off_em(p4) : sink_o;
                    const unsigned oc = XB ? ((own_xc && own_y && ownp) ? off_em(p4) : sink_o) : on;
                    const char *kb = kb_wr(3);
                    st(kb, 0, oc, v[0]);
                    st(kb, 1, on, v[1]);
                    st(kb, 2, on, v[2]);
                } else if (ownp) {
                    const char *kb = kb_wr(3);
                    const unsigned o = off_em(p4);
                    if (own_xc) st(kb, 0, o, v[0]);
                    if (yc && own_x) st(kb, 1, o, v[1]);
                    if (zc(p4) && own_x) st(kb, 2, o, v[2]);
                }
            }
                // ---- S6: phi^{n+3/2} at the cells
            {
                const T *e0h_3 = e0hr[Q2], *e0h_4 = e0hr[Q3], *bo_4 = bor[Q2], *b0p_3 = b0pr[Q1], *b0p_4 = b0pr[Q2];
                T e[3], bb[3], bn[3];
                // this row's E0y^{n+1/2} at p4 and B0x, B0z^{n+1} at p4 (and B0x at p4 + 1):
                // LDS copies in the interior launch, registers in the frame launch
                T e4y, p4x, p3x, p4z, p4zx;
                if constexpr (!GEN) {
                    e4y = LR(LQ::E0HY, L43, 0);
                    p4x = LR(LQ::B0PX, L42, 0);
                    p3x = LR(LQ::B0PX, L41, 0);
                    p4z = LR(LQ::B0PZ, L42, 0);
                    p4zx = LR1(LQ::B0PZ, L42, 0);
                } else {
                    e4y = e0h_4[1];
                    p4x = b0p_4[0];
                    p3x = b0p_3[0];
                    p4z = b0p_4[2];
                    p4zx = m3::lane_up(b0p_4[2]);
                }
                e[0] = half * (e0h_4[0] + m3::lane_up(e0h_4[0]));
                e[1] = half * (e4y + LR(LQ::E0HY, L43, up1));
                e[2] = half * (e0h_4[2] + e0h_3[2]);
                bn[0] = T(0.25) * ((p4x + LR(LQ::B0PX, L42, up1)) + (p3x + LR(LQ::B0PX, L41, up1)));
                bn[1] = T(0.25) * ((b0p_4[1] + m3::lane_up(b0p_4[1])) + (b0p_3[1] + m3::lane_up(b0p_3[1])));
                bn[2] = T(0.25) * ((p4z + p4zx) + (LR(LQ::B0PZ, L42, up1) + LR1(LQ::B0PZ, L42, up1)));
                bb[0] = half * (bo_4[0] + bn[0]) + bext_c(0);
                bb[1] = half * (bo_4[1] + bn[1]) + bext_c(1);
                bb[2] = half * (bo_4[2] + bn[2]) + bext_c(2);
                T sax = gax * (e[0] * bb[0] + e[1] * bb[1] + e[2] * bb[2]);
                T pb, upb4, dnb4, qb3s;
                if constexpr (!GEN) {
                    pb = LR(LQ::PB, L43, 0);
                    upb4 = LR1(LQ::PB, L43, 0);
                    dnb4 = LRm(LQ::PB, L43, 0);
                    qb3s = LR(LQ::PB, L42, 0);
                } else {
                    pb = pb_4;
                    upb4 = m3::lane_up(pb_4);
                    dnb4 = m3::lane_dn(pb_4);
                    qb3s = pb_3;
                }
                const T pa = pa_4;
                T lap = T(0);
                lap += ((upb4 - T(2) * pb) + dnb4) * idx0;
                lap += ((LR(LQ::PB, L43, up1) - T(2) * pb) + LR(LQ::PB, L43, -1)) * idx1;
                lap += ((qb3s - T(2) * pb) + pb_5) * idx2;
                const int gz = zs_em(p4);
                // (a run with a damping layer has no interior launch)
                const bool pml = GEN && (rp->axbc[0] == AXF_AX_PML || rp->axbc[1] == AXF_AX_PML || rp->axbc[2] == AXF_AX_PML);
                T sdt = pml ? pml_sdt<3>(*rp, xs_em, ys_em, gz) : T(0);
                T xq = dt2 * ((sax - m2 * pb) + lap) - sdt * sdt * pb;
                T pn = ((xq + sdt * pa) + T(2) * pb) - pa;
                if (sdt != T(0)) pn = pn / (T(1) + sdt);
                if constexpr (XB) {
                    // the axion ghost beyond the boundary cell of the x face of this lane's half
                    const long f = (long)gz * nn1 + ys_em;
                    const int fk = frec(gz, w + 1) * FQ::NT;
                    const T gbv = fst_t[fk + 2 + xside], gav = fst_t[fk + 0 + xside];
                    const T rr = rp->out_r[0];
                    T xx = (((T(-2) * gbv + T(2) * gav) - dt2 * (sax - m2 * gbv)) + rr * pb - rr * rr * (pb - T(2) * gbv))
                           / (rr + rr * rr);
                    const T gval = rp->axbc[0] == AXF_AX_OUTFLOW ? gav + rr * (pb - xx) : pn;
                    const bool owner = own_xc && own_y && ownp && xs_em == (xside ? n0 - 1 : 0);
                    fstx(owner, q_axg(0, xside, ln), f, gval);
                }
                if constexpr (!GEN) {
                    const bool ownc = (XB ? own_xc : own_x) && own_y && ownp;
                    m3::sto<T>(arr_ph(ln), ownc ? xo_em + yo_em + (unsigned)gz * syb : sink_o, pn);
                } else if (ownp && yc && zc(p4) && own_xc) {
                    m3::sto<T>(arr_ph(ln), xo_em + yo_em + (unsigned)gz * syb, pn);
                    // axion ghosts of the new level at the boundary cells
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        if (!GEN || rp->axbc[d] == AXF_AX_PERIODIC) continue;
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
    };

    prefetch(i_first, std::integral_constant<int, 0>{});
    if (PD == 2 && (!GEN || i_first + 1 <= i_last)) prefetch(i_first + 1, std::integral_constant<int, 1>{});
    for (;;) {
        iter(std::integral_constant<int, 0>{});
        if (++i > i_last) break;
        iter(std::integral_constant<int, 1>{});
        if (++i > i_last) break;
        iter(std::integral_constant<int, 2>{});
        if (++i > i_last) break;
        iter(std::integral_constant<int, 3>{});
        if (++i > i_last) break;
    }
}

// ------------------------------------------------------------------ host side

template <typename T> struct March3 { static constexpr int NW = sizeof(T) == 4 ? AXF_M3_NW : 6; };

// Decomposition: x segments of at most 60 own columns; row groups of NW - 2
// rows; plane chunks of about zc planes between two boundary chunks of 3
// planes.  A row group is interior when its rows y0 - 2 .. y0 + NW - 1 (the
// extra rows included) are inside [0, n1); a chunk is interior when its loads
// (planes z0 - 3 .. z1 + 1) are inside [0, n2) and it holds neither ghost
// plane nor boundary cell of a z face.  With an x-face launch the columns
// split differently in the interior row groups and chunks: 28 own columns at
// x_min and 1 .. 28 at x_max go to one x-face wavefront per row, and the
// columns between them to the fewest interior segments of equal width whose
// 64 loaded columns stay inside [0, n0).
template <typename T>
static M3Geom march3d_geom(const RunK<T>& h, int zc)
{
    constexpr int NW = March3<T>::NW, TY = NW - 2;
    using FQ = M3Face<T, NW>;
    M3Geom g;
    g.nseg = (h.nn[0] + 59) / 60;
    g.wid = (h.nn[0] + g.nseg - 1) / g.nseg;
    g.nyg = (h.nn[1] + TY - 1) / TY;
    // interior segments: columns x0 - 2 .. x0 + 61 inside [0, n0)
    g.sx0 = 1;
    g.sx1 = 1;
    while (g.sx1 < g.nseg && g.sx1 * g.wid + 61 <= h.n[0] - 1) g.sx1++;
    g.gy0 = 1;
    g.gy1 = 1;
    while (g.gy1 < g.nyg && g.gy1 * TY + NW - 1 <= h.n[1] - 1) g.gy1++;
    // a damping layer reaches into the interior: such runs take the frame
    // launch everywhere
    const bool pml = h.axbc[0] == AXF_AX_PML || h.axbc[1] == AXF_AX_PML || h.axbc[2] == AXF_AX_PML;
    if (pml || g.gy1 <= g.gy0 || g.sx1 <= g.sx0) g.gy0 = g.gy1 = g.sx0 = g.sx1 = 0;
    g.xi0 = g.sx0 * g.wid;
    g.wi = g.wid;
    g.xa = g.xc1 = 0;
    g.xb = 0;
    const int zcv = zc > 0 ? zc : 64;
    // interior block order: a band per XCD, segments fastest (measured on
    // 512^3 FP32: 39% fewer HBM reads than the plain order, 6.5 against 6.8 ms)
    const char *oe = getenv("AXF_M3_ORDER");
    g.order = oe ? atoi(oe) : 2;
    g.nn2 = h.nn[2];
    g.zf = 3;
    g.zend = h.n[2] - 2;
    if (g.zend - g.zf < 1) {            // no interior chunk: one chunk and an empty one
        g.zf = g.zend = h.nn[2];
        g.nzc = 2;
        g.zi = 1;
        g.gy0 = g.gy1 = g.sx0 = g.sx1 = 0;
        return g;
    }
    const int nzi = (g.zend - g.zf + zcv - 1) / zcv;
    g.zi = (g.zend - g.zf + nzi - 1) / nzi;
    g.nzc = nzi + 2;
    // the x-face launch: Mur x faces with an outflow or reflecting axion, in
    // FP32 with chunks whose face records fit in LDS beside the slots
    const char *xe = getenv("AXF_M3_XB");
    if (g.sx1 > g.sx0 && h.mur[0] && (h.axbc[0] == AXF_AX_OUTFLOW || h.axbc[0] == AXF_AX_REFLECT) &&
        FQ::ON && FQ::planes(0, g.zi) <= FQ::NP_MAX && !(xe && atoi(xe) == 0)) {
        // ns interior segments of w columns between the two halves: x_max
        // keeps nb = rem - ns w in [1, 28] columns (lanes 34 .. 61, so that
        // its own lanes stay two lanes clear of lane 63, as in a segment),
        // and the last segment's loads (to column 28 + (ns - 1) w + 61) stay
        // below n0
        const int xa = 28, rem = h.nn[0] - xa;
        for (int ns = 1; ns * 33 <= rem && !g.xb; ns++) {
            for (int w = 60; w >= 33; w--) {
                const int nb = rem - ns * w;
                if (nb < 1 || nb > 28 || xa + (ns - 1) * w + 61 > h.n[0] - 1) continue;
                g.xb = 1;
                g.sx0 = 0;
                g.sx1 = ns;
                g.xi0 = g.xa = xa;
                g.wi = w;
                g.xc1 = xa + ns * w;
                break;
            }
        }
    }
    return g;
}

template <typename T>
bool march3d_available(const RunK<T>& h)
{
    // 32-bit byte offsets within the three components of a kind, within the
    // boundary planes and within the laser table
    return h.D == 3 && (unsigned long long)h.arr_stride * 3 <= (1ull << 32) &&
           (unsigned long long)h.face_stride * kNumFaces < (1ull << 32) &&
           (unsigned long long)h.inc_k1 * 2 * h.inc_face * 8 < (1ull << 32);
}

template <typename T>
static void march3d_counts(const M3Geom& g, long *interior, long *xface, long *frame)
{
    const long nsx = g.sx1 - g.sx0, ny = g.gy1 - g.gy0, nzi = g.nzc - 2;
    *interior = nsx * ny * nzi;
    *xface = g.xb ? ny * nzi : 0;
    // (A) the first and last chunks, (B) the inner chunks of the row groups
    // outside [gy0, gy1), (C) the x-face columns when they have no launch
    *frame = (long)(g.nzc > 1 ? 2 : 1) * g.nseg * g.nyg + (long)g.nseg * (g.nyg - ny) * nzi +
             (g.xb ? 0 : (long)(g.nseg - nsx) * ny * nzi);
}

template <typename T>
long march3d_blocks(const RunK<T>& h, int zc)
{
    long a, b, c;
    march3d_counts<T>(march3d_geom(h, zc), &a, &b, &c);
    return a + b + c;
}

template <typename T, int MODE>
static hipError_t march3d_attr()
{
    constexpr int NW = March3<T>::NW;
    using FQ = M3Face<T, NW>;
    static bool done = false;
    if (!done) {
        const size_t bytes = MODE == 1 ? FQ::bytes(FQ::NP_MAX) : M3Lds<T, NW>::BYTES;
        hipError_t e = hipFuncSetAttribute((const void *)k_march3d<T, NW, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)bytes);
        if (e != hipSuccess) return e;
        done = true;
    }
    return hipSuccess;
}

// the interior launch on the run's stream and the x-face and frame launches
// after it, or beside it on ws->side when given (all three read only the
// state of step n and write disjoint owned points, so they may run in any
// order or together; the side launches then fill the interior's last round)
template <typename T>
hipError_t launch_march3d(const RunK<T> *rk, const RunK<T>& h, long step, int zc, hipStream_t st,
                          const WaveStreams *ws)
{
    constexpr int NW = March3<T>::NW;
    using LQ = M3Lds<T, NW>;
    using FQ = M3Face<T, NW>;
    hipError_t e = march3d_attr<T, 0>();
    if constexpr (FQ::ON) {
        if (e == hipSuccess) e = march3d_attr<T, 1>();
    }
    if (e == hipSuccess) e = march3d_attr<T, 2>();
    if (e != hipSuccess) return e;
    const M3Geom g = march3d_geom(h, zc);
    long ni, nx, nf;
    march3d_counts<T>(g, &ni, &nx, &nf);
    const bool fork = ws && ws->side && ni > 0 && nx + nf > 0;
    hipStream_t se = st;
    if (fork) {
        if ((e = hipEventRecord(ws->fork, st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(ws->side, ws->fork, 0)) != hipSuccess) return e;
        se = ws->side;
    }
    if (ni > 0) hipLaunchKernelGGL((k_march3d<T, NW, 0>), dim3((unsigned)ni), dim3(64 * NW), LQ::BYTES, st, rk, step, g);
    if constexpr (FQ::ON) {
        // every chunk of the x-face launch stages at most planes(0, zi) planes
        if (nx > 0)
            hipLaunchKernelGGL((k_march3d<T, NW, 1>), dim3((unsigned)nx), dim3(64 * NW), FQ::bytes(FQ::planes(0, g.zi)), se,
                               rk, step, g);
    }
    if (nf > 0) hipLaunchKernelGGL((k_march3d<T, NW, 2>), dim3((unsigned)nf), dim3(64 * NW), LQ::BYTES, se, rk, step, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (fork) {
        if ((e = hipEventRecord(ws->join, ws->side)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(st, ws->join, 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

template bool march3d_available<float>(const RunK<float>&);
template bool march3d_available<double>(const RunK<double>&);
template long march3d_blocks<float>(const RunK<float>&, int);
template long march3d_blocks<double>(const RunK<double>&, int);
template hipError_t launch_march3d<float>(const RunK<float> *, const RunK<float>&, long, int, hipStream_t,
                                          const WaveStreams *);
template hipError_t launch_march3d<double>(const RunK<double> *, const RunK<double>&, long, int, hipStream_t,
                                           const WaveStreams *);

}  // namespace axf
