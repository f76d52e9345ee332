// axf_internal.h -- device-side run descriptor and helpers shared by the
// kernels and the host runtime of libaxf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/axf.h"

namespace axf {

// Laser injected through x_min (parameters in FP64).
struct Laser {
    int on, pol, env, q;          // q = number of transverse axes of the beam profile
    int order;                    // the field order the laser is injected into (0 or 1)
    double omega, e_amp, ramp_t, tau0, t_center, waist, x_focus, y_c, z_c, cep, zr;
};

struct Packet {
    int on, dir;
    double amp, k, w, x0, y0, z0;
};

// Active components per dimensionality (the others stay identically zero for
// the accepted configurations): 1D keeps the transverse components of both
// polarisations, 2D keeps the in-plane-polarised zero-order set (E0x E0y B0z)
// and all first-order components, 3D keeps everything.
template <int D> __host__ __device__ constexpr bool actE0(int c) { return D == 3 ? true : (D == 2 ? c != 2 : c != 0); }
template <int D> __host__ __device__ constexpr bool actB0(int c) { return D == 3 ? true : (D == 2 ? c == 2 : c != 0); }
template <int D> __host__ __device__ constexpr bool actE1(int c) { return D >= 2 ? true : c != 0; }
template <int D> __host__ __device__ constexpr bool actB1(int c) { return D >= 2 ? true : c != 0; }

// Time levels rotate through slots: the E/B buffers and the Mur ghosts
// through nem (step n reads slot n mod nem, writes slot (n + 1) mod nem), the
// axion levels and their ghosts through nph (level L, the field at
// t = (L - 1/2) dt, in slot L mod nph).  2D runs keep five and six: a pass of
// up to four steps reads the slots of step n while its launches write those
// of steps n + 1 .. n + 4, all distinct.  1D runs keep as many: a pass of K
// steps reads the slots of step n and writes those of step n + K, which five
// and six keep apart for K = 2, 3, 4, 8, 9, 14, 16, ... (tiny arrays).  3D
// runs advance one step per launch and keep two and three (the old and new
// E/B; the two axion levels a step reads and the one it writes).
constexpr int kEmSlots = 5, kPhiSlots = 6;      // the most a run keeps
__host__ __device__ constexpr int em_slots_of(int D) { return D == 3 ? 2 : kEmSlots; }
__host__ __device__ constexpr int phi_slots_of(int D) { return D == 3 ? 3 : kPhiSlots; }
__host__ __device__ constexpr int em_slot(long step, int nem) { return (int)(step % nem); }
__host__ __device__ constexpr int phi_slot(long level, int nph) { return (int)(level % nph); }

// Uniform layout of a run's device buffer: 12 nem + nph + 3 field arrays of
// equal size at state_base + q * arr_stride (the 12 EM components of one slot
// together, slot after slot, then the axion levels and the current scratch),
// and 216 boundary planes of equal size at face_base + q * face_stride (some
// unused for a given configuration).
constexpr int kEmPerSlot = 12;
__host__ __device__ constexpr int q_em(int kind, int slot, int comp) { return slot * kEmPerSlot + kind * 3 + comp; }  // kind 0 E0, 1 B0, 2 E1, 3 B1
__host__ __device__ constexpr int q_phi(int nem, int slot) { return nem * kEmPerSlot + slot; }
__host__ __device__ constexpr int q_c(int nem, int nph, int comp) { return q_phi(nem, nph) + comp; }
__host__ __device__ constexpr int num_arrays(int nem, int nph) { return q_c(nem, nph, 3); }
__host__ __device__ constexpr int q_axg(int d, int side, int slot) { return (d * 2 + side) * kPhiSlots + slot; }
__host__ __device__ constexpr int q_mur(int o, int d, int side, int comp, int slot)
{
    return 6 * kPhiSlots + (((o * 3 + d) * 2 + side) * 3 + comp) * kEmSlots + slot;
}
constexpr int kNumFaces = 6 * kPhiSlots + 36 * kEmSlots;
constexpr int kIncLevels = 17;   // time levels per laser table fill (16 steps)
constexpr int kWinMaxCells = 64; // the most columns one move of a moving window shifts
constexpr int kDiagSums = 6;     // FP64 partial sums per block of a diagnostic record
// static diagnostic workspace (axf_diag_now_static): at most kStaticDiagRows
// block partials, then one record
constexpr int kStaticDiagRows = 1024;
constexpr int kStaticRecDoubles = 32;
constexpr int kPmlProf = 64;     // damping-layer thicknesses the wavefront interiors tabulate
constexpr long kSinkBytes = 65536;   // per-array store sink of 3D runs (128 wavefronts x 64 lanes x 8 bytes)

// Immutable per-run descriptor, stored in device memory once at creation.
// Time-level slots rotate with the step counter (em_slot, phi_slot).
template <typename T>
struct RunK {
    int D;
    int nem, nph;             // E/B and axion time-level slots (em_slots_of, phi_slots_of)
    int n[3], nn[3];          // cells, storage extents (n + 1 on Mur axes)
    int mur[3], axbc[3];
    long sx, sy;              // element strides of j and k
    long npts;                // nn0 * nn1 * nn2
    // coefficients in storage precision
    T cdt[3];                 // dt / dx
    T inv_dt, inv2dx[3], inv_dx2[3], dt2, m2, gax, cg1, half;
    T bext[3];
    int slab_lo, slab_hi;
    T pml_sdt_max;            // sigma_max * dt
    int pml_n;
    // sigma dt at distance d < pml_n from the face (d < kPmlProf), computed with
    // the point formula's operations, so a table value is the formula's bits
    T pml_prof[kPmlProf];
    T out_r[3];               // dt / dx for the outflow ghost solve
    // FP64 parameters
    double dt, dx[3], murc[3], m2d;
    double s_phi, s_1;
    Laser las;
    Packet pk;
    // state (uniform layout, see q_em / q_axg; the pointers below point into it)
    char *state_base, *face_base;
    long arr_stride, face_stride;
    long arr_sink;            // byte offset of each array's store sink (3D; see kSinkBytes)
    T *E0[kEmSlots][3], *B0[kEmSlots][3], *E1[kEmSlots][3], *B1[kEmSlots][3];
    T *phi[kPhiSlots];
    T *C[3];                  // scratch: axion current at centres (plain path)
    T *axg[3][2][kPhiSlots];          // axion ghosts [axis][side][slot]
    T *murg[2][3][2][3][kEmSlots];    // Mur ghosts [order][axis][side][component][slot]
    // incident laser field on the x_min face, tabulated per time level L
    // (t = (L - 1/2) dt) in slot L mod inc_k1: [slot][0 adjacent centre, 1 ghost][face point]
    double *inc;
    int inc_k1;
    long inc_face;
    // diagnostics
    double *part;             // per-block partial sums, 4 per block
    int diag_blocks;
    axf_diag_record *rec;     // device ring of records (slot chosen by the host)
    int rec_cap;
    // particles (Sec. II.B): count; arrays x y z, ux uy uz (zero order), the
    // same of first order (stored scaled by 1/s_1 like E1), density carried;
    // currents j0, j1 (j1 scaled) at the E points, t_n (null without particles)
    long np;
    T *pa[13];
    T *J[2][3];
    // the initial lattice: particles per cell, first plasma cell, density per
    // particle, initial momentum
    int ppc[2], plasma_lo, plasma_cells;
    T pw0, pu0[3];
};

__host__ __device__ inline long round_up(long v, long m) { return (v + m - 1) / m * m; }

// One run of a batched launch.  A batched launch covers the first `n` runs of a
// table sorted by remaining steps; blk[K] is the first block of the run in
// launches of kind K, and entry n holds the totals.  Every run computes exactly
// what its own single-run launch would.
enum BlockKind {
    kVolume = 0, kFace, kLaser, kWave, kWaveI,
    kPair, kFrameA, kFrameB,           // two-step pass: interior, frames of steps n and n + 1
    kQuadCore, kQuadRing, kQuadFrame,  // four-step pass: interior core and ring, frame (every step)
    kWave1,                            // fused 1D pass: one workgroup per window
    kNumKinds
};
struct BItem {
    const void *rk;     // the run's RunK<T> (device)
    long step0;         // the run's step counter at the first step of the call
    long rec0;          // diagnostic records written before the call
    long blk[kNumKinds];
    int chunk;          // rows per wavefront march (fused 2D, one step per pass)
    int pass_ci;        // rows per interior / frame wavefront of a two-step pass
    int pass_cf;
    int quad_ci;        // ... of a four-step pass
    int quad_cf;
};

// the run descriptor of a table entry as a wave-uniform pointer into global
// memory, so that the compiler reads its fields with scalar loads as it does
// for a descriptor passed as a kernel argument
template <typename R>
__device__ __forceinline__ const R *uniform_desc(const void *p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (const R *)(const __attribute__((address_space(1))) R *)(((unsigned long long)hi << 32) | lo);
}

// Workgroups of a launch are dealt to the 8 XCDs in turn, each XCD with its
// own L2.  xcd_band renumbers block b of nb so that each XCD takes one
// contiguous band of the launch order: tiles that share rows or planes with
// their neighbours then meet in the same L2.  A bijection on [0, nb).
__device__ __forceinline__ long xcd_band(long b, long nb)
{
    const long per = (nb + 7) / 8, full = nb % 8 == 0 ? 8 : nb % 8;
    const long x = b % 8, q = b / 8;
    return x < full ? x * per + q : full * per + (x - full) * (per - 1) + q;
}

// index of the run owning block b of a launch of kind K (largest i with blk[K] <= b)
template <int K>
__device__ __forceinline__ int find_item(const BItem *it, int n, long b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (it[mid].blk[K] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace axf
