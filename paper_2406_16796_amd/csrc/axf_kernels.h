// axf_kernels.h -- host-side launchers of the kernels of libaxf.
#pragma once

#include "axf_internal.h"

namespace axf {

// Unfused step: one launch per update phase (the correctness baseline).
template <int D, typename T>
struct Plain {
    static void e0(const RunK<T> *rk, const RunK<T>& h, int s_in, int s_b, int s_out, T scale, hipStream_t st);
    static void c(const RunK<T> *rk, const RunK<T>& h, int pa, int pb, int e_m, int e_p, int s_b, int cotimed, hipStream_t st);
    static void e1(const RunK<T> *rk, const RunK<T>& h, int s_in, int s_b, int s_out, T scale, hipStream_t st);
    static void mur(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st);
    static void mur_init(const RunK<T> *rk, const RunK<T>& h, hipStream_t st);
    static void inc_fill(const RunK<T> *rk, const RunK<T>& h, long L0, int nlev, hipStream_t st);
    static void b(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st);
    static void phi(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st);
    static void init_phi(const RunK<T> *rk, const RunK<T>& h, hipStream_t st);
    static void copy_ghosts(const RunK<T> *rk, const RunK<T>& h, int s0, int s1, hipStream_t st);
    static void diag(const RunK<T> *rk, const RunK<T>& h, long step, int slot, hipStream_t st);
    // the same record from `rows` workgroups folding the point blocks in a
    // fixed order, partials and record in the workspace `ws` (device address
    // of the static array, see static_workspace)
    static void diag_rows(const RunK<T> *rk, const RunK<T>& h, long step, double *ws, int rows, hipStream_t st);
    // semi-fused step: E0 with the axion current, B with the axion update
    static void e0c(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st);
    // the semi-fused step's launches (E0+C, E1, Mur, B, axion) on 3D tile walks
    // of tz planes per workgroup (0: default)
    static void tiled_step(const RunK<T> *rk, const RunK<T>& h, long step, int tz, hipStream_t st);
    // batched launches over the first n runs of a sorted table (device `it`,
    // host copy `host` for the grid sizes) at step s of the call
    static void batch_step(const BItem *it, const BItem *host, int n, long s, hipStream_t st);
    static void batch_inc_fill(const BItem *it, const BItem *host, int n, long s, int nlev, hipStream_t st);
    static void batch_diag(const BItem *it, const BItem *host, int n, long s, long ev, hipStream_t st);
};

// The particle side of the first-order expansion (2D runs with a plasma):
// the initial lattice and its current j^0, the current of the particles as
// they are, and one step of every particle (after the step's B and axion
// updates; it leaves dt j^{n+1} for the next E updates).
template <typename T>
struct Particles {
    static void init(const RunK<T> *rk, const RunK<T>& h, hipStream_t st);
    static void deposit(const RunK<T> *rk, const RunK<T>& h, hipStream_t st);
    static void push(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st);
};

// device address of the static diagnostic workspace on device `dev` (looked up
// once per device and kept); hipSuccess or the lookup's error
hipError_t static_workspace(int dev, double **ptr);

}  // namespace axf
