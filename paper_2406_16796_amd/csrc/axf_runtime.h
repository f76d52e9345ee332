// axf_runtime.h -- host-side run object and memory layout of libaxf.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "axf_internal.h"

namespace axf {

// Byte offsets of every array of one run inside its device buffer (-1 = absent).
struct Layout {
    int n[3], nn[3];
    long px;                     // padded row length (elements)
    size_t arr_bytes;            // bytes of one field array
    long npts;
    size_t off_rk;               // device copy of the run descriptor
    size_t off_state;            // start of the checkpointed region
    size_t off_arrays, arr_stride, off_faces, face_stride;
    size_t arr_sink;             // start of an array's store sink (3D), from the array's start
    int nem, nph;                // time-level slots of the E/B arrays and of the axion levels
    long off_em[4][kEmSlots][3];        // [E0,B0,E1,B1][slot][component]
    long off_phi[kPhiSlots];
    long off_c[3];
    long off_axg[3][2][kPhiSlots];
    long off_murg[2][3][2][3][kEmSlots];
    int diag_blocks;
    size_t off_part;
    int rec_cap;
    size_t off_rec;
    long inc_face, off_inc;
    long np;                     // particles (Sec. II.B; 0: none)
    long off_pa[13];             // their arrays (-1 = absent)
    long off_j[2][3];            // currents of both orders at the E points (-1 = absent)
    size_t total;
};

struct Run {
    axf_config cfg;
    Layout L;
    char *base = nullptr;
    hipStream_t stream = nullptr;
    double s_phi = 1.0, s_1 = 1.0;
    RunK<float> hf;
    RunK<double> hd;
    int64_t step = 0;
    bool converted = false;
    int64_t ephase_step = -1;
    int64_t rec_written = 0;
    int64_t launches = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int64_t timed_steps = 0, timed_launches = 0;
    bool batch_owned = false;
    bool use_fused = false;
    int chunk = 0;                 // fused planes per workgroup (0: default)
    int pd = 0;                    // 2D wavefront prefetch distance (0: default)
    bool lds_march = false;          // 2D fused: the LDS-marching kernel instead of the wavefront one
    bool multi = true;               // 2D fused: advance several steps per pass where possible
    int pass_ci = 0, pass_cf = 0;    // ... rows per interior / frame wavefront (0: default)
    int pass_pd = 0;                 // ... prefetch distance of the interior (0: default)
    int pass_steps = 0;              // ... most steps per pass (2, 3 or 4; 0: default)
    bool pass_ring = true;           // ... three- and four-step interior as core and ring launches
    hipStream_t side = nullptr;      // 2D fused: stream of the boundary-frame launch (created on use)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipStream_t ring = nullptr;      // 2D fused: stream of the interior's ring (passes of several steps)
    hipEvent_t ev_ring = nullptr;
    long inc_lo = -1;               // first time level held by the laser table
    bool m3_off = false;            // 3D: the tile-walk launches instead of the one-pass march
    bool m3_on = false;             // 3D FP64: the one-pass march instead of the tile walks
    int m3_chunk = 0;               // 3D march: planes per workgroup (0: default)
    long win_shifted = 0;           // columns the moving window has moved so far

    template <typename T> const RunK<T>& hk() const;
    template <typename T> const RunK<T> *rk() const { return (const RunK<T> *)(base + L.off_rk); }
};

template <> inline const RunK<float>& Run::hk<float>() const { return hf; }
template <> inline const RunK<double>& Run::hk<double>() const { return hd; }

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int validate(const axf_config *c);
// the moving window: columns moved by the start of step n; one move of the
// state by `cells` columns; the descriptor's slab and laser switch for the
// columns moved so far
long window_target(const axf_config& c, long n);
int run_window_move(Run *R, int cells);
int run_window_desc(Run *R);
Layout make_layout(const axf_config *c);
int run_init(Run *R, const axf_config *cfg, void *dev_buf, size_t bytes, hipStream_t stream);
int run_step(Run *R, int64_t nsteps);
// leapfrog conversion before the first step (idempotent)
int run_prepare(Run *R);
// the run steps with the 2D wavefront kernel; its rows per march
bool run_wave2d(const Run *R);
int run_wave_chunk(const Run *R);
// the run steps with the one-pass 3D march
bool run_march3d(const Run *R);
// rows per interior and frame wavefront of a pass of several steps, and the
// most steps per pass
void run_pass_shape(const Run *R, int ns, int *ci, int *cf);
int run_pass_steps(const Run *R);
// the most steps per pass this run's grid and shape give (1: one step per pass)
int run_pass_steps_taken(const Run *R);
// tuned 2D wavefront shapes for a configuration, if recorded: the best one-step
// shape, the best shape of passes of several steps (with their number) and
// whether those passes are faster
struct TunedShape {
    int chunk = 0, pd = 0;
    bool multi = true;
    int pass_steps = 0, pass_ci = 0, pass_cf = 0, pass_pd = 0;
};
bool tuned_shape(const axf_config *c, TunedShape *out);
int run_diag_now(Run *R, axf_diag_record *out);
int run_diag_now_static(Run *R, int rows, axf_diag_record *out);
void run_release(Run *R);
bool fused_supported(const axf_config *c);

}  // namespace axf

// the opaque handle of the C ABI is the run object itself
struct axf_run : public axf::Run {};
