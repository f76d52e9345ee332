// axf_fused.h -- launcher of the fused one-pass step kernel.
#pragma once

#include <type_traits>

#include "axf_internal.h"

namespace axf {

// A second stream for the boundary-frame launch of the 2D step and the events
// that fork it from and join it back to the run's stream.
struct WaveStreams {
    hipStream_t side;
    hipEvent_t fork, join;
    // three- and four-step passes: the stream of the interior's ring launch (null: the
    // interior in one launch, the frame launches covering the ring instead)
    hipStream_t ring = nullptr;
    hipEvent_t ring_done = nullptr;
};

// Fused step for 2D (march along y, tiles of TX cells in x) and 3D (march
// along z, tiles of TX x TY cells in x, y); `chunk` planes per workgroup.
template <int D, int TX, int TY, typename T>
struct Fused {
    static size_t lds_bytes();
    static int threads();
    static hipError_t launch(const RunK<T> *rk, const RunK<T>& h, long step, int chunk, hipStream_t st);
};

// Fused 2D step on wavefront-owned x segments (no LDS, no barriers): the
// interior launch on `st`, the boundary-frame launch on ws->side when given.
template <typename T>
hipError_t launch_wave2d(const RunK<T> *rk, const RunK<T>& h, long step, int chunk, int pd, hipStream_t st,
                         const WaveStreams *ws);
// the same over the first n runs of a batch table at step s of the call
template <typename T>
hipError_t launch_wave2d_batch(const BItem *it, const BItem *host, int n, long s, hipStream_t st,
                               const WaveStreams *ws);
// NS steps per pass (NS = 2, 3 or 4): the interior advanced NS steps in one
// launch, the frame in NS one-step launches beside it
template <typename T>
bool wave2d_pass_available(const RunK<T>& h, int ns, int ci, int cf);
template <typename T>
hipError_t launch_wave2d_pass(const RunK<T> *rk, const RunK<T>& h, long step, int ns, int ci, int cf, int pd,
                              hipStream_t st, const WaveStreams *ws, bool store_e = false);
// built-in prefetch distance of the interior march for ns steps per pass
int wave2d_default_pd(bool f64, int ns);
// the two-step pass over the first n runs of a batch table: steps s and
// s + 1 of the call for every run (each run with a pass interior)
template <typename T>
hipError_t launch_wave2d_pair_batch(const BItem *it, const BItem *host, int n, long s, hipStream_t st,
                                    const WaveStreams *ws);
// workgroups of one run's three launches of a two-step pass
template <typename T>
void wave2d_pair_blocks(const RunK<T>& h, int ci, int cf, long *interior, long *frame_a, long *frame_b);
// the four-step pass over the first n runs of a batch table: steps s .. s + 3
// of the call for every run (each run with an interior for the pass), split as
// a single run's pass is (needs the side and ring streams of `ws`)
template <typename T>
hipError_t launch_wave2d_quad_batch(const BItem *it, const BItem *host, int n, long s, hipStream_t st,
                                    const WaveStreams *ws);
// workgroups of one run's launches of a four-step pass: the interior's core,
// its ring, and the frame (launched once per step)
template <typename T>
void wave2d_quad_blocks(const RunK<T>& h, int ci, int cf, long blk[3]);
// workgroups (4 wavefronts each) of one run's two wavefront launches: the
// frame next to the domain boundary and the interior
template <typename T>
void wave2d_blocks(const RunK<T>& h, int chunk, long *edge_blocks, long *interior_blocks);

// Fused 1D step: K steps per launch on windows of cells held in LDS, halos
// of K + 1 cells (temporal blocking); the grid in one window when it fits.
// A pass reads the slots of step s and writes those of step s + K: K must
// keep them apart (wave1d_k_ok) and be at most wave1d_kmax.
bool wave1d_k_ok(int k, int nem, int nph);
template <typename T>
int wave1d_kmax();
// the longest pass of at most min(free, kmax) steps that wave1d_k_ok allows,
// preferring one that does not leave exactly one step; 0 if there is none
int wave1d_pick(long free, int kmax, int nem, int nph);
// cells per window (256, 512 or 1024) of a single run's passes or a batch's
int wave1d_window(bool batched);
// workgroups (tiles) of one run's pass with windows of `win` cells
template <typename T>
long wave1d_tiles(const RunK<T>& h, int win);
template <typename T>
hipError_t launch_wave1d(const RunK<T> *rk, const RunK<T>& h, long step, int K, int win, hipStream_t st);
// the same pass over the first n runs of a batch table at step s of the call
template <typename T>
hipError_t launch_wave1d_batch(const BItem *it, const BItem *host, int n, long s, int K, int win, hipStream_t st);

// One-pass 3D step (a z march of row wavefronts stacked along y, y neighbours
// through LDS): x segments of `wid` own columns, groups of own rows, chunks
// of `zc` planes.
struct M3Geom {
    int nseg, wid;   // x segments and own columns per segment (frame launch)
    int sx0, sx1;    // the interior launch's segments
    int xi0, wi;     // first own column of interior segment sx0, own columns per interior segment
    int xa, xc1;     // x-face launch: own columns 0 .. xa - 1 (lanes 2 ..), and xc1 .. nn0 - 1 (lanes 34 ..)
    int nyg;         // row groups
    int gy0, gy1;    // the row groups clear of the y faces
    int nzc;         // plane chunks: [0, zf), pieces of zi planes up to zend, [zend, nn2)
    int zf, zi, zend, nn2;
    int order;       // interior block order (bit 0: row groups fastest; bit 1: a band per XCD)
    int xb;          // the columns outside the interior segments have a launch of their own (Mur x, outflow or reflecting axion x)
};
// the run fits the march (32-bit offsets within an array)
template <typename T>
bool march3d_available(const RunK<T>& h);
// workgroups of one launch with chunks of zc planes (0: default)
template <typename T>
long march3d_blocks(const RunK<T>& h, int zc);
template <typename T>
hipError_t launch_march3d(const RunK<T> *rk, const RunK<T>& h, long step, int zc, hipStream_t st,
                          const WaveStreams *ws);

}  // namespace axf
