// axf_fused.h -- launcher of the fused one-pass step kernel.
#pragma once

#include <type_traits>

#include "axf_internal.h"

namespace axf {

// Fused step for 2D (march along y, tiles of TX cells in x) and 3D (march
// along z, tiles of TX x TY cells in x, y); `chunk` planes per workgroup.
template <int D, int TX, int TY, typename T>
struct Fused {
    static size_t lds_bytes();
    static int threads();
    static hipError_t launch(const RunK<T> *rk, const RunK<T>& h, long step, int chunk, hipStream_t st);
};

// Fused 2D step on wavefront-owned x segments (no LDS, no barriers).
template <typename T>
hipError_t launch_wave2d(const RunK<T> *rk, const RunK<T>& h, long step, int chunk, hipStream_t st);
// the same over the first n runs of a batch table at step s of the call
template <typename T>
hipError_t launch_wave2d_batch(const BItem *it, const BItem *host, int n, long s, hipStream_t st);
// workgroups (4 wavefronts each) of one run's wavefront launch
int wave2d_blocks(int nn0, int nn1, int chunk);

}  // namespace axf
