// axf_window.hip -- the moving window of Sec. III.B: once the laser is in,
// the simulation window follows it along +x at c.  A move by `cells` columns
// happens at a step boundary, on the state of the leapfrog form (E^{n-1/2},
// B^n, phi^{n-1/2}, phi^{n+1/2} and the boundary planes of those levels):
//   - every field array and every plane of the y and z faces shifts left by
//     `cells` columns; the new columns at x_max are vacuum;
//   - the x_min ghosts take the values that lay at their place before the
//     move (the Mur ghost of E_y, E_z: E^{n-1/2} of column cells - 1; the
//     axion ghosts: both levels of cell cells - 1); the x_max ghosts are vacuum;
//   - the B_ext slab keeps its place in the lab, so it moves left in the
//     window, and the laser is no longer injected.
#include "axf_runtime.h"
#include "axf_stencil.h"

#include <vector>

namespace axf {

namespace {

constexpr int kWinArrays = 32;    // arrays per row-shift launch

template <typename T>
struct WinRows {
    T *base[kWinArrays];
    long pitch[kWinArrays];       // elements from one row to the next
    long first[kWinArrays + 1];   // first block (row) of each array; first[n] = rows in all
    int n;                        // arrays in this launch
    int len;                      // row length (the x extent)
    int cells;
};

// The x-face ghosts of the window after the move, from the columns before
// it: one thread per point (j, k) of the x faces.
template <typename T>
__global__ void __launch_bounds__(256) k_win_xghosts(const RunK<T> *__restrict__ rp, int cells, int so, int la, int lb)
{
    const RunK<T>& r = *rp;
    const long f = (long)blockIdx.x * 256 + threadIdx.x;          // face index k nn1 + j
    if (f >= (long)r.nn[1] * r.nn[2]) return;
    const int j = (int)(f % r.nn[1]), k = (int)(f / r.nn[1]);
    const long src = lin(r, cells - 1, j, k);
    for (int o = 0; o < 2; o++)
        for (int c = 1; c < 3; c++) {
            T *lo = r.murg[o][0][0][c][so], *hi = r.murg[o][0][1][c][so];
            const T *E = o == 0 ? r.E0[so][c] : r.E1[so][c];
            if (lo) lo[f] = E ? E[src] : T(0);
            if (hi) hi[f] = T(0);
        }
    if (r.axbc[0] != AXF_AX_PERIODIC && j < r.n[1] && k < r.n[2]) {
        const int lv[2] = {la, lb};
        for (int q = 0; q < 2; q++) {
            r.axg[0][0][lv[q]][f] = r.phi[lv[q]][src];
            r.axg[0][1][lv[q]][f] = T(0);
        }
    }
}

// One workgroup of 256 threads per row: the row moves left by `cells`.
// With R > 0 (rows of at most 256 R elements) the whole row passes through
// registers: every read, one barrier, every write, so that a thread has R
// loads in flight.  With R = 0 the row goes in chunks of 256: every read of
// a chunk lands before its writes (the barrier), and no later chunk reads
// what an earlier one wrote (a chunk writes [c0, c0 + 256) and reads
// [c0 + cells, c0 + 256 + cells)).
template <typename T, int R>
__global__ void __launch_bounds__(256) k_win_rows(WinRows<T> w)
{
    const long b = blockIdx.x;
    int a = 0;
    while (a + 1 < w.n && w.first[a + 1] <= b) a++;
    T *row = w.base[a] + (b - w.first[a]) * w.pitch[a];
    const int t = (int)threadIdx.x;
    if constexpr (R > 0) {
        T v[R];
#pragma unroll
        for (int q = 0; q < R; q++) {
            const int i = q * 256 + t;
            v[q] = (i + w.cells < w.len) ? row[i + w.cells] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; q++) {
            const int i = q * 256 + t;
            if (i < w.len) row[i] = v[q];
        }
    } else {
        for (int c0 = 0; c0 < w.len; c0 += 256) {
            const int i = c0 + t;
            const T v = (i + w.cells < w.len) ? row[i + w.cells] : T(0);
            __syncthreads();
            if (i < w.len) row[i] = v;
        }
    }
}

// the row-shift launch for rows of w.len elements
template <typename T>
void launch_win_rows(const WinRows<T>& w, long rows, hipStream_t st)
{
    const dim3 g((unsigned)rows), b(256);
    if (w.len <= 4 * 256) hipLaunchKernelGGL((k_win_rows<T, 4>), g, b, 0, st, w);
    else if (w.len <= 8 * 256) hipLaunchKernelGGL((k_win_rows<T, 8>), g, b, 0, st, w);
    else if (w.len <= 16 * 256) hipLaunchKernelGGL((k_win_rows<T, 16>), g, b, 0, st, w);
    else if (w.len <= 32 * 256) hipLaunchKernelGGL((k_win_rows<T, 32>), g, b, 0, st, w);
    else hipLaunchKernelGGL((k_win_rows<T, 0>), g, b, 0, st, w);
}

// the run descriptor's slab (window coordinates) and laser switch
template <typename T>
__global__ void k_win_desc(RunK<T> *rp, int slab_lo, int slab_hi, int las_on)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        rp->slab_lo = slab_lo;
        rp->slab_hi = slab_hi;
        rp->las.on = las_on;
    }
}

template <typename T>
RunK<T>& host_desc(Run *R);
template <>
RunK<float>& host_desc<float>(Run *R) { return R->hf; }
template <>
RunK<double>& host_desc<double>(Run *R) { return R->hd; }

template <typename T>
int window_desc(Run *R)
{
    RunK<T>& h = host_desc<T>(R);
    h.slab_lo = (int)(R->cfg.slab_lo - R->win_shifted);
    h.slab_hi = (int)(R->cfg.slab_hi - R->win_shifted);
    h.las.on = R->cfg.laser_on && R->win_shifted == 0;
    hipLaunchKernelGGL((k_win_desc<T>), dim3(1), dim3(64), 0, R->stream, (RunK<T> *)R->rk<T>(), h.slab_lo, h.slab_hi,
                       h.las.on);
    return hipGetLastError() == hipSuccess ? AXF_OK : fail(AXF_EHIP, "window descriptor update");
}

template <typename T>
int window_move(Run *R, int cells)
{
    const RunK<T>& h = R->hk<T>();
    const RunK<T> *rk = R->rk<T>();
    const long s = R->step;
    const int so = em_slot(s, h.nem), la = phi_slot(s, h.nph), lb = phi_slot(s + 1, h.nph);
    const long nface = (long)h.nn[1] * h.nn[2];
    hipLaunchKernelGGL((k_win_xghosts<T>), dim3((unsigned)((nface + 255) / 256)), dim3(256), 0, R->stream, rk, cells, so,
                       la, lb);
    // the arrays and planes that move, as rows along x
    struct Arr { T *p; long rows, pitch; };
    std::vector<Arr> arrs;
    const long rows = (long)h.nn[1] * h.nn[2];
    for (int c = 0; c < 3; c++) {
        T *const kinds[4] = {h.E0[so][c], h.B0[so][c], h.E1[so][c], h.B1[so][c]};
        for (T *p : kinds)
            if (p) arrs.push_back({p, rows, h.sx});
    }
    arrs.push_back({h.phi[la], rows, h.sx});
    arrs.push_back({h.phi[lb], rows, h.sx});
    for (int d = 1; d < 3; d++) {
        const long prow = d == 1 ? h.nn[2] : h.nn[1];     // planes (x, z) and (x, y), x fastest
        for (int side = 0; side < 2; side++) {
            for (int o = 0; o < 2; o++)
                for (int c = 0; c < 3; c++)
                    if (c != d && h.murg[o][d][side][c][so]) arrs.push_back({h.murg[o][d][side][c][so], prow, h.nn[0]});
            if (h.axg[d][side][la]) arrs.push_back({h.axg[d][side][la], prow, h.nn[0]});
            if (h.axg[d][side][lb]) arrs.push_back({h.axg[d][side][lb], prow, h.nn[0]});
        }
    }
    for (size_t a0 = 0; a0 < arrs.size(); a0 += kWinArrays) {
        WinRows<T> w;
        w.n = (int)std::min(arrs.size() - a0, (size_t)kWinArrays);
        w.len = h.nn[0];
        w.cells = cells;
        long tot = 0;
        for (int q = 0; q < w.n; q++) {
            w.base[q] = arrs[a0 + q].p;
            w.pitch[q] = arrs[a0 + q].pitch;
            w.first[q] = tot;
            tot += arrs[a0 + q].rows;
        }
        w.first[w.n] = tot;
        launch_win_rows<T>(w, tot, R->stream);
    }
    if (hipGetLastError() != hipSuccess) return fail(AXF_EHIP, "window move launch");
    R->win_shifted += cells;
    R->ephase_step = -1;
    return window_desc<T>(R);
}

}  // namespace

int run_window_move(Run *R, int cells)
{
    return R->cfg.precision == AXF_F32 ? window_move<float>(R, cells) : window_move<double>(R, cells);
}

int run_window_desc(Run *R)
{
    return R->cfg.precision == AXF_F32 ? window_desc<float>(R) : window_desc<double>(R);
}

long window_target(const axf_config& c, long n)
{
    if (c.win_cells <= 0 || n < 1) return 0;
    const double t = (double)n * c.dt;
    if (t < c.win_t0) return 0;
    return (long)c.win_cells * (long)floor((t - c.win_t0) / ((double)c.win_cells * c.dx[0]));
}

}  // namespace axf
