// axf_particles.hip -- the particle side of the first-order expansion
// (Sec. II.B) for 2D runs: cold electrons (charge -1, mass 1) pushed by the
// zero-order fields, and their first-order perturbations.
//
// Zero order: a Boris push (J. P. Boris 1970) by E0 and B0 + B_ext.  First
// order: the derivative of that push along the perturbation, so that x1, u1
// follow the linearised motion of Sec. II.B,
//   dx1/dt = v1,  dp1/dt = q (E_p + v0 x B_p + v1 x B_nop),
//   v1 = (gamma0^2 u1 - u0 (u0.u1)) / gamma0^3,
// with the fields felt to first order F_p = sum S F1 + sum (grad S . x1) F0.
// Currents are deposited at the E points with the same linear shape:
//   j0 = q w S v0,   j1 = q w [(grad S . x1) v0 + S v1],
// the three-term expansion of Sec. II.B (the first term is j0).
//
// Time levels: x^n, u^n at integer times.  A step drifts x half a step with
// v^n, kicks u with E^{n+1/2} and B^{n+1/2} (the mean of B^n and B^{n+1})
// at that midpoint, drifts again with v^{n+1}, and deposits dt j^{n+1} at
// x^{n+1}; the E updates of the next step subtract it.  One thread per
// particle; the deposit is an atomic addition, so the sums' order (and
// their last bits) vary from run to run.  Lanes of a wavefront hold
// consecutive particles, in consecutive cells of a row at the start: a lane
// adds its lower neighbour's value at the point they share, which halves
// the atomics of a row of particles.
//
// The 2D field set keeps E0x, E0y, B0z and all first-order components, so
// the zero-order motion stays in the plane (B_ext along z, in-plane initial
// momenta): u0z = 0 and j0z = 0 throughout.
#include "axf_kernels.h"
#include "axf_stencil.h"

namespace axf {

namespace {

// the two points along axis d (0 or 1: particles move in 2D runs) of a
// component nodal (or centred) along d, their weights and the weights'
// derivatives
template <typename T>
struct Sh1 {
    int i[2];
    T w[2], dw[2];
};

template <typename T>
__device__ __forceinline__ void shape1(const RunK<T>& r, int d, bool nodal, T x, Sh1<T>& s)
{
    const T idx = T(2) * r.inv2dx[d];
    const T u = x * idx - (nodal ? T(0) : T(0.5));
    const T f0 = floor(u), f = u - f0;
    int i0 = (int)f0, i1 = i0 + 1;
    if (!r.mur[d]) {
        i0 = wrapi(i0, r.n[d]);
        i1 = wrapi(i1, r.n[d]);
    }
    s.i[0] = i0;
    s.i[1] = i1;
    s.w[0] = T(1) - f;
    s.w[1] = f;
    s.dw[0] = -idx;
    s.dw[1] = idx;
}

// value and gradient term of component c at X: sum S F and sum (grad S . dX) F,
// F the mean of two arrays (b: null for one), on the B points (isB) or the E
// points, with B_ext (bx) added
template <typename T>
__device__ __forceinline__ void gather(const RunK<T>& r, const T *a, const T *b, int c, bool isB, bool bx,
                                       const T X[2], const T dX[2], T& val, T& grad)
{
    val = T(0);
    grad = T(0);
    const T ext = bx ? r.bext[c] : T(0);
    if (!a && ext == T(0)) return;
    Sh1<T> sx, sy;
    shape1(r, 0, isB ? c != 0 : c == 0, X[0], sx);
    shape1(r, 1, isB ? c != 1 : c == 1, X[1], sy);
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int p = 0; p < 2; p++) {
            const long id = lin(r, sx.i[p], sy.i[q], 0);
            T f = a ? (b ? r.half * (a[id] + b[id]) : a[id]) : T(0);
            if (bx) f += bext_at(r, c, sx.i[p]);
            const T w = sx.w[p] * sy.w[q];
            const T gw = sx.dw[p] * sy.w[q] * dX[0] + sx.w[p] * sy.dw[q] * dX[1];
            val += w * f;
            grad += gw * f;
        }
}

// J_c += a S + b (grad S . dX) at the E_c points
template <typename T>
__device__ __forceinline__ void deposit(const RunK<T>& r, T *J, int c, const T X[2], const T dX[2], T a, T b)
{
    if (!J) return;
    Sh1<T> sx, sy;
    shape1(r, 0, c == 0, X[0], sx);
    shape1(r, 1, c == 1, X[1], sy);
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int p = 0; p < 2; p++) {
            const T w = sx.w[p] * sy.w[q];
            const T gw = sx.dw[p] * sy.w[q] * dX[0] + sx.w[p] * sy.dw[q] * dX[1];
            atomicAdd(&J[lin(r, sx.i[p], sy.i[q], 0)], a * w + b * gw);
        }
}

// wrap on periodic axes; false once a particle comes within 1.5 cells of a Mur face
template <typename T>
__device__ __forceinline__ bool place(const RunK<T>& r, T X[2])
{
    for (int d = 0; d < 2; d++) {
        const T L = T(r.n[d] * r.dx[d]), h = T(1.5 * r.dx[d]);
        if (!r.mur[d]) {
            if (X[d] < T(0)) X[d] += L;
            if (X[d] >= L) X[d] -= L;
        } else if (X[d] < h || X[d] > L - h) {
            return false;
        }
    }
    return true;
}

template <typename T>
__device__ __forceinline__ void cross(const T a[3], const T b[3], T o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename T>
__device__ __forceinline__ T dot3(const T a[3], const T b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// the Boris push of u by E, B (hq = q dt / (2 m)) and its derivative along
// (du, dE, dB)
template <typename T>
__device__ __forceinline__ void boris(const T u[3], const T du[3], const T E[3], const T dE[3], const T B[3],
                                      const T dB[3], T hq, T un[3], T dun[3])
{
    T um[3], dum[3], t[3], dtv[3], sv[3], ds[3], up[3], dup[3], c1[3], c2[3];
    for (int q = 0; q < 3; q++) {
        um[q] = u[q] + hq * E[q];
        dum[q] = du[q] + hq * dE[q];
    }
    const T g = sqrt(T(1) + dot3(um, um)), dg = dot3(um, dum) / g;
    for (int q = 0; q < 3; q++) {
        t[q] = hq * B[q] / g;
        dtv[q] = hq * dB[q] / g - hq * B[q] * dg / (g * g);
    }
    const T tt = dot3(t, t), dtt = T(2) * dot3(t, dtv), den = T(1) + tt;
    for (int q = 0; q < 3; q++) {
        sv[q] = T(2) * t[q] / den;
        ds[q] = T(2) * dtv[q] / den - T(2) * t[q] * dtt / (den * den);
    }
    cross(um, t, c1);
    for (int q = 0; q < 3; q++) up[q] = um[q] + c1[q];
    cross(dum, t, c1);
    cross(um, dtv, c2);
    for (int q = 0; q < 3; q++) dup[q] = dum[q] + c1[q] + c2[q];
    T upl[3], dupl[3];
    cross(up, sv, c1);
    for (int q = 0; q < 3; q++) upl[q] = um[q] + c1[q];
    cross(dup, sv, c1);
    cross(up, ds, c2);
    for (int q = 0; q < 3; q++) dupl[q] = dum[q] + c1[q] + c2[q];
    for (int q = 0; q < 3; q++) {
        un[q] = upl[q] + hq * E[q];
        dun[q] = dupl[q] + hq * dE[q];
    }
}

template <typename T>
__device__ __forceinline__ void velocity(const T u[3], const T du[3], T v[3], T dv[3])
{
    const T g = sqrt(T(1) + dot3(u, u)), ud = dot3(u, du);
    for (int q = 0; q < 3; q++) {
        v[q] = u[q] / g;
        dv[q] = (g * g * du[q] - u[q] * ud) / (g * g * g);
    }
}

// dt j0 and dt j1 (stored scale) of one particle at X, dX with v, dv
template <typename T>
__device__ __forceinline__ void deposit_particle(const RunK<T>& r, T w, const T X[2], const T dX[2], const T v[3],
                                                 const T dv[3])
{
    const T qw = T(-r.dt) * w;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        deposit(r, r.J[0][c], c, X, dX, qw * v[c], T(0));
        deposit(r, r.J[1][c], c, X, dX, qw * dv[c], qw * v[c]);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_part_init(const RunK<T> *__restrict__ rp)
{
    const RunK<T>& r = *rp;
    const long p = blockIdx.x * 256L + threadIdx.x;
    if (p >= r.np) return;
    const int px = r.ppc[0], py = r.n[1] > 1 ? r.ppc[1] : 1;
    long q = p;
    const int a = (int)(q % px);
    q /= px;
    const int b = (int)(q % py);
    q /= py;
    const int i = r.plasma_lo + (int)(q % r.plasma_cells);
    const int j = (int)(q / r.plasma_cells);
    r.pa[0][p] = (T)((i + (a + 0.5) / px) * r.dx[0]);
    r.pa[1][p] = r.n[1] > 1 ? (T)((j + (b + 0.5) / py) * r.dx[1]) : T(0);
    r.pa[2][p] = T(0);
    for (int c = 0; c < 3; c++) {
        r.pa[3 + c][p] = r.pu0[c];
        r.pa[6 + c][p] = T(0);
        r.pa[9 + c][p] = T(0);
    }
    r.pa[12][p] = r.pw0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_jzero(const RunK<T> *__restrict__ rp)
{
    const RunK<T>& r = *rp;
    const long p = blockIdx.x * 256L + threadIdx.x;
    if (p >= r.sy * r.nn[2]) return;
    for (int o = 0; o < 2; o++)
        for (int c = 0; c < 3; c++)
            if (r.J[o][c]) r.J[o][c][p] = T(0);
}

// j^n from the particles as they are (the initial current)
template <typename T>
__global__ void __launch_bounds__(256) k_deposit(const RunK<T> *__restrict__ rp)
{
    const RunK<T>& r = *rp;
    const long p = blockIdx.x * 256L + threadIdx.x;
    if (p >= r.np) return;
    const T w = r.pa[12][p];
    if (w == T(0)) return;
    T X[2] = {r.pa[0][p], r.pa[1][p]}, dX[2] = {r.pa[6][p], r.pa[7][p]};
    T u[3], du[3], v[3], dv[3];
    for (int c = 0; c < 3; c++) {
        u[c] = r.pa[3 + c][p];
        du[c] = r.pa[9 + c][p];
    }
    velocity(u, du, v, dv);
    deposit_particle(r, w, X, dX, v, dv);
}

// J_c += a S + b (grad S . dX) at the E_c points, every lane of the wavefront
// taking part (live: this lane has a particle to deposit).  Along x a lane's
// upper point is often the next lane's lower point (consecutive particles sit
// in consecutive cells of a row): the next lane then adds both values with one
// atomic and this lane leaves that point out.
template <typename T>
__device__ __forceinline__ void deposit_w(const RunK<T>& r, T *J, int c, const T X[2], const T dX[2], T a, T b,
                                          bool live)
{
    if (!J) return;
    Sh1<T> sx, sy;
    shape1(r, 0, c == 0, X[0], sx);
    shape1(r, 1, c == 1, X[1], sy);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const long i0 = lin(r, sx.i[0], sy.i[q], 0), i1 = lin(r, sx.i[1], sy.i[q], 0);
        const T v0 = a * (sx.w[0] * sy.w[q]) + b * (sx.dw[0] * sy.w[q] * dX[0] + sx.w[0] * sy.dw[q] * dX[1]);
        const T v1 = a * (sx.w[1] * sy.w[q]) + b * (sx.dw[1] * sy.w[q] * dX[0] + sx.w[1] * sy.dw[q] * dX[1]);
        const long pi1 = __shfl_up(i1, 1), ni0 = __shfl_down(i0, 1);
        const T pv1 = __shfl_up(v1, 1);
        const int plive = __shfl_up((int)live, 1), nlive = __shfl_down((int)live, 1);
        const bool absorb = lane > 0 && plive && pi1 == i0;
        const bool given = lane < 63 && nlive && ni0 == i1;
        // a zero term changes no sum (the arrays start at +0), and a plasma at
        // rest deposits nothing but zeros to zero order
        const T s0 = absorb ? v0 + pv1 : v0;
        if (live && s0 != T(0)) atomicAdd(&J[i0], s0);
        if (live && !given && v1 != T(0)) atomicAdd(&J[i1], v1);
    }
}

// one step of every particle with E^{n+1/2} (slot sn) and B^{n+1/2} (mean of
// slots so and sn), then dt j^{n+1}.  Every lane of a wavefront with a live
// particle runs to the end, so that the deposit's lane exchanges see the
// whole wavefront: a lane past the last particle reads the last one's state,
// a lane without a live particle gathers at the grid's centre, and neither
// stores or deposits anything.
template <typename T>
__global__ void __launch_bounds__(256) k_push(const RunK<T> *__restrict__ rp, long step)
{
    const RunK<T>& r = *rp;
    const long p0 = blockIdx.x * 256L + threadIdx.x;
    const bool valid = p0 < r.np;
    const long p = valid ? p0 : r.np - 1;
    T w = r.pa[12][p];
    bool live = valid && w != T(0);
    const int so = em_slot(step, r.nem), sn = em_slot(step + 1, r.nem);
    const T hdt = T(0.5 * r.dt), hq = T(-0.5 * r.dt);
    T X[2] = {r.pa[0][p], r.pa[1][p]}, dX[2] = {r.pa[6][p], r.pa[7][p]};
    T u[3], du[3], v[3], dv[3];
    for (int c = 0; c < 3; c++) {
        u[c] = r.pa[3 + c][p];
        du[c] = r.pa[9 + c][p];
    }
    velocity(u, du, v, dv);
    for (int d = 0; d < 2; d++) {
        X[d] += hdt * v[d];
        dX[d] += hdt * dv[d];
    }
    if (live && !place(r, X)) {
        r.pa[12][p] = T(0);
        live = false;
    }
    if (__ballot(live) == 0) return;   // uniform: the wavefront has nothing left to do
    if (!live) {
        X[0] = T(0.5 * r.n[0] * r.dx[0]);
        X[1] = T(0.5 * r.n[1] * r.dx[1]);
    }
    T E0[3], Ep[3], B0[3], Bp[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        T f, gf, f1, g1;
        gather(r, r.E0[sn][c], (const T *)nullptr, c, false, false, X, dX, f, gf);
        gather(r, r.E1[sn][c], (const T *)nullptr, c, false, false, X, dX, f1, g1);
        E0[c] = f;
        Ep[c] = f1 + gf;
        gather(r, r.B0[so][c], r.B0[sn][c], c, true, true, X, dX, f, gf);
        gather(r, r.B1[so][c], r.B1[sn][c], c, true, false, X, dX, f1, g1);
        B0[c] = f;
        Bp[c] = f1 + gf;
    }
    T un[3], dun[3];
    boris(u, du, E0, Ep, B0, Bp, hq, un, dun);
    velocity(un, dun, v, dv);
    for (int d = 0; d < 2; d++) {
        X[d] += hdt * v[d];
        dX[d] += hdt * dv[d];
    }
    const bool in = place(r, X);
    if (live) {
        r.pa[0][p] = X[0];
        r.pa[1][p] = X[1];
        r.pa[6][p] = dX[0];
        r.pa[7][p] = dX[1];
        for (int c = 0; c < 3; c++) {
            r.pa[3 + c][p] = un[c];
            r.pa[9 + c][p] = dun[c];
        }
        if (!in) r.pa[12][p] = T(0);
    }
    live = live && in;
    if (!live) X[0] = T(0.5 * r.n[0] * r.dx[0]), X[1] = T(0.5 * r.n[1] * r.dx[1]);
    const T qw = T(-r.dt) * w;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        deposit_w(r, r.J[0][c], c, X, dX, qw * v[c], T(0), live);
        deposit_w(r, r.J[1][c], c, X, dX, qw * dv[c], qw * v[c], live);
    }
}

unsigned blocks_of(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename T>
void Particles<T>::init(const RunK<T> *rk, const RunK<T>& h, hipStream_t st)
{
    if (h.np == 0) return;
    hipLaunchKernelGGL((k_part_init<T>), dim3(blocks_of(h.np)), dim3(256), 0, st, rk);
    deposit(rk, h, st);
}

template <typename T>
void Particles<T>::deposit(const RunK<T> *rk, const RunK<T>& h, hipStream_t st)
{
    if (h.np == 0) return;
    hipLaunchKernelGGL((k_jzero<T>), dim3(blocks_of(h.sy * h.nn[2])), dim3(256), 0, st, rk);
    hipLaunchKernelGGL((k_deposit<T>), dim3(blocks_of(h.np)), dim3(256), 0, st, rk);
}

template <typename T>
void Particles<T>::push(const RunK<T> *rk, const RunK<T>& h, long step, hipStream_t st)
{
    if (h.np == 0) return;
    hipLaunchKernelGGL((k_jzero<T>), dim3(blocks_of(h.sy * h.nn[2])), dim3(256), 0, st, rk);
    hipLaunchKernelGGL((k_push<T>), dim3(blocks_of(h.np)), dim3(256), 0, st, rk, step);
}

template struct Particles<float>;
template struct Particles<double>;

}  // namespace axf
