// axf_batch.hip -- batches of independent runs and the continuous-batching
// server.
//
// Both sit on one stepping engine.  The engine groups runs by the kernels they
// share: dimensionality, precision, the 2D wavefront kernels (and whether the
// grid has an interior for two- and four-step passes) vs the phase sequence.
// Each group's runs are sorted by remaining steps, so the runs still active at
// a step are a prefix of the group's table.  One step (or pass of two or four
// steps) is then one launch per kernel kind and group, whatever the number of
// runs: the 2D wavefront launches, the six unfused phases (1D) or five with E0 and the
// axion current merged (3D); the laser-table fill every 16 steps; the
// diagnostics at the runs' cadence.  Every block of a batched
// launch executes its run's own single-run body with the run's own step
// counter, so a run's result is bit-identical alone and in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "axf_fused.h"
#include "axf_kernels.h"
#include "axf_runtime.h"

namespace axf {

#define BCHK(call)                                               \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hip_fail(e_, #call);        \
    } while (0)

static long cdiv(long a, long b) { return (a + b - 1) / b; }
static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// the run takes passes of ns (2 or 4) steps in batched launches (2D wavefront
// path with an interior for the pass; four only where the run's own passes
// may take four)
static bool run_passes(const Run *R, int ns)
{
    if (!run_wave2d(R) || !R->multi || run_pass_steps(R) < ns) return false;
    int ci = 0, cf = 0;
    run_pass_shape(R, ns, &ci, &cf);
    return R->cfg.precision == AXF_F64 ? wave2d_pass_available(R->hk<double>(), ns, ci, cf)
                                       : wave2d_pass_available(R->hk<float>(), ns, ci, cf);
}
static bool run_pairs(const Run *R) { return run_passes(R, 2); }
static bool run_quads(const Run *R) { return run_pairs(R) && run_passes(R, 4); }

// blocks of each launch kind for one run (the single-run launchers' grids)
static void run_blocks(const Run *R, bool wave, bool pair, bool quad, bool w1, long blk[kNumKinds])
{
    const Layout& L = R->L;
    blk[kVolume] = cdiv(L.npts, 256);
    long face = 0;
    for (int d = 0; d < R->cfg.ndim; d++) {
        if (R->cfg.em_bc[d] != AXF_EM_MUR) continue;
        int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
        face = std::max(face, (long)L.nn[a] * L.nn[b]);
    }
    blk[kFace] = cdiv(face, 256);
    blk[kLaser] = R->cfg.laser_on ? cdiv(L.inc_face, 256) : 0;
    blk[kWave] = blk[kWaveI] = 0;
    if (wave) {
        if (R->cfg.precision == AXF_F64) wave2d_blocks(R->hk<double>(), run_wave_chunk(R), &blk[kWave], &blk[kWaveI]);
        else wave2d_blocks(R->hk<float>(), run_wave_chunk(R), &blk[kWave], &blk[kWaveI]);
    }
    blk[kPair] = blk[kFrameA] = blk[kFrameB] = 0;
    if (pair) {
        int ci = 0, cf = 0;
        run_pass_shape(R, 2, &ci, &cf);
        if (R->cfg.precision == AXF_F64) wave2d_pair_blocks(R->hk<double>(), ci, cf, &blk[kPair], &blk[kFrameA], &blk[kFrameB]);
        else wave2d_pair_blocks(R->hk<float>(), ci, cf, &blk[kPair], &blk[kFrameA], &blk[kFrameB]);
    }
    blk[kQuadCore] = blk[kQuadRing] = blk[kQuadFrame] = 0;
    if (quad) {
        int ci = 0, cf = 0;
        run_pass_shape(R, 4, &ci, &cf);
        if (R->cfg.precision == AXF_F64) wave2d_quad_blocks(R->hk<double>(), ci, cf, &blk[kQuadCore]);
        else wave2d_quad_blocks(R->hk<float>(), ci, cf, &blk[kQuadCore]);
    }
    blk[kWave1] = 0;
    if (w1) {
        const int win = wave1d_window(true);
        blk[kWave1] = R->cfg.precision == AXF_F64 ? wave1d_tiles(R->hd, win) : wave1d_tiles(R->hf, win);
    }
}

// ------------------------------------------------------------------ engine

struct Group {
    int D = 0;
    bool f64 = false, wave = false, pair = false, quad = false, w1 = false, any_diag = false;
    std::vector<int> idx;       // runs, sorted by steps this call (descending)
    size_t off = 0;             // first table entry
    int nact = 0;
    int64_t s = 0;              // steps of this call done
    int64_t inc_lo = -1;        // first level (call step) of the active runs' laser tables
};

class Engine {
public:
    ~Engine()
    {
        if (host_) hipHostFree(host_);
        if (ws_.side) {
            hipStreamSynchronize(ws_.side);
            hipEventDestroy(ws_.fork);
            hipEventDestroy(ws_.join);
            hipStreamDestroy(ws_.side);
        }
        if (ws_.ring) {
            hipStreamSynchronize(ws_.ring);
            hipEventDestroy(ws_.ring_done);
            hipStreamDestroy(ws_.ring);
        }
    }

    // `dev` holds `cap` table entries of device memory owned by the caller
    int init(BItem *dev, size_t cap)
    {
        dev_ = dev;
        cap_ = cap;
        BCHK(hipHostMalloc((void **)&host_, cap * sizeof(BItem), hipHostMallocDefault));
        BCHK(hipStreamCreateWithFlags(&ws_.side, hipStreamNonBlocking));
        BCHK(hipEventCreateWithFlags(&ws_.fork, hipEventDisableTiming));
        BCHK(hipEventCreateWithFlags(&ws_.join, hipEventDisableTiming));
        BCHK(hipStreamCreateWithFlags(&ws_.ring, hipStreamNonBlocking));
        BCHK(hipEventCreateWithFlags(&ws_.ring_done, hipEventDisableTiming));
        return AXF_OK;
    }

    static size_t entries_for(size_t runs) { return runs + 16; }

    // four-step passes for runs with an interior for them (batches); the
    // server keeps two-step passes: with four, its saturated throughput fell
    // (128 requests/s: 12.2-12.4 against 12.7 Gcell/s) while a 512-run scan
    // gained (37.2 -> 39.6)
    bool quads = true;

    int step(Run *const *runs, const int64_t *ns, int count, hipStream_t st);

private:
    template <int D, typename T>
    int group_step(Group& g, long s, int ns, std::vector<int64_t>& nrec, std::vector<int64_t>& inc_at,
                   Run *const *runs, hipStream_t st);

    BItem *dev_ = nullptr, *host_ = nullptr;
    size_t cap_ = 0;
    // side stream of the 2D frame launches, ring stream of four-step passes
    WaveStreams ws_{nullptr, nullptr, nullptr, nullptr, nullptr};
};

// one step s of the call, or steps s .. s + ns - 1 as a pass of ns = 2 or 4
// steps (the caller takes one only where no diagnostic record falls on any
// of its steps and no laser-table fill on any but the first)
template <int D, typename T>
int Engine::group_step(Group& g, long s, int ns, std::vector<int64_t>& nrec, std::vector<int64_t>& inc_at,
                       Run *const *runs, hipStream_t st)
{
    const bool two = ns > 1;
    const BItem *dt = dev_ + g.off, *ht = host_ + g.off;
    const int n = g.nact;
    // the laser tables hold the levels s .. s + ns of these steps (a fill
    // every 16 steps while the group steps through the unfused kernels)
    if (!(g.inc_lo >= 0 && s >= g.inc_lo && s + ns < g.inc_lo + kIncLevels)) {
        Plain<D, T>::batch_inc_fill(dt, ht, n, s, kIncLevels, st);
        g.inc_lo = s;
        for (int k = 0; k < n; k++) inc_at[g.idx[k]] = s;
    }
    bool launched = false;
    if constexpr (D == 2) {
        if (g.wave) {
            hipError_t e = ns == 4   ? launch_wave2d_quad_batch<T>(dt, ht, n, s, st, &ws_)
                           : ns == 2 ? launch_wave2d_pair_batch<T>(dt, ht, n, s, st, &ws_)
                                     : launch_wave2d_batch<T>(dt, ht, n, s, st, &ws_);
            if (e != hipSuccess) return hip_fail(e, "batched wavefront step");
            launched = true;
        }
    }
    if (!launched) Plain<D, T>::batch_step(dt, ht, n, s, st);
    if (two || !g.any_diag) return AXF_OK;
    // diagnostics of the runs whose cadence hits this step
    int hits = 0;
    bool same = true;
    for (int k = 0; k < n; k++) {
        const Run *R = runs[g.idx[k]];
        const int64_t de = R->cfg.diag_every;
        if (de > 0 && (R->step + s) % de == 0) hits++;
        same = same && nrec[g.idx[k]] == nrec[g.idx[0]];
    }
    if (hits == 0) return AXF_OK;
    if (hits == n && same) {
        Plain<D, T>::batch_diag(dt, ht, n, s, nrec[g.idx[0]], st);
        for (int k = 0; k < n; k++) nrec[g.idx[k]]++;
        return AXF_OK;
    }
    for (int k = 0; k < n; k++) {
        Run *R = runs[g.idx[k]];
        const int64_t de = R->cfg.diag_every;
        if (de <= 0 || (R->step + s) % de != 0) continue;
        const int64_t slot = (R->rec_written + nrec[g.idx[k]]) % R->hk<T>().rec_cap;
        Plain<D, T>::diag(R->rk<T>(), R->hk<T>(), R->step + s, (int)slot, st);
        nrec[g.idx[k]]++;
    }
    return AXF_OK;
}

int Engine::step(Run *const *runs, const int64_t *ns, int count, hipStream_t st)
{
    std::vector<Group> groups;
    int64_t smax = 0;
    for (int i = 0; i < count; i++) {
        if (ns[i] < 0) return fail(AXF_EINVAL, "negative step count for run %d", i);
        if (ns[i] == 0) continue;
        Run *R = runs[i];
        int rc = run_prepare(R);
        if (rc) return rc;
        const int D = R->cfg.ndim;
        const bool f64 = R->cfg.precision == AXF_F64, wave = run_wave2d(R), pair = run_pairs(R);
        const bool quad = quads && run_quads(R);
        const bool w1 = D == 1 && R->use_fused;
        Group *g = nullptr;
        for (auto& q : groups)
            if (q.D == D && q.f64 == f64 && q.wave == wave && q.pair == pair && q.quad == quad && q.w1 == w1) g = &q;
        if (!g) {
            groups.emplace_back();
            g = &groups.back();
            g->D = D;
            g->f64 = f64;
            g->wave = wave;
            g->pair = pair;
            g->quad = quad;
            g->w1 = w1;
        }
        g->idx.push_back(i);
        g->any_diag = g->any_diag || R->cfg.diag_every > 0;
        smax = std::max(smax, ns[i]);
    }
    if (smax == 0) return AXF_OK;
    size_t off = 0;
    for (auto& g : groups) off += g.idx.size() + 1;
    if (off > cap_) return fail(AXF_ENOMEM, "batch table of %zu entries exceeds its %zu", off, cap_);
    off = 0;
    for (auto& g : groups) {
        std::stable_sort(g.idx.begin(), g.idx.end(), [&](int a, int b) { return ns[a] > ns[b]; });
        g.off = off;
        g.nact = (int)g.idx.size();
        long acc[kNumKinds] = {};
        for (size_t k = 0; k <= g.idx.size(); k++) {
            BItem& b = host_[off + k];
            b = BItem{};
            for (int q = 0; q < kNumKinds; q++) b.blk[q] = acc[q];
            if (k == g.idx.size()) break;
            const Run *R = runs[g.idx[k]];
            b.rk = R->base + R->L.off_rk;
            b.step0 = R->step;
            b.rec0 = R->rec_written;
            b.chunk = run_wave_chunk(R);
            run_pass_shape(R, 2, &b.pass_ci, &b.pass_cf);
            run_pass_shape(R, 4, &b.quad_ci, &b.quad_cf);
            long nb[kNumKinds];
            run_blocks(R, g.wave, g.pair, g.quad, g.w1, nb);
            for (int q = 0; q < kNumKinds; q++) acc[q] += nb[q];
        }
        off += g.idx.size() + 1;
    }
    BCHK(hipMemcpyAsync(dev_, host_, off * sizeof(BItem), hipMemcpyHostToDevice, st));
    // the staging buffer is rewritten by the next call: finish the copy now
    BCHK(hipStreamSynchronize(st));

    std::vector<int64_t> nrec(count, 0), inc_at(count, -1);
    // a diagnostic record of some active run of the group falls on step s
    auto diag_at = [&](const Group& g, int64_t s) {
        if (!g.any_diag) return false;
        for (int k = 0; k < g.nact; k++) {
            const Run *R = runs[g.idx[k]];
            if (R->cfg.diag_every > 0 && (R->step + s) % R->cfg.diag_every == 0) return true;
        }
        return false;
    };
    for (bool busy = true; busy;) {
        busy = false;
        for (auto& g : groups) {
            const int64_t s = g.s;
            while (g.nact > 0 && ns[g.idx[g.nact - 1]] <= s) g.nact--;
            if (g.nact == 0) continue;
            busy = true;
            // a pass of k steps when every active run takes all k, no record
            // falls on any of them and no table fill on any but the first
            auto pass_fits = [&](int k) {
                if (ns[g.idx[g.nact - 1]] < s + k) return false;
                for (int q = 0; q < k; q++)
                    if ((q > 0 && (s + q) % (kIncLevels - 1) == 0) || diag_at(g, s + q)) return false;
                return true;
            };
            if (g.w1) {
                // a fused 1D pass over the steps before the next record of any
                // active run (the record's step takes the unfused kernels)
                int64_t free = ns[g.idx[g.nact - 1]] - s;
                for (int k = 0; k < g.nact; k++) {
                    const Run *R = runs[g.idx[k]];
                    const int64_t de = R->cfg.diag_every, at = R->step + s;
                    if (de > 0) free = std::min<int64_t>(free, (at + de - 1) / de * de - at);
                }
                const Run *R0 = runs[g.idx[0]];
                const int kmax = g.f64 ? wave1d_kmax<double>() : wave1d_kmax<float>();
                const int k = free >= 2 ? wave1d_pick(free, kmax, R0->L.nem, R0->L.nph) : 0;
                if (k >= 2) {
                    const BItem *dt = dev_ + g.off, *ht = host_ + g.off;
                    const int win = wave1d_window(true);
                    hipError_t e = g.f64 ? launch_wave1d_batch<double>(dt, ht, g.nact, s, k, win, st)
                                         : launch_wave1d_batch<float>(dt, ht, g.nact, s, k, win, st);
                    if (e != hipSuccess) return hip_fail(e, "batched fused 1D pass");
                    g.s += k;
                    continue;
                }
            }
            const int np = g.D != 2 ? 1 : (g.quad && pass_fits(4)) ? 4 : (g.pair && pass_fits(2)) ? 2 : 1;
            int rc;
            switch (g.D * 2 + (g.f64 ? 1 : 0)) {
            case 2: rc = group_step<1, float>(g, s, 1, nrec, inc_at, runs, st); break;
            case 3: rc = group_step<1, double>(g, s, 1, nrec, inc_at, runs, st); break;
            case 4: rc = group_step<2, float>(g, s, np, nrec, inc_at, runs, st); break;
            case 5: rc = group_step<2, double>(g, s, np, nrec, inc_at, runs, st); break;
            case 6: rc = group_step<3, float>(g, s, 1, nrec, inc_at, runs, st); break;
            default: rc = group_step<3, double>(g, s, 1, nrec, inc_at, runs, st); break;
            }
            if (rc) return rc;
            g.s += np;
        }
    }
    BCHK(hipGetLastError());
    for (int i = 0; i < count; i++) {
        if (ns[i] == 0) continue;
        Run *R = runs[i];
        if (R->cfg.laser_on) R->inc_lo = inc_at[i] >= 0 ? R->step + inc_at[i] : -1;
        R->step += ns[i];
        R->rec_written += nrec[i];
    }
    return AXF_OK;
}

}  // namespace axf

using namespace axf;

// ------------------------------------------------------------------ batches

struct axf_batch {
    std::vector<axf_run *> runs;
    Engine eng;
    hipStream_t stream = nullptr;
};

static int batch_layout(const axf_config *cfgs, int32_t count, std::vector<size_t> *offs, size_t *total)
{
    if (!cfgs || count <= 0) return fail(AXF_EINVAL, "a batch needs at least one configuration");
    size_t off = align256(Engine::entries_for(count) * sizeof(BItem));
    for (int32_t i = 0; i < count; i++) {
        int rc = validate(&cfgs[i]);
        if (rc == AXF_OK && cfgs[i].win_cells != 0) rc = fail(AXF_EINVAL, "batches take fixed windows only");
        if (rc == AXF_OK && (cfgs[i].ppc[0] > 0 || cfgs[i].laser_order != 0))
            rc = fail(AXF_EINVAL, "batches take runs without particles and with a zero-order laser");
        if (rc) return fail(rc, "run %d: %s", i, axf_last_error());
        if (offs) offs->push_back(off);
        off += align256(make_layout(&cfgs[i]).total);
    }
    *total = off;
    return AXF_OK;
}

extern "C" {

int axf_batch_footprint(const axf_config *cfgs, int32_t count, size_t *bytes)
{
    if (!bytes) return fail(AXF_EINVAL, "null output");
    return batch_layout(cfgs, count, nullptr, bytes);
}

int axf_batch_create(const axf_config *cfgs, int32_t count, void *dev_buf, size_t bytes, void *stream,
                     axf_batch **out)
{
    if (!out) return fail(AXF_EINVAL, "null output");
    *out = nullptr;
    std::vector<size_t> offs;
    size_t total = 0;
    int rc = batch_layout(cfgs, count, &offs, &total);
    if (rc) return rc;
    if (!dev_buf) return fail(AXF_EINVAL, "null device buffer");
    if (((uintptr_t)dev_buf & 255) != 0) return fail(AXF_EINVAL, "device buffer must be 256-byte aligned");
    if (bytes < total) return fail(AXF_ENOMEM, "device buffer of %zu bytes < batch footprint %zu", bytes, total);
    axf_batch *B = new (std::nothrow) axf_batch();
    if (!B) return fail(AXF_ENOMEM, "host allocation failed");
    B->stream = (hipStream_t)stream;
    char *base = (char *)dev_buf;
    rc = B->eng.init((BItem *)base, Engine::entries_for(count));
    for (int32_t i = 0; i < count && rc == AXF_OK; i++) {
        axf_run *R = new (std::nothrow) axf_run();
        if (!R) {
            rc = fail(AXF_ENOMEM, "host allocation failed");
            break;
        }
        R->batch_owned = true;
        B->runs.push_back(R);
        rc = run_init(R, &cfgs[i], base + offs[i], make_layout(&cfgs[i]).total, B->stream);
    }
    if (rc) {
        for (auto *R : B->runs) delete R;
        delete B;
        return rc;
    }
    *out = B;
    return AXF_OK;
}

int axf_batch_step(axf_batch *b, const int64_t *nsteps)
{
    if (!b || !nsteps) return fail(AXF_EINVAL, "null argument");
    std::vector<Run *> runs(b->runs.begin(), b->runs.end());
    return b->eng.step(runs.data(), nsteps, (int)runs.size(), b->stream);
}

int axf_batch_run(axf_batch *b, int32_t i, axf_run **view)
{
    if (!b || !view) return fail(AXF_EINVAL, "null argument");
    if (i < 0 || i >= (int32_t)b->runs.size()) return fail(AXF_ENOTFOUND, "run %d not in the batch of %zu", i, b->runs.size());
    *view = b->runs[i];
    return AXF_OK;
}

int axf_batch_destroy(axf_batch *b)
{
    if (!b) return AXF_OK;
    hipStreamSynchronize(b->stream);
    for (auto *R : b->runs) {
        run_release(R);
        delete R;
    }
    delete b;
    return AXF_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ server
//
// A host thread owns the GPU work.  Each round it admits queued requests that
// fit (a free slot and a first-fit range of the pool), initialises them, and
// advances every resident run through the engine by a work slice of about
// macro_steps x 2^20 cell-updates (at least one step), so newly admitted runs
// join the batched launches of the runs already on the device and small runs
// are not held behind large ones.  Runs that reach their step count (or are cancelled) are retired:
// their final diagnostic record becomes the result and their memory returns to
// the pool.  Queued requests are considered in the order of a deadline: the
// arrival time plus the request's work (cells x steps) at kRefRate, so a
// burst is admitted shortest first while a large request overtakes every
// request that arrives more than its own service time after it.  A request
// passed over for more than kStarveRounds rounds for want of memory stops the
// requests after it in that order from overtaking it.

namespace {

constexpr int kStarveRounds = 4;
constexpr double kRefRate = 1e10;   // cell-updates per second of the deadline

struct Request {
    uint64_t id;
    axf_config cfg;
    int64_t nsteps;
    size_t bytes;
    double t_submit;
    int skipped = 0;
    double deadline() const { return t_submit + (double)cfg.n[0] * cfg.n[1] * cfg.n[2] * (double)nsteps / kRefRate; }
};

struct Resident {
    uint64_t id;
    axf_run *R;
    int64_t nsteps, done;
    size_t off, bytes;
    double t_submit, t_admit;
    bool cancel;
};

// first-fit allocator over [0, size) in 256-byte units
class Pool {
public:
    void reset(size_t size) { free_.clear(); free_[0] = size; }
    bool take(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

}  // namespace

struct axf_server {
    char *pool = nullptr;        // run memory (after the engine table)
    size_t pool_bytes = 0;
    int max_slots = 0;
    int64_t macro = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    Engine eng;
    Pool alloc;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> queue;
    std::vector<Resident> res;
    std::deque<axf_result> done;
    std::set<uint64_t> cancels;
    size_t used = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread th;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

    void finish(Resident& r, int status, double t)
    {
        axf_result out{};
        out.id = r.id;
        out.status = status;
        out.steps = r.done;
        out.cells = (int64_t)r.R->cfg.n[0] * r.R->cfg.n[1] * r.R->cfg.n[2];
        out.t_submit = r.t_submit;
        out.t_admit = r.t_admit;
        if (status == AXF_OK) {
            int rc = run_diag_now(r.R, &out.final);
            if (rc) out.status = rc;
        }
        out.t_done = t;
        run_release(r.R);
        delete r.R;
        std::lock_guard<std::mutex> lk(mu);
        alloc.give(r.off, r.bytes);
        used -= r.bytes;
        done.push_back(out);
    }

    // a request that could not be started (no host memory): report and release
    void fail_request(const Request& q, size_t off, int status, double t)
    {
        axf_result out{};
        out.id = q.id;
        out.status = status;
        out.cells = (int64_t)q.cfg.n[0] * q.cfg.n[1] * q.cfg.n[2];
        out.t_submit = q.t_submit;
        out.t_admit = out.t_done = t;
        std::lock_guard<std::mutex> lk(mu);
        alloc.give(off, q.bytes);
        used -= q.bytes;
        done.push_back(out);
    }

    // steps of one round: a work budget of macro x 2^20 cell-updates per run,
    // at least one step, at most what remains (small runs finish in a round,
    // large runs share the GPU in slices)
    int64_t round_steps(const Resident& r) const
    {
        const double cells = (double)r.R->cfg.n[0] * r.R->cfg.n[1] * r.R->cfg.n[2];
        const double budget = (double)macro * 1048576.0;
        const int64_t want = std::max<int64_t>(1, (int64_t)(budget / cells));
        return std::min(want, r.nsteps - r.done);
    }

    void loop()
    {
        hipSetDevice(device);
        for (;;) {
            std::vector<Request> admit;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !queue.empty() || !res.empty(); });
                if (stop) break;
                for (auto& r : res)
                    if (cancels.erase(r.id)) r.cancel = true;
                int slots = max_slots - (int)res.size();
                bool blocked = false;
                // earliest deadline first (ties: arrival order)
                std::stable_sort(queue.begin(), queue.end(),
                                 [](const Request& a, const Request& b) { return a.deadline() < b.deadline(); });
                for (auto it = queue.begin(); it != queue.end() && slots > 0;) {
                    size_t off;
                    if (!blocked && alloc.take(it->bytes, &off)) {
                        used += it->bytes;
                        admit.push_back(*it);
                        pending_off.push_back(off);
                        it = queue.erase(it);
                        slots--;
                    } else {
                        if (++it->skipped > kStarveRounds) blocked = true;
                        ++it;
                    }
                }
            }
            const double ta = now();
            for (size_t k = 0; k < admit.size(); k++) {
                Request& q = admit[k];
                const size_t off = pending_off[k];
                axf_run *R = new (std::nothrow) axf_run();
                if (!R) {
                    fail_request(q, off, AXF_ENOMEM, ta);
                    continue;
                }
                R->batch_owned = true;
                int rc = run_init(R, &q.cfg, pool + off, q.bytes, stream);
                Resident r{q.id, R, q.nsteps, 0, off, q.bytes, q.t_submit, ta, false};
                if (rc) {
                    finish(r, rc, now());
                    continue;
                }
                std::lock_guard<std::mutex> lk(mu);
                res.push_back(r);
            }
            pending_off.clear();
            if (res.empty()) continue;
            std::vector<Run *> runs;
            std::vector<int64_t> ns;
            for (auto& r : res) {
                runs.push_back(r.R);
                ns.push_back(r.cancel ? 0 : round_steps(r));
            }
            int rc = eng.step(runs.data(), ns.data(), (int)runs.size(), stream);
            if (rc == AXF_OK && hipStreamSynchronize(stream) != hipSuccess) rc = AXF_EHIP;
            const double t = now();
            std::vector<Resident> keep;
            for (size_t k = 0; k < res.size(); k++) {
                Resident& r = res[k];
                if (rc == AXF_OK) r.done += ns[k];
                if (rc != AXF_OK) finish(r, rc, t);
                else if (r.cancel) finish(r, 1, t);
                else if (r.done >= r.nsteps) finish(r, AXF_OK, t);
                else keep.push_back(r);
            }
            std::lock_guard<std::mutex> lk(mu);
            res.swap(keep);
        }
        // shut down: resident runs end as cancelled
        for (auto& r : res) finish(r, 1, now());
        res.clear();
    }

    std::vector<size_t> pending_off;
};

extern "C" {

int axf_server_create(void *pool, size_t pool_bytes, int32_t max_slots, int32_t macro_steps, void *stream,
                      axf_server **out)
{
    if (!out) return fail(AXF_EINVAL, "null output");
    *out = nullptr;
    if (!pool) return fail(AXF_EINVAL, "null pool");
    if (((uintptr_t)pool & 255) != 0) return fail(AXF_EINVAL, "pool must be 256-byte aligned");
    if (max_slots <= 0 || macro_steps <= 0) return fail(AXF_EINVAL, "max_slots and macro_steps must be positive");
    const size_t table = align256(Engine::entries_for((size_t)max_slots) * sizeof(BItem));
    if (pool_bytes <= table) return fail(AXF_ENOMEM, "pool of %zu bytes leaves no room for runs", pool_bytes);
    hipPointerAttribute_t attr;
    int device = 0;
    if (hipPointerGetAttributes(&attr, pool) == hipSuccess) device = attr.device;
    else hipGetDevice(&device);
    axf_server *S = new (std::nothrow) axf_server();
    if (!S) return fail(AXF_ENOMEM, "host allocation failed");
    S->pool = (char *)pool + table;
    S->pool_bytes = pool_bytes - table;
    S->max_slots = max_slots;
    S->macro = macro_steps;
    S->stream = (hipStream_t)stream;
    S->device = device;
    S->alloc.reset(S->pool_bytes);
    S->eng.quads = false;
    int rc = S->eng.init((BItem *)pool, Engine::entries_for((size_t)max_slots));
    if (rc) {
        delete S;
        return rc;
    }
    S->th = std::thread([S] { S->loop(); });
    *out = S;
    return AXF_OK;
}

int axf_server_submit(axf_server *s, const axf_config *cfg, int64_t nsteps, uint64_t *id)
{
    if (!s || !cfg || !id) return fail(AXF_EINVAL, "null argument");
    if (nsteps <= 0) return fail(AXF_EINVAL, "nsteps must be positive");
    int rc = validate(cfg);
    if (rc == AXF_OK && cfg->win_cells != 0) rc = fail(AXF_EINVAL, "served requests take fixed windows only");
    if (rc == AXF_OK && (cfg->ppc[0] > 0 || cfg->laser_order != 0))
        rc = fail(AXF_EINVAL, "served requests take runs without particles and with a zero-order laser");
    if (rc) return rc;
    const size_t bytes = align256(make_layout(cfg).total);
    if (bytes > s->pool_bytes) return fail(AXF_ENOMEM, "request of %zu bytes exceeds the pool of %zu", bytes, s->pool_bytes);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(AXF_ESTATE, "server is shutting down");
    Request q{s->next_id++, *cfg, nsteps, bytes, s->now()};
    s->queue.push_back(q);
    *id = q.id;
    s->cv.notify_one();
    return AXF_OK;
}

int axf_server_cancel(axf_server *s, uint64_t id)
{
    if (!s) return fail(AXF_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
        if (it->id != id) continue;
        axf_result out{};
        out.id = id;
        out.status = 1;
        out.cells = (int64_t)it->cfg.n[0] * it->cfg.n[1] * it->cfg.n[2];
        out.t_submit = it->t_submit;
        out.t_admit = out.t_done = s->now();
        s->done.push_back(out);
        s->queue.erase(it);
        return AXF_OK;
    }
    for (auto& r : s->res)
        if (r.id == id) {
            s->cancels.insert(id);
            return AXF_OK;
        }
    return fail(AXF_ENOTFOUND, "request %llu is neither queued nor resident", (unsigned long long)id);
}

int axf_server_poll(axf_server *s, axf_result *out, int32_t max, int32_t *n)
{
    if (!s || !n || (max > 0 && !out)) return fail(AXF_EINVAL, "bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return AXF_OK;
}

int axf_server_stats(axf_server *s, int32_t *queued, int32_t *resident, size_t *bytes_used)
{
    if (!s) return fail(AXF_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = (int32_t)s->queue.size();
    if (resident) *resident = (int32_t)s->res.size();
    if (bytes_used) *bytes_used = s->used;
    return AXF_OK;
}

int axf_server_destroy(axf_server *s)
{
    if (!s) return AXF_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    hipStreamSynchronize(s->stream);
    delete s;
    return AXF_OK;
}

}  // extern "C"
