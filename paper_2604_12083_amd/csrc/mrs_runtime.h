// Host runtime objects behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <cstring>
#include <string>
#include <vector>

#include "mrs.h"
#include "mrs_internal.h"

namespace mrs {

// Device memory cache: blocks in size classes (powers of two and their
// 1.5 multiples, from 256 bytes) kept on free lists when released, so that
// a user that allocates and releases repeatedly (the server: a request's
// state and work lists) calls hipMalloc only while the cache warms up and
// never hipFree (which waits for the whole device) until the cache is
// destroyed.  A block may be released only once no queued device work uses
// it.  Not thread-safe.
struct DevPool {
    std::map<size_t, std::vector<void *>> free;
    size_t held = 0;  // bytes obtained from hipMalloc
    static size_t size_class(size_t n);
    hipError_t get(size_t n, void **p, size_t *cap);
    void put(void *p, size_t cap);
    DevPool() = default;
    DevPool(const DevPool &) = delete;
    DevPool &operator=(const DevPool &) = delete;
    ~DevPool();
};

// Device allocation owned by the runtime, from hipMalloc or, when `pool` is
// set before the first reserve, from that pool.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevPool *pool = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            if (pool) pool->put(p, bytes);
            else (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    // Grow-only: keeps the allocation when it is already large enough.
    hipError_t reserve(size_t n) {
        if (n <= bytes) return hipSuccess;
        release();
        if (pool) return pool->get(n, &p, &bytes);
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) { p = nullptr; return e; }
        bytes = n;
        return hipSuccess;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// How the pair kernel covers one ensemble.
struct PairCfg {
    int mode = PAIR_TILE;  // PAIR_TILE, PAIR_SPLIT or PAIR_QUAD
    int tpl = 1;           // targets per lane (tile mode; 1 in QUAD mode)
    int K = 1;             // source chunks (partial sums per target)
    int chunk = 0;         // sources per chunk
    // tail split: sources [tail_start, N) in chunks of tail_chunk sources,
    // partial slots k_big.. (tail_start = 0: none, every chunk is `chunk`)
    int tail_start = 0, tail_chunk = 0, k_big = 0;
    int sched = SCHED_GRID;  // schedule of the tiled kernel (PairSched)
};

// Work lists of one launch sequence over a set of ensembles.
struct Plan {
    int prec = 0;
    int n_ens = 0;
    std::vector<EnsDesc> h_desc;
    std::vector<PairItem> split, tile1, tile2, quad;
    std::vector<PairItem> tail1, tail2, tailq;  // tail-split items, dispatched after tile1 / tile2 / quad
    std::vector<RodItem> rods;
    std::vector<PointItem> pts;
    std::vector<PointItem> lj;   // 64-point target blocks of the ensembles with LJ repulsion
    std::vector<PointItem> ljb;  // their LJ source blocks, kBlock / 64 per item
    DevBuf d_desc, d_split, d_tile1, d_tile2, d_quad, d_rods, d_pts, d_lj, d_ljb;
    int sched = SCHED_GRID;  // persistent if any ensemble of the plan asks for it
    DevBuf d_queue;          // kQueueWords uint32, zero between launches
    // cached graphs: key = (integrator, dt bits, steps, elastic)
    std::map<std::tuple<int, uint64_t, int, int>, hipGraphExec_t> graphs;
    int64_t pairs_per_eval = 0;
    PairCfg cfg;  // configuration of a single-ensemble plan
    ~Plan();
};

struct ProfRec {
    std::string name;
    hipEvent_t start, stop;
};

}  // namespace mrs

struct mrs_context {
    int device = 0;
    int n_cu = 256;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    // further streams of the pipelined Parareal (created on first use)
    hipStream_t aux_stream[3] = {nullptr, nullptr, nullptr};
    std::string err;
    // scratch of the one-shot evaluation
    mrs::DevBuf eval_rec, eval_part, eval_desc, eval_items, eval_rod;
    mrs::DevBuf eval_io;  // mrs_eval_host's device copies of X, f, n, U, Omega (grow-only)
    // non-finite flag raised by the reduction kernels of every ensemble of the
    // context: one int32 in pinned, device-mapped host memory (flag_host is its
    // host address, flag_dev the address the kernels write)
    int32_t *flag_host = nullptr;
    int32_t *flag_dev = nullptr;
    // end of the last one-shot evaluation (mrs_eval_device / mrs_eval_host),
    // recorded on its stream: the next one waits for it before it reuses the
    // evaluation scratch, whatever stream it is queued on
    hipEvent_t eval_done = nullptr;
    bool eval_pending = false;
    // pinned staging for small uploads, reused after its event completes
    void *stage_host = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_event = nullptr;
    bool stage_pending = false;
    // profiling
    bool prof_on = false;
    std::string prof_sel;  // bracket only kernels whose name contains this (empty = all)
    std::vector<mrs::ProfRec> prof;
    std::vector<hipEvent_t> event_pool;
    // tuning table: (prec, log2 bucket of N) -> config
    std::map<std::pair<int, int>, mrs::PairCfg> tune;
    // measured evaluation times of tuned entries: (tuned ms, automatic ms)
    std::map<std::pair<int, int>, std::pair<double, double>> tune_ms;
    std::string arch;          // device architecture name (tuning tables are per device kind)
    int tune_first_use = 0;    // > 0: tune unseen size classes when a plan is built, with this many runs
    std::string tune_path;     // tuning table file, rewritten after every tuning (empty: none)
    // batch plans
    std::map<std::pair<std::vector<uint64_t>, int>, std::unique_ptr<mrs::Plan>> batch_plans;
    std::vector<mrs_ensemble *> ensembles;
    std::recursive_mutex mu;
};

struct mrs_ensemble {
    mrs_context *ctx = nullptr;
    uint64_t uid = 0;  // unique per process; plan caches key on it, never on addresses
    int32_t n_fil = 0;
    int64_t N = 0;
    std::vector<int32_t> offsets;  // CSR over the filaments in the stored (spatial) order
    // Point k of the stored order is point perm[k] of the caller's order
    // (filaments kept whole; see spatial_order in mrs_runtime.cpp).
    std::vector<int64_t> perm;
    double eps = 0, mu = 0;
    mrs_rod_params rod{};
    bool has_ext = false;
    // swimming (Sec. IV): waveform (A, k, f) and Lennard-Jones (sigma, energy)
    bool has_wave = false, has_lj = false;
    double wave[3] = {0, 0, 0}, lj[2] = {0, 0};
    mrs::DevBuf off, X, D, U, W, Xs, Ds, Ua, Wa, Ks, fext, next, rec, part;
    mrs::DevBuf clock;              // time at the start of the next step (one double)
    int32_t n_ljblk = 0;
    mrs::DevBuf fil, flj, lj_blk, lj_box, lj_mask;  // with LJ: filament per point, forces, source
                                                    // blocks and their boxes, masks
    std::unique_ptr<mrs::Plan> plan[2];  // per precision
    mrs::DevPool *pool = nullptr;        // where its device arrays come from (null: hipMalloc)
    uint64_t loads_gen = 0;              // bumped whenever the external loads change
    // Parareal workers: clones of this ensemble kept between calls (their
    // batch plans and graphs with them), valid while workers_uid == uid and
    // workers_loads == loads_gen; a worker's owner is the ensemble it copies
    std::vector<mrs_ensemble *> workers;
    uint64_t workers_uid = 0, workers_loads = 0;
    mrs_ensemble *owner = nullptr;
};

namespace mrs {

// Error helpers
mrs_status fail(mrs_context *ctx, mrs_status st, const char *fmt, ...);
// Clear the context's non-finite flag before queuing work whose results are
// checked; after that work has finished, numeric_check returns MRS_ENUMERIC
// (and clears the flag) if a reduction kernel raised it.
void numeric_reset(mrs_context *ctx);
mrs_status numeric_check(mrs_context *ctx);
// MRS_ENUMERIC if any of p[0..n) is not finite.
mrs_status check_host_finite(mrs_context *ctx, const double *p, size_t n, const char *what);
// may_tune: a missing size class may be tuned first (tune on first use)
mrs_status ensemble_plan(mrs_ensemble *E, int prec, Plan **out, bool may_tune = true);
// Tune the size class of n in precision prec if tuning on first use is on
// and the class has no entry yet (never while ctx->stream is capturing).
mrs_status tune_if_unseen(mrs_context *ctx, int64_t n, int prec);
void add_items(Plan &P, int e, int64_t N, int n_fil, const PairCfg &c);
// Lennard-Jones blocks of ensemble e of plan P when it has the repulsion on.
void add_lj_items(Plan &P, int e, const mrs_ensemble *E);
hipError_t finalize_plan(Plan &P);
hipError_t run_pairs(mrs_context *ctx, Plan &P, hipStream_t s);
hipEvent_t take_event(mrs_context *ctx);
// Parareal workers of E for n_slices slices (clones made or reused).
mrs_status ensemble_workers(mrs_ensemble *E, int n_workers, std::vector<mrs_ensemble *> &out);
// Device arrays of a new ensemble, from `pool` if given.  With init, the
// offsets, the clock (0) and zero velocities are copied synchronously;
// without, the caller queues them.
mrs_status ensemble_alloc(mrs_context *ctx, int32_t n_fil, const int32_t *offsets, double eps, double mu,
                          const mrs_rod_params *rod, bool has_ext, std::unique_ptr<mrs_ensemble> &E,
                          DevPool *pool = nullptr, bool init = true);
// Removes an ensemble from its context and frees it without waiting for the
// device: no queued work may use it any more.
void ensemble_detach(mrs_ensemble *E);
// Stored order of an ensemble's filaments (spatial); stored point k is
// caller point perm[k].
void spatial_order(int32_t n_fil, const int32_t *off, const double *X, std::vector<int32_t> &soff,
                   std::vector<int64_t> &perm);
// Row-major caller arrays (n x w) to and from the stored SoA layout.
void aos_to_soa(const double *src, double *dst, int64_t n, int w, const std::vector<int64_t> &perm);
void soa_to_aos(const double *src, double *dst, int64_t n, int w, const std::vector<int64_t> &perm);
// Device arrays of every list of a plan come from `pool` (before finalize_plan).
void plan_use_pool(Plan &P, DevPool *pool);
mrs_status ensemble_clone(mrs_ensemble *S, mrs_ensemble **out);
const char *epi_name(int epi);

// Launch `launch()` on stream s; with profiling on, bracket it with events.
template <class F>
inline hipError_t timed(mrs_context *ctx, const char *name, hipStream_t s, F &&launch) {
    if (!ctx->prof_on || (!ctx->prof_sel.empty() && !std::strstr(name, ctx->prof_sel.c_str()))) return launch();
    hipEvent_t a = take_event(ctx), b = take_event(ctx);
    if (a) (void)hipEventRecord(a, s);
    hipError_t e = launch();
    if (b) (void)hipEventRecord(b, s);
    if (a && b) ctx->prof.push_back({name, a, b});
    return e;
}


PairCfg choose_cfg(mrs_context *ctx, int64_t N, int prec);
// The configuration for N points: `tuned` (a tuning-table entry) or, if null,
// the automatic one for a device with n_cu compute units.  Host only.
PairCfg choose_cfg_for(const PairCfg *tuned, int64_t N, int prec, int n_cu);
// Reorders tiled pair blocks so that those with near pairs along a filament
// (source range overlapping the target range) are dispatched first.
void near_blocks_first(std::vector<PairItem> &v);
// Dispatch order of a plan's tiled blocks: near blocks first, the short
// tail-split blocks last (moved from tail1 / tail2 to the end of tile1 / tile2).
void order_items(Plan &P);
// Power-of-two size class of the tuning table.
int size_bucket(int64_t N);
size_t ensemble_bytes(int64_t N, int n_fil, bool has_ext, int K64, int K32);
hipError_t run_stage(mrs_context *ctx, Plan &P, int stage_state, int elastic, int epi, int stage, int scheme,
                     double dt, hipStream_t s);
// Stages and epilogue scheme of a Runge-Kutta integrator.
inline int rk_stages(int integ) { return integ == MRS_RK2 ? 2 : 4; }
inline int rk_scheme(int integ) { return integ == MRS_RK2 ? RK_SCHEME_RK2 : RK_SCHEME_RK4; }
hipError_t upload(mrs_context *ctx, void *dst, const void *src, size_t bytes, hipStream_t s);
// Queue nsteps steps of one ensemble, or of a batch (as mrs_batch_step), on
// stream s without waiting for them.  The caller holds ctx->mu.
mrs_status ensemble_enqueue(mrs_ensemble *E, int integ, double dt, int nsteps, int prec, int elastic,
                            hipStream_t s);
mrs_status batch_enqueue(mrs_context *ctx, int32_t n_ens, mrs_ensemble *const *ens, int integ, double dt,
                         int nsteps, int prec, int elastic, int use_graph, hipStream_t s);
// The context's further stream i in [0, 3) (non-blocking, default
// priority); null if it cannot be created.
hipStream_t aux_stream(mrs_context *ctx, int i);

}  // namespace mrs
