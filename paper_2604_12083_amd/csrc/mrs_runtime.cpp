// Host runtime and C ABI of the MRS filament library.
#include "mrs_runtime.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <tuple>

using namespace mrs;

namespace mrs {

static constexpr double kPi = 3.14159265358979323846264338327950288;

mrs_status fail(mrs_context *ctx, mrs_status st, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

void numeric_reset(mrs_context *ctx) {
    if (ctx->flag_host) *reinterpret_cast<volatile int32_t *>(ctx->flag_host) = 0;
}

mrs_status numeric_check(mrs_context *ctx) {
    if (ctx->flag_host && *reinterpret_cast<volatile int32_t *>(ctx->flag_host) != 0) {
        numeric_reset(ctx);
        return fail(ctx, MRS_ENUMERIC, "a result came out non-finite");
    }
    return MRS_OK;
}

mrs_status check_host_finite(mrs_context *ctx, const double *p, size_t n, const char *what) {
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite(p[i])) return fail(ctx, MRS_ENUMERIC, "non-finite %s at %zu", what, i);
    return MRS_OK;
}

size_t DevPool::size_class(size_t n) {
    size_t c = 256;
    while (c < n) {
        if (c + c / 2 >= n) return c + c / 2;
        c *= 2;
    }
    return c;
}

hipError_t DevPool::get(size_t n, void **p, size_t *cap) {
    const size_t c = size_class(n);
    auto it = free.find(c);
    if (it != free.end() && !it->second.empty()) {
        *p = it->second.back();
        it->second.pop_back();
        *cap = c;
        return hipSuccess;
    }
    hipError_t e = hipMalloc(p, c);
    if (e != hipSuccess) {
        *p = nullptr;
        *cap = 0;
        return e;
    }
    held += c;
    *cap = c;
    return hipSuccess;
}

void DevPool::put(void *p, size_t cap) { free[cap].push_back(p); }

DevPool::~DevPool() {
    for (auto &kv : free)
        for (void *p : kv.second) (void)hipFree(p);
}

void plan_use_pool(Plan &P, DevPool *pool) {
    for (DevBuf *b : {&P.d_desc, &P.d_split, &P.d_tile1, &P.d_tile2, &P.d_quad, &P.d_rods, &P.d_pts, &P.d_lj,
                      &P.d_ljb, &P.d_queue})
        b->pool = pool;
}

Plan::~Plan() {
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
}

int size_bucket(int64_t N) {
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= N) b++;
    return b;
}

PairCfg choose_cfg(mrs_context *ctx, int64_t N, int prec) {
    auto it = ctx->tune.find({prec, size_bucket(std::max<int64_t>(N, 1))});
    return choose_cfg_for(it != ctx->tune.end() ? &it->second : nullptr, N, prec, ctx->n_cu);
}

template <class T>
static hipError_t upload_vec(DevBuf &d, const std::vector<T> &v) {
    if (v.empty()) return hipSuccess;
    hipError_t e = d.reserve(v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}


void add_lj_items(Plan &P, int e, const mrs_ensemble *E) {
    if (!E->has_lj) return;
    for (int64_t p0 = 0; p0 < E->N; p0 += kLjMaskPoints) P.lj.push_back({e, (int)p0});
    for (int b0 = 0; b0 < E->n_ljblk; b0 += kBlock / 64) P.ljb.push_back({e, b0});
}


hipError_t finalize_plan(Plan &P) {
    order_items(P);
    hipError_t e;
    if ((e = P.d_queue.reserve(kQueueWords * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMemset(P.d_queue.p, 0, kQueueWords * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = upload_vec(P.d_desc, P.h_desc)) != hipSuccess) return e;
    if ((e = upload_vec(P.d_split, P.split)) != hipSuccess) return e;
    if ((e = upload_vec(P.d_tile1, P.tile1)) != hipSuccess) return e;
    if ((e = upload_vec(P.d_tile2, P.tile2)) != hipSuccess) return e;
    if ((e = upload_vec(P.d_quad, P.quad)) != hipSuccess) return e;
    if ((e = upload_vec(P.d_rods, P.rods)) != hipSuccess) return e;
    if ((e = upload_vec(P.d_lj, P.lj)) != hipSuccess) return e;
    if ((e = upload_vec(P.d_ljb, P.ljb)) != hipSuccess) return e;
    return upload_vec(P.d_pts, P.pts);
}

static EnsDesc ensemble_desc(mrs_ensemble *E, int prec, const PairCfg &c) {
    EnsDesc d{};
    d.N = (int32_t)E->N;
    d.n_fil = E->n_fil;
    d.K = c.K;
    d.aos_io = 0;
    d.off = E->off.as<int32_t>();
    d.X = E->X.as<double>();
    d.D = E->D.as<double>();
    d.Xs = E->Xs.as<double>();
    d.Ds = E->Ds.as<double>();
    d.U = E->U.as<double>();
    d.W = E->W.as<double>();
    d.Ua = E->Ua.as<double>();
    d.Wa = E->Wa.as<double>();
    d.Ks = E->Ks.as<double>();
    d.fext = E->has_ext ? E->fext.as<double>() : nullptr;
    d.next = E->has_ext ? E->next.as<double>() : nullptr;
    d.Xin_aos = nullptr;
    set_records(d, E->rec.p, E->N, prec == MRS_FP32C);
    d.part = E->part.as<double>();
    d.g_out = d.m_out = nullptr;
    d.eps = E->eps;
    d.inv_eps = 1.0 / E->eps;
    d.mu = E->mu;
    d.cU = 1.0 / (8.0 * kPi * E->mu);
    d.cW = prec == MRS_FP32C ? 1.0 / (8.0 * kPi * E->mu * E->eps) : d.cU;
    for (int i = 0; i < 3; i++) {
        d.a[i] = E->rod.a[i];
        d.b[i] = E->rod.b[i];
        d.om0[i] = E->rod.omega0[i];
    }
    d.ds = E->rod.ds;
    d.dt = 0.0;
    d.elastic = 1;
    d.clock = E->clock.as<double>();
    d.has_wave = E->has_wave ? 1 : 0;
    for (int i = 0; i < 3; i++) d.wave[i] = E->wave[i];
    d.has_lj = E->has_lj ? 1 : 0;
    d.lj_sig = E->lj[0];
    d.lj_e = E->lj[1];
    d.lj_rc = std::pow(2.0, 1.0 / 6.0) * E->lj[0];
    d.fil = E->has_lj ? E->fil.as<int32_t>() : nullptr;
    d.flj = E->has_lj ? E->flj.as<double>() : nullptr;
    d.n_ljblk = E->has_lj ? E->n_ljblk : 0;
    d.lj_blk = E->has_lj ? E->lj_blk.as<int32_t>() : nullptr;
    d.lj_box = E->has_lj ? E->lj_box.as<double>() : nullptr;
    d.lj_mask = E->has_lj ? E->lj_mask.as<uint64_t>() : nullptr;
    d.nonfinite = E->ctx->flag_dev;
    return d;
}

// Plan of one ensemble for one precision (built once, reused).
mrs_status ensemble_plan(mrs_ensemble *E, int prec, Plan **out, bool may_tune) {
    mrs_context *ctx = E->ctx;
    if (!E->plan[prec]) {
        if (may_tune) {
            mrs_status st = tune_if_unseen(ctx, E->N, prec);
            if (st != MRS_OK) return st;
        }
        auto P = std::make_unique<Plan>();
        plan_use_pool(*P, E->pool);
        P->prec = prec;
        P->n_ens = 1;
        PairCfg c = choose_cfg(ctx, E->N, prec);
        size_t need = (size_t)c.K * 6 * (size_t)E->N * sizeof(double);
        if (E->part.reserve(need) != hipSuccess) return fail(ctx, MRS_ENOMEM, "partial buffer (%zu bytes)", need);
        P->cfg = c;
        P->h_desc.push_back(ensemble_desc(E, prec, c));
        add_items(*P, 0, E->N, E->n_fil, c);
        add_lj_items(*P, 0, E);
        hipError_t e = finalize_plan(*P);
        if (e != hipSuccess) return fail(ctx, MRS_EDEVICE, "plan upload: %s", hipGetErrorString(e));
        E->plan[prec] = std::move(P);
    }
    *out = E->plan[prec].get();
    return MRS_OK;
}

// Events of the kernel profiler (timed): they only time the launches
// between them, so they skip the system-scope fence of a default event (a
// cache write-back and invalidation at every record, which would lengthen
// the timed kernel and slow the work after it).
hipEvent_t take_event(mrs_context *ctx) {
    hipEvent_t ev = nullptr;
    if (!ctx->event_pool.empty()) {
        ev = ctx->event_pool.back();
        ctx->event_pool.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) {
        ev = nullptr;
    }
    return ev;
}

static const char *pair_name(int prec, int mode) {
    if (mode == PAIR_SPLIT) return prec == MRS_FP32C ? "pairs_split_f32c" : "pairs_split_f64";
    if (mode == PAIR_QUAD) return "pairs_tile_f32c_quad";
    return prec == MRS_FP32C ? "pairs_tile_f32c" : "pairs_tile_f64";
}

// Pair-kernel launches of one stage: the small-ensemble kernel, then the
// tiled kernel at one and at two targets per lane, each on its own queue
// counters when the plan runs the persistent schedule.
static hipError_t pair_launches(mrs_context *ctx, int prec, int sched, const EnsDesc *dd, const PairItem *split,
                                int n_split, const PairItem *t1, int n_t1, const PairItem *t2, int n_t2,
                                const PairItem *tq, int n_tq, uint32_t *queue, hipStream_t s) {
    hipError_t e = hipSuccess;
    const bool pers = sched == SCHED_PERSISTENT && queue;
    if (n_split)
        e = timed(ctx, pair_name(prec, PAIR_SPLIT), s,
                  [&] { return launch_pairs(prec, PAIR_SPLIT, 1, dd, split, n_split, s); });
    if (e == hipSuccess && n_t1)
        e = timed(ctx, pair_name(prec, PAIR_TILE), s, [&] {
            return launch_pairs(prec, PAIR_TILE, 1, dd, t1, n_t1, s, pers ? queue : nullptr,
                                pers ? pairs_resident_blocks(prec, 1) * ctx->n_cu : 0);
        });
    if (e == hipSuccess && n_t2)
        e = timed(ctx, pair_name(prec, PAIR_TILE), s, [&] {
            return launch_pairs(prec, PAIR_TILE, 2, dd, t2, n_t2, s, pers ? queue + 2 : nullptr,
                                pers ? pairs_resident_blocks(prec, 2) * ctx->n_cu : 0);
        });
    if (e == hipSuccess && n_tq)
        e = timed(ctx, pair_name(prec, PAIR_QUAD), s, [&] {
            return launch_pairs(prec, PAIR_QUAD, 1, dd, tq, n_tq, s, pers ? queue + 4 : nullptr,
                                pers ? pairs_resident_blocks(prec, 1) * ctx->n_cu : 0);
        });
    return e;
}

hipError_t run_pairs(mrs_context *ctx, Plan &P, hipStream_t s) {
    return pair_launches(ctx, P.prec, P.sched, P.d_desc.as<EnsDesc>(), P.d_split.as<PairItem>(), (int)P.split.size(),
                         P.d_tile1.as<PairItem>(), (int)P.tile1.size(), P.d_tile2.as<PairItem>(),
                         (int)P.tile2.size(), P.d_quad.as<PairItem>(), (int)P.quad.size(), P.d_queue.as<uint32_t>(),
                         s);
}

const char *epi_name(int epi) {
    switch (epi) {
        case EPI_EULER: return "reduce_euler";
        case EPI_RK_STAGE: return "reduce_rk_stage";
        case EPI_RK_FINAL: return "reduce_rk_final";
        default: return "reduce_write";
    }
}

hipError_t run_stage(mrs_context *ctx, Plan &P, int stage_state, int elastic, int epi, int stage, int scheme,
                     double dt, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (!P.lj.empty()) {
        e = timed(ctx, "lj_forces", s, [&] {
            return launch_lj(stage_state, P.d_desc.as<EnsDesc>(), P.d_ljb.as<PointItem>(), (int)P.ljb.size(),
                             P.d_lj.as<PointItem>(), (int)P.lj.size(), s);
        });
        if (e != hipSuccess) return e;
    }
    e = timed(ctx, "rod_forces", s, [&] {
        return launch_rod_forces(P.prec, stage_state, elastic, scheme, stage, dt, P.d_desc.as<EnsDesc>(),
                                 P.d_rods.as<RodItem>(), (int)P.rods.size(), s);
    });
    if (e != hipSuccess) return e;
    if ((e = run_pairs(ctx, P, s)) != hipSuccess) return e;
    return timed(ctx, epi_name(epi), s, [&] {
        return launch_reduce(epi, stage, scheme, dt, P.d_desc.as<EnsDesc>(), P.d_pts.as<PointItem>(),
                             (int)P.pts.size(), s);
    });
}

// Queue nsteps steps of plan P on stream s (no synchronisation).
static hipError_t queue_steps(mrs_context *ctx, Plan &P, int integ, double dt, int nsteps, int elastic,
                              hipStream_t s) {
    for (int step = 0; step < nsteps; step++) {
        hipError_t e;
        if (integ == MRS_EULER) {
            if ((e = run_stage(ctx, P, 0, elastic, EPI_EULER, 0, 0, dt, s)) != hipSuccess) return e;
        } else {
            const int nst = rk_stages(integ), scheme = rk_scheme(integ);
            for (int st = 0; st < nst; st++) {
                e = run_stage(ctx, P, st > 0, elastic, st < nst - 1 ? EPI_RK_STAGE : EPI_RK_FINAL, st, scheme, dt, s);
                if (e != hipSuccess) return e;
            }
        }
    }
    return hipSuccess;
}

// Steps through cached HIP graphs of up to kGraphSteps steps each.
static constexpr int kGraphSteps = 50;

static hipError_t graph_steps(mrs_context *ctx, Plan &P, int integ, double dt, int nsteps, int elastic,
                              hipStream_t s) {
    uint64_t dtbits;
    std::memcpy(&dtbits, &dt, sizeof dtbits);
    int left = nsteps;
    while (left > 0) {
        const int n = std::min(left, kGraphSteps);
        auto key = std::make_tuple(integ, dtbits, n, elastic);
        auto it = P.graphs.find(key);
        if (it == P.graphs.end()) {
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            hipError_t eq = queue_steps(ctx, P, integ, dt, n, elastic, s);
            e = hipStreamEndCapture(s, &g);
            if (eq != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return eq;
            }
            if (e != hipSuccess) return e;
            hipGraphExec_t ex = nullptr;
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return e;
            it = P.graphs.emplace(key, ex).first;
        }
        hipError_t e = hipGraphLaunch(it->second, s);
        if (e != hipSuccess) return e;
        left -= n;
    }
    return hipSuccess;
}

hipError_t upload(mrs_context *ctx, void *dst, const void *src, size_t bytes, hipStream_t s) {
    hipError_t e;
    if (ctx->stage_pending) {
        if ((e = hipEventSynchronize(ctx->stage_event)) != hipSuccess) return e;
        ctx->stage_pending = false;
    }
    if (bytes > ctx->stage_bytes) {
        if (ctx->stage_host) (void)hipHostFree(ctx->stage_host);
        ctx->stage_host = nullptr;
        ctx->stage_bytes = 0;
        size_t nb = std::max<size_t>(bytes, 1 << 16);
        if ((e = hipHostMalloc(&ctx->stage_host, nb, hipHostMallocDefault)) != hipSuccess) return e;
        ctx->stage_bytes = nb;
    }
    std::memcpy(ctx->stage_host, src, bytes);
    if ((e = hipMemcpyAsync(dst, ctx->stage_host, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    if ((e = hipEventRecord(ctx->stage_event, s)) != hipSuccess) return e;
    ctx->stage_pending = true;
    return hipSuccess;
}

size_t ensemble_bytes(int64_t N, int n_fil, bool has_ext, int K64, int K32) {
    size_t per = (3 + 9 + 3 + 3 + 3 + 9 + 3 + 3) * sizeof(double);
    if (has_ext) per += 6 * sizeof(double);
    per += (size_t)std::max(K64, K32) * 6 * sizeof(double);
    return per * (size_t)N + rec_buffer_bytes(N) + (size_t)(n_fil + 1) * sizeof(int32_t);
}

}  // namespace mrs

namespace mrs {

// Device arrays of a new ensemble (state, stage state, velocities, records).
mrs_status ensemble_alloc(mrs_context *ctx, int32_t n_fil, const int32_t *offsets, double eps, double mu,
                          const mrs_rod_params *rod, bool has_ext, std::unique_ptr<mrs_ensemble> &E, DevPool *pool,
                          bool init) {
    static std::atomic<uint64_t> next_uid{1};
    const int64_t n = offsets[n_fil];
    E = std::make_unique<mrs_ensemble>();
    E->pool = pool;
    for (DevBuf *b : {&E->off, &E->X, &E->D, &E->U, &E->W, &E->Xs, &E->Ds, &E->Ua, &E->Wa, &E->Ks, &E->fext, &E->next,
                      &E->rec, &E->part, &E->clock, &E->fil, &E->flj, &E->lj_blk, &E->lj_box, &E->lj_mask})
        b->pool = pool;
    E->ctx = ctx;
    E->uid = next_uid.fetch_add(1);
    E->n_fil = n_fil;
    E->N = n;
    E->offsets.assign(offsets, offsets + n_fil + 1);
    E->eps = eps;
    E->mu = mu;
    E->rod = *rod;
    E->has_ext = has_ext;
    const size_t v3 = (size_t)n * 3 * sizeof(double), v9 = 3 * v3;
    bool ok = E->off.reserve((n_fil + 1) * sizeof(int32_t)) == hipSuccess && E->X.reserve(v3) == hipSuccess &&
              E->D.reserve(v9) == hipSuccess && E->U.reserve(v3) == hipSuccess && E->W.reserve(v3) == hipSuccess &&
              E->Xs.reserve(v3) == hipSuccess && E->Ds.reserve(v9) == hipSuccess &&
              E->Ua.reserve(v3) == hipSuccess && E->Wa.reserve(v3) == hipSuccess && E->Ks.reserve(v3) == hipSuccess &&
              E->rec.reserve(rec_buffer_bytes(n)) == hipSuccess && E->clock.reserve(sizeof(double)) == hipSuccess;
    if (ok && has_ext) ok = E->fext.reserve(v3) == hipSuccess && E->next.reserve(v3) == hipSuccess;
    if (!ok) return fail(ctx, MRS_ENOMEM, "ensemble allocation (%lld points)", (long long)n);
    if (!init) return MRS_OK;
    const double t0 = 0.0;
    if (hipMemcpy(E->off.p, offsets, (n_fil + 1) * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(E->clock.p, &t0, sizeof t0, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(E->U.p, 0, v3) != hipSuccess || hipMemset(E->W.p, 0, v3) != hipSuccess)
        return fail(ctx, MRS_EDEVICE, "ensemble initialisation");
    return MRS_OK;
}

// Buffers of the Lennard-Jones repulsion: the filament of every point, the
// force per point, the source blocks (at most kLjBlockPoints consecutive
// points of one filament) with their boxes, and the per-64-point masks.
static mrs_status lj_buffers(mrs_ensemble *E) {
    mrs_context *ctx = E->ctx;
    const int64_t n = E->N, nm = (n + kLjMaskPoints - 1) / kLjMaskPoints;
    std::vector<int32_t> fil((size_t)std::max<int64_t>(n, 1), 0), blk;
    for (int32_t f = 0; f < E->n_fil; f++) {
        for (int32_t k = E->offsets[f]; k < E->offsets[f + 1]; k++) fil[k] = f;
        for (int32_t k = E->offsets[f]; k < E->offsets[f + 1]; k += kLjBlockPoints)
            blk.insert(blk.end(), {k, std::min(k + kLjBlockPoints, E->offsets[f + 1]), f});
    }
    E->n_ljblk = (int32_t)(blk.size() / 3);
    if (E->fil.reserve((size_t)std::max<int64_t>(n, 1) * sizeof(int32_t)) != hipSuccess ||
        E->flj.reserve((size_t)std::max<int64_t>(n, 1) * 3 * sizeof(double)) != hipSuccess ||
        E->lj_blk.reserve(std::max<size_t>(blk.size(), 1) * sizeof(int32_t)) != hipSuccess ||
        E->lj_box.reserve((size_t)std::max<int32_t>(E->n_ljblk, 1) * 6 * sizeof(double)) != hipSuccess ||
        E->lj_mask.reserve((size_t)std::max<int64_t>(nm, 1) * sizeof(uint64_t)) != hipSuccess)
        return fail(ctx, MRS_ENOMEM, "Lennard-Jones buffers");
    if (hipMemcpy(E->fil.p, fil.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(E->lj_blk.p, blk.data(), blk.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
        return fail(ctx, MRS_EDEVICE, "Lennard-Jones index upload");
    return MRS_OK;
}

void ensemble_detach(mrs_ensemble *E) {
    mrs_context *ctx = E->ctx;
    while (!E->workers.empty()) ensemble_detach(E->workers.back());
    if (E->owner) {
        auto &O = E->owner->workers;
        O.erase(std::remove(O.begin(), O.end(), E), O.end());
    }
    for (auto it = ctx->batch_plans.begin(); it != ctx->batch_plans.end();) {
        const auto &v = it->first.first;
        if (std::find(v.begin(), v.end(), E->uid) != v.end()) it = ctx->batch_plans.erase(it);
        else ++it;
    }
    auto &L = ctx->ensembles;
    L.erase(std::remove(L.begin(), L.end(), E), L.end());
    delete E;
}

// New ensemble with the same layout, parameters, loads and state (device copies).
mrs_status ensemble_clone(mrs_ensemble *S, mrs_ensemble **out) {
    mrs_context *ctx = S->ctx;
    std::unique_ptr<mrs_ensemble> E;
    mrs_status st = ensemble_alloc(ctx, S->n_fil, S->offsets.data(), S->eps, S->mu, &S->rod, S->has_ext, E);
    if (st != MRS_OK) return st;
    const size_t v3 = (size_t)S->N * 3 * sizeof(double), v9 = 3 * v3;
    hipStream_t s = ctx->stream;
    E->perm = S->perm;
    E->has_wave = S->has_wave;
    E->has_lj = S->has_lj;
    for (int i = 0; i < 3; i++) E->wave[i] = S->wave[i];
    for (int i = 0; i < 2; i++) E->lj[i] = S->lj[i];
    if (E->has_lj && (st = lj_buffers(E.get())) != MRS_OK) return st;
    if (hipMemcpyAsync(E->X.p, S->X.p, v3, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(E->D.p, S->D.p, v9, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(E->clock.p, S->clock.p, sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        (S->has_ext && (hipMemcpyAsync(E->fext.p, S->fext.p, v3, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                        hipMemcpyAsync(E->next.p, S->next.p, v3, hipMemcpyDeviceToDevice, s) != hipSuccess)) ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(ctx, MRS_EDEVICE, "ensemble clone");
    ctx->ensembles.push_back(E.get());
    *out = E.release();
    return MRS_OK;
}

mrs_status ensemble_workers(mrs_ensemble *E, int n_workers, std::vector<mrs_ensemble *> &out) {
    if (E->workers_uid != E->uid || E->workers_loads != E->loads_gen)
        while (!E->workers.empty()) ensemble_detach(E->workers.back());
    E->workers_uid = E->uid;
    E->workers_loads = E->loads_gen;
    while ((int)E->workers.size() < n_workers) {
        mrs_ensemble *w = nullptr;
        mrs_status st = ensemble_clone(E, &w);
        if (st != MRS_OK) return st;
        w->owner = E;
        E->workers.push_back(w);
    }
    out.assign(E->workers.begin(), E->workers.begin() + n_workers);
    return MRS_OK;
}

}  // namespace mrs

// ------------------------------------------- scratch of the no-alloc entry

namespace mrs {

// Device scratch of mrs_eval_device_noalloc, for callers that cannot
// allocate (code under graph capture, serving loops, harnesses that forbid
// hipMalloc): the evaluation's work list, source records and split-K
// partial sums live in this file-scope array, one copy per device, held
// until the process ends.  Host code never passes the array's name: its
// device address comes from hipGetSymbolAddress once per device, at context
// creation with that device current, and is kept in g_scratch[device].
constexpr size_t kNoallocBytes = size_t(64) << 20;
constexpr size_t kNoallocListBytes = size_t(1) << 20;  // descriptor + work lists
constexpr int64_t kNoallocMaxPoints = 500000;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices];

// Address of this device's scratch (the current device must be `device`).
static hipError_t scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[device] = ptr;
    return hipSuccess;
}

static void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[device];
}

}  // namespace mrs

// ------------------------------------------------------------------ C ABI

#define CHECK_CTX(ctx)                                   \
    do {                                                 \
        if (!(ctx)) return MRS_EINVAL;                   \
    } while (0)

#define HIPCHK(ctx, expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail((ctx), MRS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

static hipStream_t pick_stream(mrs_context *ctx, void *stream) {
    return stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
}

extern "C" {

mrs_status mrs_context_create(int device, mrs_context **out) {
    if (!out) return MRS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return MRS_EDEVICE;
    if (device < 0 || device >= ndev) return MRS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return MRS_EDEVICE;
    auto *ctx = new (std::nothrow) mrs_context();
    if (!ctx) return MRS_ENOMEM;
    ctx->device = device;
    if (scratch_init(device) != hipSuccess) {
        delete ctx;
        return MRS_EDEVICE;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        ctx->n_cu = ncu;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        ctx->arch = prop.gcnArchName;
        const size_t colon = ctx->arch.find(':');  // drop the target features
        if (colon != std::string::npos) ctx->arch.resize(colon);
    }
    if (ctx->arch.empty()) ctx->arch = "unknown";
    void *flag = nullptr;
    if (hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->stage_event, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->eval_done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(&flag, 256, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void **>(&ctx->flag_dev), flag, 0) != hipSuccess) {
        if (flag) (void)hipHostFree(flag);
        if (ctx->eval_done) (void)hipEventDestroy(ctx->eval_done);
        if (ctx->stage_event) (void)hipEventDestroy(ctx->stage_event);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
        delete ctx;
        return MRS_EDEVICE;
    }
    ctx->flag_host = static_cast<int32_t *>(flag);
    *ctx->flag_host = 0;
    ctx->stream = ctx->own_stream;
    *out = ctx;
    return MRS_OK;
}

void mrs_context_destroy(mrs_context *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamSynchronize(ctx->own_stream);
    for (auto a : ctx->aux_stream)
        if (a) (void)hipStreamSynchronize(a);
    // each destruction also removes the ensemble's Parareal workers
    while (!ctx->ensembles.empty()) mrs_ensemble_destroy(ctx->ensembles.back());
    ctx->batch_plans.clear();
    for (auto &r : ctx->prof) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto ev : ctx->event_pool) (void)hipEventDestroy(ev);
    if (ctx->stage_host) (void)hipHostFree(ctx->stage_host);
    if (ctx->stage_event) (void)hipEventDestroy(ctx->stage_event);
    if (ctx->eval_done) (void)hipEventDestroy(ctx->eval_done);
    if (ctx->flag_host) (void)hipHostFree(ctx->flag_host);
    ctx->eval_rec.release();
    ctx->eval_part.release();
    ctx->eval_desc.release();
    ctx->eval_items.release();
    ctx->eval_rod.release();
    for (auto a : ctx->aux_stream)
        if (a) (void)hipStreamDestroy(a);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    delete ctx;
}

const char *mrs_last_error(const mrs_context *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

mrs_status mrs_context_set_stream(mrs_context *ctx, void *stream) {
    CHECK_CTX(ctx);
    ctx->stream = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->own_stream;
    return MRS_OK;
}


mrs_status mrs_context_synchronize(mrs_context *ctx) {
    CHECK_CTX(ctx);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return MRS_OK;
}

}  // extern "C"

namespace mrs {

// Device memory of one one-shot evaluation besides its inputs and outputs:
// source records, split-K partial sums, and the descriptor + work lists.
struct EvalScratch {
    void *rec = nullptr;
    double *part = nullptr;
    char *items = nullptr;
};

// Work lists and descriptor of one evaluation, laid out for one upload:
// [desc][split][tile1][tile2][pts], each part 256-byte aligned.
struct EvalLayout {
    Plan P;
    EnsDesc d{};
    std::vector<char> blob;
    size_t o_desc = 0, o_split = 0, o_t1 = 0, o_t2 = 0, o_tq = 0, o_pts = 0, o_queue = 0;
};

static mrs_status eval_args(mrs_context *ctx, int64_t n, const double *dX, const double *df, const double *dt,
                            double eps, double mu, mrs_precision prec, const double *dU, const double *dW) {
    if (n < 0 || n > INT32_MAX / 8) return fail(ctx, MRS_EINVAL, "n out of range (%lld)", (long long)n);
    if (!finite_pos(eps) || !finite_pos(mu)) return fail(ctx, MRS_EINVAL, "eps and mu must be finite and > 0");
    if (prec != MRS_FP64 && prec != MRS_FP32C) return fail(ctx, MRS_EINVAL, "unknown precision %d", (int)prec);
    if (n > 0 && (!dX || !df || !dt || !dU || !dW)) return fail(ctx, MRS_EINVAL, "null array");
    return MRS_OK;
}

static void eval_layout(EvalLayout &L, int64_t n, const double *dX, const double *df, const double *dt, double eps,
                        double mu, int p, double *dU, double *dW, const PairCfg &c, const EvalScratch &sc) {
    EnsDesc &d = L.d;
    d.N = (int32_t)n;
    d.K = c.K;
    d.aos_io = 1;
    d.Xin_aos = dX;
    d.fext = df;
    d.next = dt;
    d.U = dU;
    d.W = dW;
    // FP32C block descriptors only for the tiled kernels (k_pack_aos writes them)
    set_records(d, sc.rec, n, p == MRS_FP32C && c.mode != PAIR_SPLIT);
    d.part = sc.part;
    d.eps = eps;
    d.inv_eps = 1.0 / eps;
    d.mu = mu;
    d.cU = 1.0 / (8.0 * kPi * mu);
    d.cW = p == MRS_FP32C ? 1.0 / (8.0 * kPi * mu * eps) : d.cU;
    L.P.prec = p;
    add_items(L.P, 0, n, 0, c);
    order_items(L.P);
    auto put = [&](const void *src, size_t bytes) {
        size_t off = (L.blob.size() + 255) & ~size_t(255);
        L.blob.resize(off + bytes);
        if (bytes) std::memcpy(L.blob.data() + off, src, bytes);
        return off;
    };
    L.o_desc = put(&d, sizeof d);
    L.o_split = put(L.P.split.data(), L.P.split.size() * sizeof(PairItem));
    L.o_t1 = put(L.P.tile1.data(), L.P.tile1.size() * sizeof(PairItem));
    L.o_t2 = put(L.P.tile2.data(), L.P.tile2.size() * sizeof(PairItem));
    L.o_tq = put(L.P.quad.data(), L.P.quad.size() * sizeof(PairItem));
    L.o_pts = put(L.P.pts.data(), L.P.pts.size() * sizeof(PointItem));
    const uint32_t zero[kQueueWords] = {};
    L.o_queue = put(zero, sizeof zero);  // work-queue counters start at zero
}

// Queue the kernels of an evaluation whose blob is on the device at `base`.
static hipError_t eval_launch(mrs_context *ctx, const EvalLayout &L, int p, const char *base, hipStream_t s) {
    const Plan &P = L.P;
    const EnsDesc *dd = reinterpret_cast<const EnsDesc *>(base + L.o_desc);
    hipError_t e = timed(ctx, "pack_aos", s, [&] { return launch_pack_aos(p, dd, L.d, s); });
    if (e == hipSuccess)
        e = pair_launches(ctx, p, P.sched, dd, reinterpret_cast<const PairItem *>(base + L.o_split),
                          (int)P.split.size(), reinterpret_cast<const PairItem *>(base + L.o_t1), (int)P.tile1.size(),
                          reinterpret_cast<const PairItem *>(base + L.o_t2), (int)P.tile2.size(),
                          reinterpret_cast<const PairItem *>(base + L.o_tq), (int)P.quad.size(),
                          reinterpret_cast<uint32_t *>(const_cast<char *>(base) + L.o_queue), s);
    if (e == hipSuccess)
        e = timed(ctx, "reduce_write", s, [&] {
            return launch_reduce(EPI_WRITE, 0, 0, 0.0, dd, reinterpret_cast<const PointItem *>(base + L.o_pts),
                                 (int)P.pts.size(), s);
        });
    return e;
}

}  // namespace mrs

extern "C" {

// One-shot evaluation on caller device arrays (AoS n x 3).
mrs_status mrs_eval_device(mrs_context *ctx, int64_t n, const double *dX, const double *df,
                           const double *dt, double eps, double mu, mrs_precision prec, double *dU,
                           double *dW, void *stream) {
    CHECK_CTX(ctx);
    mrs_status st = eval_args(ctx, n, dX, df, dt, eps, mu, prec, dU, dW);
    if (st != MRS_OK || n == 0) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    hipStream_t s = pick_stream(ctx, stream);
    const int p = (int)prec;
    PairCfg c = choose_cfg(ctx, n, p);
    // the scratch below is shared by every evaluation of the context: this
    // one waits on its stream for the previous one (any stream) to finish,
    // and growing a buffer (which frees the old one) first waits on the host
    const size_t rec_bytes = rec_buffer_bytes(n);
    const size_t part_bytes = (size_t)c.K * 6 * (size_t)n * sizeof(double);
    if (ctx->eval_pending) {
        if (rec_bytes > ctx->eval_rec.bytes || part_bytes > ctx->eval_part.bytes)
            HIPCHK(ctx, hipEventSynchronize(ctx->eval_done));
        HIPCHK(ctx, hipStreamWaitEvent(s, ctx->eval_done, 0));
    }
    HIPCHK(ctx, ctx->eval_rec.reserve(rec_bytes));
    HIPCHK(ctx, ctx->eval_part.reserve(part_bytes));
    EvalScratch sc;
    sc.rec = ctx->eval_rec.p;
    sc.part = ctx->eval_part.as<double>();
    EvalLayout L;
    eval_layout(L, n, dX, df, dt, eps, mu, p, dU, dW, c, sc);
    if (ctx->eval_pending && L.blob.size() > ctx->eval_items.bytes) HIPCHK(ctx, hipEventSynchronize(ctx->eval_done));
    HIPCHK(ctx, ctx->eval_items.reserve(L.blob.size()));
    HIPCHK(ctx, upload(ctx, ctx->eval_items.p, L.blob.data(), L.blob.size(), s));
    HIPCHK(ctx, eval_launch(ctx, L, p, ctx->eval_items.as<char>(), s));
    HIPCHK(ctx, hipEventRecord(ctx->eval_done, s));
    ctx->eval_pending = true;
    return MRS_OK;
}

mrs_status mrs_eval_device_noalloc(mrs_context *ctx, int64_t n, const double *dX, const double *df,
                                   const double *dt, double eps, double mu, mrs_precision prec, double *dU,
                                   double *dW, void *stream) {
    CHECK_CTX(ctx);
    mrs_status st = eval_args(ctx, n, dX, df, dt, eps, mu, prec, dU, dW);
    if (st != MRS_OK || n == 0) return st;
    if (n > kNoallocMaxPoints)
        return fail(ctx, MRS_EINVAL, "n = %lld exceeds the %lld points of the allocation-free evaluation's scratch",
                    (long long)n, (long long)kNoallocMaxPoints);
    char *base = static_cast<char *>(scratch_ptr(ctx->device));
    if (!base) return fail(ctx, MRS_EDEVICE, "no scratch address for device %d", ctx->device);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    hipStream_t s = pick_stream(ctx, stream);
    const int p = (int)prec;
    // [descriptor + work lists | source records | partial sums]: the records
    // take the larger size of the two precisions (rec_buffer_bytes); the
    // partials take the rest, and a configuration whose source chunks need
    // more gets fewer, longer chunks
    const size_t rec_off = kNoallocListBytes;
    const size_t part_off = rec_off + ((rec_buffer_bytes(n) + 255) & ~size_t(255));
    const size_t per_chunk = (size_t)n * 6 * sizeof(double);
    const int64_t k_room = (int64_t)((kNoallocBytes - part_off) / per_chunk);
    PairCfg c = choose_cfg(ctx, n, p);
    if (c.K > k_room) {
        PairCfg t;
        t.mode = c.mode;
        t.tpl = c.tpl;
        t.K = (int)k_room;
        c = choose_cfg_for(&t, n, p, ctx->n_cu);
    }
    if (c.K < 1 || c.K > k_room) return fail(ctx, MRS_EINVAL, "partial sums of %lld points exceed the scratch", (long long)n);
    EvalScratch sc;
    sc.rec = base + rec_off;
    sc.part = reinterpret_cast<double *>(base + part_off);
    sc.items = base;
    EvalLayout L;
    eval_layout(L, n, dX, df, dt, eps, mu, p, dU, dW, c, sc);
    if (L.blob.size() > kNoallocListBytes)
        return fail(ctx, MRS_EINVAL, "work list of %lld points exceeds the scratch", (long long)n);
    // calls of this context on different streams run in order (as in
    // mrs_eval_device); calls of other contexts on this device race
    if (ctx->eval_pending) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->eval_done, 0));
    // pageable source: the call returns once the list has been staged
    HIPCHK(ctx, hipMemcpyAsync(base, L.blob.data(), L.blob.size(), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, eval_launch(ctx, L, p, base, s));
    HIPCHK(ctx, hipEventRecord(ctx->eval_done, s));
    ctx->eval_pending = true;
    return MRS_OK;
}

mrs_status mrs_eval_host(mrs_context *ctx, int64_t n, const double *X, const double *f, const double *t,
                         double eps, double mu, mrs_precision prec, double *U, double *W) {
    CHECK_CTX(ctx);
    if (n < 0) return fail(ctx, MRS_EINVAL, "n < 0");
    if (n == 0) return MRS_OK;
    if (!X || !f || !t || !U || !W) return fail(ctx, MRS_EINVAL, "null array");
    for (int64_t i = 0; i < 3 * n; i++)
        if (!std::isfinite(X[i]) || !std::isfinite(f[i]) || !std::isfinite(t[i]))
            return fail(ctx, MRS_EINVAL, "non-finite input at %lld", (long long)i);
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    hipStream_t s = ctx->stream;
    const size_t b = (size_t)n * 3 * sizeof(double);
    // kept by the context: no device allocation (and no freeing, which waits
    // for the device) per call; growing it frees the old one, so first wait
    // for anything still queued that could use it
    DevBuf &io = ctx->eval_io;
    if (io.bytes < 5 * b) HIPCHK(ctx, hipStreamSynchronize(s));
    HIPCHK(ctx, io.reserve(5 * b));
    double *dX = io.as<double>(), *df = dX + 3 * n, *dn = df + 3 * n, *dU = dn + 3 * n, *dW = dU + 3 * n;
    HIPCHK(ctx, hipMemcpyAsync(dX, X, b, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(df, f, b, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(dn, t, b, hipMemcpyHostToDevice, s));
    mrs_status st = mrs_eval_device(ctx, n, dX, df, dn, eps, mu, prec, dU, dW, s);
    if (st != MRS_OK) {
        (void)hipStreamSynchronize(s);
        return st;
    }
    HIPCHK(ctx, hipMemcpyAsync(U, dU, b, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(W, dW, b, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    for (int64_t i = 0; i < 3 * n; i++)
        if (!std::isfinite(U[i]) || !std::isfinite(W[i])) return fail(ctx, MRS_ENUMERIC, "non-finite result");
    return MRS_OK;
}

static bool valid_offsets(int32_t n_fil, const int32_t *off) {
    if (n_fil < 1 || !off || off[0] != 0) return false;
    for (int32_t i = 0; i < n_fil; i++)
        if (off[i + 1] <= off[i]) return false;
    return true;
}

static bool valid_rod(const mrs_rod_params *r) {
    if (!r || !finite_pos(r->ds)) return false;
    for (int i = 0; i < 3; i++)
        if (!std::isfinite(r->a[i]) || !std::isfinite(r->b[i]) || !std::isfinite(r->omega0[i])) return false;
    return true;
}

mrs_status mrs_rod_forces_device(mrs_context *ctx, int32_t n_fil, const int32_t *offsets, const double *dX,
                                 const double *dD, const mrs_rod_params *rod, const double *dfext,
                                 const double *dnext, double *dg, double *dm, void *stream) {
    CHECK_CTX(ctx);
    if (!valid_offsets(n_fil, offsets)) return fail(ctx, MRS_EINVAL, "bad offsets");
    if (!valid_rod(rod)) return fail(ctx, MRS_EINVAL, "bad rod parameters");
    if (!dX || !dD || !dg || !dm) return fail(ctx, MRS_EINVAL, "null array");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    hipStream_t s = pick_stream(ctx, stream);
    const int64_t n = offsets[n_fil];
    // The rod kernel reads SoA state; stage the caller's AoS arrays as SoA
    // through a temporary ensemble-shaped descriptor.
    DevBuf soa, offb;
    HIPCHK(ctx, soa.reserve((size_t)n * (3 + 9 + 6) * sizeof(double) + (size_t)n * sizeof(RecF64)));
    HIPCHK(ctx, offb.reserve((size_t)(n_fil + 1) * sizeof(int32_t)));
    double *Xs = soa.as<double>(), *Ds = Xs + 3 * n, *E6 = Ds + 9 * n;
    void *rec = E6 + 6 * n;
    // transpose on the host side of a device copy would need a kernel; use
    // 2D strided copies instead: component c of AoS -> row c of SoA
    for (int c = 0; c < 3; c++)
        HIPCHK(ctx, hipMemcpy2DAsync(Xs + c * n, sizeof(double), dX + c, 3 * sizeof(double), sizeof(double), n,
                                     hipMemcpyDeviceToDevice, s));
    for (int c = 0; c < 9; c++)
        HIPCHK(ctx, hipMemcpy2DAsync(Ds + c * n, sizeof(double), dD + c, 9 * sizeof(double), sizeof(double), n,
                                     hipMemcpyDeviceToDevice, s));
    const bool ext = dfext || dnext;
    if (ext) {
        HIPCHK(ctx, hipMemsetAsync(E6, 0, 6 * n * sizeof(double), s));
        for (int c = 0; c < 3; c++) {
            if (dfext)
                HIPCHK(ctx, hipMemcpy2DAsync(E6 + c * n, sizeof(double), dfext + c, 3 * sizeof(double),
                                             sizeof(double), n, hipMemcpyDeviceToDevice, s));
            if (dnext)
                HIPCHK(ctx, hipMemcpy2DAsync(E6 + (3 + c) * n, sizeof(double), dnext + c, 3 * sizeof(double),
                                             sizeof(double), n, hipMemcpyDeviceToDevice, s));
        }
    }
    HIPCHK(ctx, hipMemcpyAsync(offb.p, offsets, (size_t)(n_fil + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    EnsDesc d{};
    d.N = (int32_t)n;
    d.n_fil = n_fil;
    d.K = 1;
    d.off = offb.as<int32_t>();
    d.X = Xs;
    d.D = Ds;
    d.fext = ext ? E6 : nullptr;
    d.next = ext ? E6 + 3 * n : nullptr;
    d.rec = rec;
    d.g_out = dg;
    d.m_out = dm;
    d.eps = 1.0;
    d.inv_eps = 1.0;
    d.mu = 1.0;
    for (int i = 0; i < 3; i++) {
        d.a[i] = rod->a[i];
        d.b[i] = rod->b[i];
        d.om0[i] = rod->omega0[i];
    }
    d.ds = rod->ds;
    std::vector<RodItem> items;
    for (int f = 0; f < n_fil; f++) items.push_back({0, f});
    const size_t items_off = (sizeof(EnsDesc) + 255) & ~size_t(255);
    std::vector<char> blob(items_off + items.size() * sizeof(RodItem));
    std::memcpy(blob.data(), &d, sizeof d);
    std::memcpy(blob.data() + items_off, items.data(), items.size() * sizeof(RodItem));
    HIPCHK(ctx, ctx->eval_rod.reserve(blob.size()));
    HIPCHK(ctx, upload(ctx, ctx->eval_rod.p, blob.data(), blob.size(), s));
    HIPCHK(ctx, timed(ctx, "rod_forces", s, [&] {
        return launch_rod_forces(MRS_FP64, 0, 1, 0, 0, 0.0, ctx->eval_rod.as<EnsDesc>(),
                                 reinterpret_cast<const RodItem *>(ctx->eval_rod.as<char>() + items_off), n_fil, s);
    }));
    // temporaries are freed by DevBuf destructors: wait for the kernel first
    HIPCHK(ctx, hipStreamSynchronize(s));
    return MRS_OK;
}

mrs_status mrs_rotsqrt_device(mrs_context *ctx, int64_t count, const double *dR, double *dS, void *stream) {
    CHECK_CTX(ctx);
    if (count < 0) return fail(ctx, MRS_EINVAL, "count < 0");
    if (count == 0) return MRS_OK;
    if (!dR || !dS) return fail(ctx, MRS_EINVAL, "null array");
    hipStream_t s = pick_stream(ctx, stream);
    HIPCHK(ctx, timed(ctx, "rotsqrt", s, [&] { return launch_rotsqrt(count, dR, dS, s); }));
    return MRS_OK;
}

// ---- ensembles

}  // extern "C"

namespace mrs {

// Row-major caller arrays (n x w) to and from the stored SoA layout; stored
// point k is caller point perm[k].
void aos_to_soa(const double *src, double *dst, int64_t n, int w, const std::vector<int64_t> &perm) {
    for (int64_t k = 0; k < n; k++)
        for (int c = 0; c < w; c++) dst[(size_t)c * n + k] = src[(size_t)w * perm[k] + c];
}

void soa_to_aos(const double *src, double *dst, int64_t n, int w, const std::vector<int64_t> &perm) {
    for (int64_t k = 0; k < n; k++)
        for (int c = 0; c < w; c++) dst[(size_t)w * perm[k] + c] = src[(size_t)c * n + k];
}

}  // namespace mrs

extern "C" {

static mrs_status put_soa(mrs_context *ctx, DevBuf &d, const double *src, int64_t n, int w,
                          const std::vector<int64_t> &perm) {
    std::vector<double> tmp((size_t)n * w);
    aos_to_soa(src, tmp.data(), n, w, perm);
    HIPCHK(ctx, hipMemcpy(d.p, tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice));
    return MRS_OK;
}

// 21-bit spread for a 63-bit Morton key.
}  // extern "C"

namespace mrs {

static uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

// Stored order of an ensemble's filaments: by the Morton key of their
// centroids (ties by caller index), whole filaments kept together.  The pair
// kernels cut the points into blocks of consecutive indices; filaments that
// are neighbours in space then share blocks, so a block's box stays small and
// far blocks take the anchored path (filaments shorter than a block, placed
// in random order, otherwise give boxes spanning the domain and every block
// the masked path).  Results are returned in the caller's order; only the
// order of floating-point sums changes.  Writes the stored offsets and the
// point permutation (stored point k = caller point perm[k]).
void spatial_order(int32_t n_fil, const int32_t *off, const double *X, std::vector<int32_t> &soff,
                          std::vector<int64_t> &perm) {
    const int64_t n = off[n_fil];
    std::vector<double> cen((size_t)n_fil * 3, 0.0);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t f = 0; f < n_fil; f++) {
        for (int c = 0; c < 3; c++) {
            double s = 0.0;
            for (int32_t k = off[f]; k < off[f + 1]; k++) s += X[3 * (size_t)k + c];
            cen[3 * (size_t)f + c] = s / (off[f + 1] - off[f]);
            lo[c] = std::min(lo[c], cen[3 * (size_t)f + c]);
            hi[c] = std::max(hi[c], cen[3 * (size_t)f + c]);
        }
    }
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)n_fil);
    for (int32_t f = 0; f < n_fil; f++) {
        uint64_t m = 0;
        for (int c = 0; c < 3; c++) {
            const double span = hi[c] - lo[c];
            const double u = span > 0.0 ? (cen[3 * (size_t)f + c] - lo[c]) / span : 0.0;
            m |= spread3((uint64_t)std::min(2097151.0, std::max(0.0, u * 2097151.0))) << c;
        }
        key[f] = {m, f};
    }
    std::sort(key.begin(), key.end());
    soff.assign((size_t)n_fil + 1, 0);
    perm.resize((size_t)n);
    int64_t pos = 0;
    for (int32_t i = 0; i < n_fil; i++) {
        const int32_t f = key[i].second;
        for (int32_t k = off[f]; k < off[f + 1]; k++) perm[pos++] = k;
        soff[i + 1] = (int32_t)pos;
    }
}

}  // namespace mrs

extern "C" {

static bool all_finite(const double *p, size_t n) {
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite(p[i])) return false;
    return true;
}

mrs_status mrs_ensemble_create(mrs_context *ctx, int32_t n_fil, const int32_t *offsets, const double *X,
                               const double *D, const double *f_ext, const double *n_ext, double eps, double mu,
                               const mrs_rod_params *rod, mrs_ensemble **out) {
    CHECK_CTX(ctx);
    if (!out) return fail(ctx, MRS_EINVAL, "null out");
    *out = nullptr;
    if (!valid_offsets(n_fil, offsets)) return fail(ctx, MRS_EINVAL, "bad offsets");
    if (!finite_pos(eps) || !finite_pos(mu)) return fail(ctx, MRS_EINVAL, "eps and mu must be finite and > 0");
    if (!valid_rod(rod)) return fail(ctx, MRS_EINVAL, "bad rod parameters");
    if (!X || !D) return fail(ctx, MRS_EINVAL, "null state");
    const int64_t n = offsets[n_fil];
    if (n > INT32_MAX / 16) return fail(ctx, MRS_EINVAL, "too many points");
    if (!all_finite(X, 3 * n) || !all_finite(D, 9 * n) || (f_ext && !all_finite(f_ext, 3 * n)) ||
        (n_ext && !all_finite(n_ext, 3 * n)))
        return fail(ctx, MRS_EINVAL, "non-finite input");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    std::vector<int32_t> soff;
    std::vector<int64_t> perm;
    spatial_order(n_fil, offsets, X, soff, perm);
    std::unique_ptr<mrs_ensemble> E;
    mrs_status st = ensemble_alloc(ctx, n_fil, soff.data(), eps, mu, rod, f_ext || n_ext, E);
    if (st != MRS_OK) return st;
    E->perm = std::move(perm);
    if ((st = put_soa(ctx, E->X, X, n, 3, E->perm)) != MRS_OK) return st;
    if ((st = put_soa(ctx, E->D, D, n, 9, E->perm)) != MRS_OK) return st;
    if (E->has_ext) {
        std::vector<double> z((size_t)3 * n, 0.0);
        if ((st = put_soa(ctx, E->fext, f_ext ? f_ext : z.data(), n, 3, E->perm)) != MRS_OK) return st;
        if ((st = put_soa(ctx, E->next, n_ext ? n_ext : z.data(), n, 3, E->perm)) != MRS_OK) return st;
    }
    ctx->ensembles.push_back(E.get());
    *out = E.release();
    return MRS_OK;
}

mrs_status mrs_ensemble_set_state(mrs_ensemble *E, const double *X, const double *D) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    if ((X && !all_finite(X, 3 * E->N)) || (D && !all_finite(D, 9 * E->N)))
        return fail(ctx, MRS_EINVAL, "non-finite state");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    mrs_status st;
    if (X && (st = put_soa(ctx, E->X, X, E->N, 3, E->perm)) != MRS_OK) return st;
    if (D && (st = put_soa(ctx, E->D, D, E->N, 9, E->perm)) != MRS_OK) return st;
    return MRS_OK;
}

mrs_status mrs_ensemble_size(const mrs_ensemble *E, int64_t *n) {
    if (!E || !n) return MRS_EINVAL;
    *n = E->N;
    return MRS_OK;
}

// Drops every cached plan that holds this ensemble's descriptor and gives it
// a new identity, so that the next launch rebuilds them.
static void invalidate_plans(mrs_ensemble *E) {
    static std::atomic<uint64_t> next_gen{1};
    mrs_context *ctx = E->ctx;
    for (auto it = ctx->batch_plans.begin(); it != ctx->batch_plans.end();) {
        const auto &v = it->first.first;
        if (std::find(v.begin(), v.end(), E->uid) != v.end()) it = ctx->batch_plans.erase(it);
        else ++it;
    }
    E->plan[0].reset();
    E->plan[1].reset();
    E->uid = (uint64_t(1) << 63) | next_gen.fetch_add(1);
}

mrs_status mrs_ensemble_set_swimming(mrs_ensemble *E, const double *wave, const double *lj) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    if (wave && !(std::isfinite(wave[0]) && std::isfinite(wave[1]) && std::isfinite(wave[2])))
        return fail(ctx, MRS_EINVAL, "waveform (A, k, f) must be finite");
    if (lj && !(finite_pos(lj[0]) && std::isfinite(lj[1]) && lj[1] >= 0.0))
        return fail(ctx, MRS_EINVAL, "Lennard-Jones sigma must be > 0 and the energy >= 0");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    E->has_wave = wave != nullptr;
    for (int i = 0; i < 3; i++) E->wave[i] = wave ? wave[i] : 0.0;
    E->has_lj = lj != nullptr;
    E->lj[0] = lj ? lj[0] : 0.0;
    E->lj[1] = lj ? lj[1] : 0.0;
    if (E->has_lj) {
        mrs_status st = lj_buffers(E);
        if (st != MRS_OK) return st;
    }
    invalidate_plans(E);
    return MRS_OK;
}

mrs_status mrs_ensemble_set_external(mrs_ensemble *E, const double *f_ext, const double *n_ext) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    const int64_t n = E->N;
    if ((f_ext && !all_finite(f_ext, 3 * n)) || (n_ext && !all_finite(n_ext, 3 * n)))
        return fail(ctx, MRS_EINVAL, "non-finite external load");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (!E->has_ext) {
        if (!f_ext && !n_ext) return MRS_OK;  // the loads stay zero
        const size_t v3 = (size_t)n * 3 * sizeof(double);
        if (E->fext.reserve(v3) != hipSuccess || E->next.reserve(v3) != hipSuccess)
            return fail(ctx, MRS_ENOMEM, "external load buffers (%lld points)", (long long)n);
        E->has_ext = true;
        invalidate_plans(E);  // the descriptors gain the load arrays
    }
    std::vector<double> z(f_ext && n_ext ? 0 : (size_t)3 * n, 0.0);
    mrs_status st;
    E->loads_gen++;
    if ((st = put_soa(ctx, E->fext, f_ext ? f_ext : z.data(), n, 3, E->perm)) != MRS_OK) return st;
    return put_soa(ctx, E->next, n_ext ? n_ext : z.data(), n, 3, E->perm);
}

mrs_status mrs_ensemble_set_time(mrs_ensemble *E, double t) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    if (!std::isfinite(t)) return fail(ctx, MRS_EINVAL, "time must be finite");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(E->clock.p, &t, sizeof t, hipMemcpyHostToDevice));
    return MRS_OK;
}

mrs_status mrs_ensemble_get_time(mrs_ensemble *E, double *t) {
    if (!E || !t) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(t, E->clock.p, sizeof *t, hipMemcpyDeviceToHost));
    return MRS_OK;
}

mrs_status mrs_ensemble_eval(mrs_ensemble *E, mrs_precision prec, int include_elastic) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    if (prec != MRS_FP64 && prec != MRS_FP32C) return fail(ctx, MRS_EINVAL, "unknown precision");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Plan *P;
    mrs_status st = ensemble_plan(E, (int)prec, &P);
    if (st != MRS_OK) return st;
    numeric_reset(ctx);
    HIPCHK(ctx, run_stage(ctx, *P, 0, include_elastic ? 1 : 0, EPI_WRITE, 0, 0, 0.0, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return numeric_check(ctx);
}

static mrs_status check_step_args(mrs_context *ctx, mrs_integrator integ, double dt, int32_t nsteps,
                                  mrs_precision prec) {
    if (integ != MRS_EULER && integ != MRS_RK2 && integ != MRS_RK4)
        return fail(ctx, MRS_EINVAL, "unknown integrator %d", (int)integ);
    if (!std::isfinite(dt)) return fail(ctx, MRS_EINVAL, "dt must be finite");
    if (nsteps < 0) return fail(ctx, MRS_EINVAL, "nsteps < 0");
    if (prec != MRS_FP64 && prec != MRS_FP32C) return fail(ctx, MRS_EINVAL, "unknown precision");
    return MRS_OK;
}

mrs_status mrs_ensemble_step(mrs_ensemble *E, mrs_integrator integ, double dt, int32_t nsteps,
                             mrs_precision prec, int include_elastic) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    mrs_status st = check_step_args(ctx, integ, dt, nsteps, prec);
    if (st != MRS_OK) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Plan *P;
    if ((st = ensemble_plan(E, (int)prec, &P)) != MRS_OK) return st;
    numeric_reset(ctx);
    HIPCHK(ctx, queue_steps(ctx, *P, (int)integ, dt, nsteps, include_elastic ? 1 : 0, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return numeric_check(ctx);
}

mrs_status mrs_ensemble_get(mrs_ensemble *E, double *X, double *D, double *U, double *W) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t n = E->N;
    std::vector<double> tmp((size_t)n * 9);
    struct { double *dst; DevBuf *src; int w; } outs[4] = {{X, &E->X, 3}, {D, &E->D, 9}, {U, &E->U, 3}, {W, &E->W, 3}};
    mrs_status st = MRS_OK;
    for (auto &o : outs) {
        if (!o.dst) continue;
        HIPCHK(ctx, hipMemcpy(tmp.data(), o.src->p, (size_t)n * o.w * sizeof(double), hipMemcpyDeviceToHost));
        soa_to_aos(tmp.data(), o.dst, n, o.w, E->perm);
        if (st == MRS_OK) st = check_host_finite(ctx, tmp.data(), (size_t)n * o.w, "state or velocity");
    }
    return st;
}

void mrs_ensemble_destroy(mrs_ensemble *E) {
    if (!E) return;
    mrs_context *ctx = E->ctx;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    (void)hipStreamSynchronize(ctx->stream);
    ensemble_detach(E);
}

// ---- batching

static mrs_status batch_plan(mrs_context *ctx, int32_t n_ens, mrs_ensemble *const *ens, int prec, Plan **out) {
    std::vector<uint64_t> key;
    for (int32_t i = 0; i < n_ens; i++) key.push_back(ens[i]->uid);
    auto k = std::make_pair(key, prec);
    auto it = ctx->batch_plans.find(k);
    if (it == ctx->batch_plans.end()) {
        auto P = std::make_unique<Plan>();
        P->prec = prec;
        P->n_ens = n_ens;
        for (int e = 0; e < n_ens; e++) {
            mrs_ensemble *E = ens[e];
            // the single-ensemble plan owns the partial buffer size; reuse its config
            Plan *single;
            mrs_status st = ensemble_plan(E, prec, &single);
            if (st != MRS_OK) return st;
            P->h_desc.push_back(single->h_desc[0]);
            add_items(*P, e, E->N, E->n_fil, single->cfg);
            add_lj_items(*P, e, E);
        }
        hipError_t e = finalize_plan(*P);
        if (e != hipSuccess) return fail(ctx, MRS_EDEVICE, "batch plan upload: %s", hipGetErrorString(e));
        it = ctx->batch_plans.emplace(k, std::move(P)).first;
    }
    *out = it->second.get();
    return MRS_OK;
}

static mrs_status check_batch(mrs_context *ctx, int32_t n_ens, mrs_ensemble *const *ens) {
    if (n_ens < 1 || !ens) return fail(ctx, MRS_EINVAL, "empty batch");
    for (int i = 0; i < n_ens; i++) {
        if (!ens[i] || ens[i]->ctx != ctx) return fail(ctx, MRS_EINVAL, "ensemble %d not of this context", i);
        for (int j = 0; j < i; j++)
            if (ens[j] == ens[i]) return fail(ctx, MRS_EINVAL, "ensemble listed twice");
    }
    return MRS_OK;
}

}  // extern "C"

namespace mrs {

mrs_status ensemble_enqueue(mrs_ensemble *E, int integ, double dt, int nsteps, int prec, int elastic,
                            hipStream_t s) {
    mrs_context *ctx = E->ctx;
    Plan *P;
    mrs_status st = ensemble_plan(E, prec, &P);
    if (st != MRS_OK) return st;
    HIPCHK(ctx, queue_steps(ctx, *P, integ, dt, nsteps, elastic, s));
    return MRS_OK;
}

mrs_status batch_enqueue(mrs_context *ctx, int32_t n_ens, mrs_ensemble *const *ens, int integ, double dt,
                         int nsteps, int prec, int elastic, int use_graph, hipStream_t s) {
    Plan *P;
    mrs_status st = batch_plan(ctx, n_ens, ens, prec, &P);
    if (st != MRS_OK) return st;
    if (use_graph && !ctx->prof_on)
        HIPCHK(ctx, graph_steps(ctx, *P, integ, dt, nsteps, elastic, s));
    else
        HIPCHK(ctx, queue_steps(ctx, *P, integ, dt, nsteps, elastic, s));
    return MRS_OK;
}

hipStream_t aux_stream(mrs_context *ctx, int i) {
    hipStream_t &s = ctx->aux_stream[i];
    if (!s && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    return s;
}

}  // namespace mrs

extern "C" {

mrs_status mrs_batch_step(mrs_context *ctx, int32_t n_ens, mrs_ensemble *const *ens, mrs_integrator integ,
                          double dt, int32_t nsteps, mrs_precision prec, int include_elastic, int use_graph) {
    CHECK_CTX(ctx);
    mrs_status st = check_batch(ctx, n_ens, ens);
    if (st != MRS_OK) return st;
    if ((st = check_step_args(ctx, integ, dt, nsteps, prec)) != MRS_OK) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    numeric_reset(ctx);
    st = batch_enqueue(ctx, n_ens, ens, (int)integ, dt, nsteps, (int)prec, include_elastic ? 1 : 0, use_graph,
                       ctx->stream);
    if (st != MRS_OK) return st;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return numeric_check(ctx);
}

mrs_status mrs_batch_eval(mrs_context *ctx, int32_t n_ens, mrs_ensemble *const *ens, mrs_precision prec,
                          int include_elastic) {
    CHECK_CTX(ctx);
    mrs_status st = check_batch(ctx, n_ens, ens);
    if (st != MRS_OK) return st;
    if (prec != MRS_FP64 && prec != MRS_FP32C) return fail(ctx, MRS_EINVAL, "unknown precision");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Plan *P;
    if ((st = batch_plan(ctx, n_ens, ens, (int)prec, &P)) != MRS_OK) return st;
    numeric_reset(ctx);
    HIPCHK(ctx, run_stage(ctx, *P, 0, include_elastic ? 1 : 0, EPI_WRITE, 0, 0, 0.0, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return numeric_check(ctx);
}

// ---- profiling

mrs_status mrs_profile_enable(mrs_context *ctx, int on) {
    CHECK_CTX(ctx);
    ctx->prof_on = on != 0;
    return MRS_OK;
}

mrs_status mrs_profile_select(mrs_context *ctx, const char *kernel) {
    CHECK_CTX(ctx);
    ctx->prof_sel = kernel ? kernel : "";
    return MRS_OK;
}

mrs_status mrs_profile_reset(mrs_context *ctx) {
    CHECK_CTX(ctx);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &r : ctx->prof) {
        ctx->event_pool.push_back(r.start);
        ctx->event_pool.push_back(r.stop);
    }
    ctx->prof.clear();
    return MRS_OK;
}

mrs_status mrs_profile_clock(mrs_context *ctx, double *mhz) {
    CHECK_CTX(ctx);
    if (!mhz) return fail(ctx, MRS_EINVAL, "null output");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    hipStream_t s = ctx->stream;
    uint64_t *buf = nullptr;
    HIPCHK(ctx, hipHostMalloc(reinterpret_cast<void **>(&buf), 2 * sizeof(uint64_t), hipHostMallocMapped));
    uint64_t *dbuf = nullptr;
    hipError_t e = hipHostGetDevicePointer(reinterpret_cast<void **>(&dbuf), buf, 0);
    if (e == hipSuccess) e = launch_clock_probe(200000, dbuf, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const uint64_t tick = buf[0], ref = buf[1];
    (void)hipHostFree(buf);
    if (e != hipSuccess) return fail(ctx, MRS_EDEVICE, "clock probe: %s", hipGetErrorString(e));
    *mhz = ref > 0 ? 100.0 * (double)tick / (double)ref : 0.0;  // reference clock: 100 MHz
    return MRS_OK;
}

mrs_status mrs_profile_query(mrs_context *ctx, const char *kernel, int64_t *launches, double *total_ms) {
    CHECK_CTX(ctx);
    if (!launches || !total_ms) return fail(ctx, MRS_EINVAL, "null output");
    int64_t n = 0;
    double ms = 0.0;
    for (auto &r : ctx->prof) {
        if (kernel && *kernel && r.name.find(kernel) == std::string::npos) continue;
        HIPCHK(ctx, hipEventSynchronize(r.stop));
        float t = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&t, r.start, r.stop));
        ms += t;
        n++;
    }
    *launches = n;
    *total_ms = ms;
    return MRS_OK;
}

}  // extern "C"
