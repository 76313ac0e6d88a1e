// Serving loop of the MRS filament library: continuous batching of
// independent ensemble requests on one device.
//
// A scheduler thread owns the context and keeps the device busy with a
// pipeline of ticks:
//   1. admission: queued requests are taken in arrival order (first fit)
//      while a slot is free and the request's device footprint fits the HBM
//      budget; its state is staged in pinned memory (filaments in spatial
//      order, SoA) and copied to the device on an upload stream, into arrays
//      from the server's device-memory cache, while earlier ticks run;
//   2. tick: ONE batched launch sequence on the compute stream advances the
//      selected requests by one unit of work (an evaluation, one Euler step
//      or one RK step, whose first stage is shared with the evaluation and
//      Euler requests); it first waits (event) for the uploads of requests
//      it runs for the first time.  Up to kTicksInFlight ticks are queued
//      ahead, so the device does not wait for the host between ticks;
//   3. retirement: after a request's last tick its state and velocities are
//      copied to pinned memory on the compute stream; when that tick's event
//      has fired, the results are reordered for the caller and the request's
//      device arrays go back to the cache.
// Requests arriving while ticks run join at a later tick, so work of requests
// of different sizes and kinds overlaps inside the same kernels.  The server
// calls hipMalloc only while its caches warm up and never hipFree before
// mrs_server_stop.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "mrs_runtime.h"

using namespace mrs;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Ticks queued on the device ahead of the host.
constexpr int kTicksInFlight = 2;

// Pinned host memory cache (same size classes as DevPool); not thread-safe.
struct PinPool {
    std::map<size_t, std::vector<void *>> free;
    hipError_t get(size_t n, void **p, size_t *cap) {
        const size_t c = DevPool::size_class(n);
        auto it = free.find(c);
        if (it != free.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            *cap = c;
            return hipSuccess;
        }
        *cap = c;
        return hipHostMalloc(p, c, hipHostMallocDefault);
    }
    void put(void *p, size_t cap) {
        if (p) free[cap].push_back(p);
    }
    ~PinPool() {
        for (auto &kv : free)
            for (void *p : kv.second) (void)hipHostFree(p);
    }
};

struct PinBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct Request {
    uint64_t ticket = 0;
    mrs_request spec{};
    std::vector<int32_t> off;
    std::vector<double> X, D, f, n;
    mrs_ensemble *ens = nullptr;
    int64_t N = 0;
    int32_t steps_done = 0;  // units of work queued (steps, or 1 for an evaluation)
    int64_t footprint = -1;
    mrs_result_info info{};
    bool done = false;
    bool launched_all = false;  // every unit queued; waiting for retirement
    double credit = 0.0;  // pair budget earned and not yet spent (deficit round robin)
    int64_t cost = 0;     // pair interactions of one unit of work (eval or step)
    hipEvent_t up_event = nullptr;  // upload finished (the first tick waits for it)
    bool up_wait = false;           // the next tick that runs it must wait for up_event
    PinBuf pin_in, pin_out;         // pinned staging of the upload and of the results
    std::vector<double> Xo, Do, Uo, Wo;
};

// Work lists of one tick over a set of requests.
struct TickPlan {
    std::vector<uint64_t> key;  // ensemble uids of the set, in order
    Plan all;       // stage 0 over every request of the set
    Plan rk[2];     // later stages of the RK4 (scheme 0) and RK2 (scheme 1) step requests
    std::vector<PointItem> pts_write, pts_euler, pts_rk0[2];
    DevBuf d_pts_write, d_pts_euler, d_pts_rk0[2];
    bool has_rk[2] = {false, false};
    int64_t last_tick = -1;  // the last tick that used it (it may be freed once that tick is done)
};

// A tick queued on the device.
struct Tick {
    int64_t index = 0;
    hipEvent_t start = nullptr, done = nullptr;
    std::vector<Request *> finishing;  // requests whose last unit ran in it (results copied after it)
    int64_t pairs = 0;
};

}  // namespace

struct mrs_server {
    mrs_context *ctx = nullptr;
    int prec = 0;
    int64_t budget = 0;
    int32_t max_slots = 1;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::vector<Request *> active;  // admitted and not retired
    std::map<uint64_t, Request *> table;
    int64_t in_use = 0;
    uint64_t next_ticket = 1;
    bool stopping = false;
    mrs_server_stats st{};
    double t_start = 0.0;
    int64_t fail_tick = -1;
    std::atomic<int64_t> tick_pairs{0};  // 0 = no per-tick bound
    std::atomic<int32_t> admit_order{MRS_ADMIT_ARRIVAL};
    std::atomic<double> admit_max_wait{0.0};  // least-work order: age after which arrival order applies
    // scheduler-thread state
    hipStream_t up_stream = nullptr;
    DevPool pool;
    PinPool pins;
    std::vector<hipEvent_t> events;  // idle events
    std::deque<Tick> in_flight;
    int64_t ticks_launched = 0, ticks_completed = 0;
    // tick plans of recently used request sets (small LRU); declared after
    // the pool, so that they return their arrays to it before it is freed
    std::vector<std::unique_ptr<TickPlan>> plans;
};

namespace {

hipEvent_t take_event(mrs_server *S) {
    if (!S->events.empty()) {
        hipEvent_t e = S->events.back();
        S->events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void give_event(mrs_server *S, hipEvent_t e) {
    if (e) S->events.push_back(e);
}

int64_t request_footprint(mrs_context *ctx, int prec, const Request &r) {
    PairCfg c = choose_cfg(ctx, r.N, prec);
    const bool ext = r.spec.f_ext || r.spec.n_ext;
    return (int64_t)ensemble_bytes(r.N, r.spec.n_fil, ext, c.K, c.K);
}

template <class T>
hipError_t upload_list(DevBuf &d, const std::vector<T> &v) {
    if (v.empty()) return hipSuccess;
    hipError_t e = d.reserve(v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

constexpr size_t kPlanCache = 16;

// Tick plan of the requests `run` (cached per set; the cache is small LRU and
// never frees a plan that a tick still queued on the device may use).
mrs_status tick_plan(mrs_server *S, const std::vector<Request *> &run, TickPlan **out) {
    std::vector<uint64_t> key;
    for (auto *r : run) key.push_back(r->ens->uid);
    for (size_t i = 0; i < S->plans.size(); i++)
        if (S->plans[i]->key == key) {
            std::rotate(S->plans.begin(), S->plans.begin() + i, S->plans.begin() + i + 1);
            *out = S->plans.front().get();
            return MRS_OK;
        }
    auto T = std::make_unique<TickPlan>();
    plan_use_pool(T->all, &S->pool);
    plan_use_pool(T->rk[0], &S->pool);
    plan_use_pool(T->rk[1], &S->pool);
    for (DevBuf *b : {&T->d_pts_write, &T->d_pts_euler, &T->d_pts_rk0[0], &T->d_pts_rk0[1]}) b->pool = &S->pool;
    T->key = key;
    T->all.prec = T->rk[0].prec = T->rk[1].prec = S->prec;
    for (size_t e = 0; e < run.size(); e++) {
        Request *r = run[e];
        Plan *single;
        mrs_status st = ensemble_plan(r->ens, S->prec, &single, /*may_tune=*/false);
        if (st != MRS_OK) return st;
        EnsDesc d = single->h_desc[0];
        d.dt = r->spec.dt;
        d.elastic = r->spec.include_elastic ? 1 : 0;
        T->all.h_desc.push_back(d);
        T->rk[0].h_desc.push_back(d);
        T->rk[1].h_desc.push_back(d);
        add_items(T->all, (int)e, r->N, r->spec.n_fil, single->cfg);
        const bool rk = r->spec.kind == MRS_REQ_STEPS && r->spec.integ != MRS_EULER;
        const int sch = rk ? rk_scheme(r->spec.integ) : 0;
        if (rk) {
            add_items(T->rk[sch], (int)e, r->N, r->spec.n_fil, single->cfg);
            T->has_rk[sch] = true;
        }
        std::vector<PointItem> *dst = r->spec.kind == MRS_REQ_EVAL ? &T->pts_write
                                      : rk                           ? &T->pts_rk0[sch]
                                                                     : &T->pts_euler;
        for (int64_t p0 = 0; p0 < r->N; p0 += kReducePoints) dst->push_back({(int)e, (int)p0});
    }
    hipError_t he = finalize_plan(T->all);
    for (int k = 0; k < 2; k++)
        if (he == hipSuccess && T->has_rk[k]) he = finalize_plan(T->rk[k]);
    if (he == hipSuccess) he = upload_list(T->d_pts_write, T->pts_write);
    if (he == hipSuccess) he = upload_list(T->d_pts_euler, T->pts_euler);
    for (int k = 0; k < 2; k++)
        if (he == hipSuccess) he = upload_list(T->d_pts_rk0[k], T->pts_rk0[k]);
    if (he != hipSuccess) return fail(S->ctx, MRS_EDEVICE, "tick plan upload: %s", hipGetErrorString(he));
    S->plans.insert(S->plans.begin(), std::move(T));
    // evict the least recently used plans beyond the cache size whose last tick is done
    for (size_t i = S->plans.size(); i-- > kPlanCache;)
        if (S->plans[i]->last_tick < S->ticks_completed) S->plans.erase(S->plans.begin() + i);
    *out = S->plans.front().get();
    return MRS_OK;
}

// Forget cached plans that mention a retired request's ensemble (their last
// tick is done: the request's own last tick came after every tick using it).
void drop_plans(mrs_server *S, uint64_t uid) {
    for (auto it = S->plans.begin(); it != S->plans.end();) {
        const auto &k = (*it)->key;
        if (std::find(k.begin(), k.end(), uid) != k.end()) it = S->plans.erase(it);
        else ++it;
    }
}

int evals_per_unit(const Request *r) {
    return (r->spec.kind == MRS_REQ_STEPS && r->spec.integ != MRS_EULER) ? rk_stages(r->spec.integ) : 1;
}

int32_t units(const Request *r) { return r->spec.kind == MRS_REQ_EVAL ? 1 : r->spec.nsteps; }

// Requests that advance in the next tick: every launchable one without a tick
// bound; with one, deficit round robin over them.
std::vector<Request *> pick_tick(mrs_server *S, const std::vector<Request *> &cand) {
    const int64_t budget = S->tick_pairs.load();
    if (budget <= 0) return cand;
    std::vector<Request *> run;
    const double quantum = (double)budget / (double)cand.size();
    Request *best = nullptr;
    for (auto *r : cand) {
        r->credit += quantum;
        if (r->credit >= (double)r->cost) run.push_back(r);
        if (!best || r->credit / (double)r->cost > best->credit / (double)best->cost) best = r;
    }
    if (run.empty()) run.push_back(best);  // always make progress
    for (auto *r : run) r->credit = std::max(0.0, r->credit - (double)r->cost);
    return run;
}

hipError_t launch_tick(mrs_server *S, TickPlan &T) {
    mrs_context *ctx = S->ctx;
    hipStream_t s = ctx->stream;
    const double nan = std::nan("");
    hipError_t e = timed(ctx, "rod_forces", s, [&] {
        return launch_rod_forces(S->prec, 0, -1, 0, 0, nan, T.all.d_desc.as<EnsDesc>(), T.all.d_rods.as<RodItem>(),
                                 (int)T.all.rods.size(), s);
    });
    if (e == hipSuccess) e = run_pairs(ctx, T.all, s);
    const EnsDesc *dd = T.all.d_desc.as<EnsDesc>();
    if (e == hipSuccess && !T.pts_write.empty())
        e = timed(ctx, epi_name(EPI_WRITE), s, [&] {
            return launch_reduce(EPI_WRITE, 0, 0, nan, dd, T.d_pts_write.as<PointItem>(), (int)T.pts_write.size(), s);
        });
    if (e == hipSuccess && !T.pts_euler.empty())
        e = timed(ctx, epi_name(EPI_EULER), s, [&] {
            return launch_reduce(EPI_EULER, 0, 0, nan, dd, T.d_pts_euler.as<PointItem>(), (int)T.pts_euler.size(), s);
        });
    for (int k = 0; k < 2; k++)
        if (e == hipSuccess && !T.pts_rk0[k].empty())
            e = timed(ctx, epi_name(EPI_RK_STAGE), s, [&] {
                return launch_reduce(EPI_RK_STAGE, 0, k, nan, dd, T.d_pts_rk0[k].as<PointItem>(),
                                     (int)T.pts_rk0[k].size(), s);
            });
    for (int k = 0; k < 2; k++) {
        const int nst = k == RK_SCHEME_RK2 ? 2 : 4;
        for (int st = 1; e == hipSuccess && T.has_rk[k] && st < nst; st++)
            e = run_stage(ctx, T.rk[k], 1, -1, st < nst - 1 ? EPI_RK_STAGE : EPI_RK_FINAL, st, k, nan, s);
    }
    return e;
}

// Pair interactions of a request's whole work.
double total_work(const Request *r) {
    return (double)evals_per_unit(r) * (double)r->N * (double)r->N * (double)units(r);
}

// Pick queued requests to admit, first fit, in the server's admission
// order: arrival order, or least total work first with the requests that
// have waited longer than the age bound taken first, in arrival order.
// Caller holds S->mu.
std::vector<Request *> select_admissions(mrs_server *S) {
    std::vector<Request *> order(S->queue.begin(), S->queue.end());
    if (S->admit_order.load() == MRS_ADMIT_LEAST_WORK) {
        const double max_wait = S->admit_max_wait.load(), now = now_s();
        auto aged = [&](const Request *r) { return max_wait > 0.0 && now - r->info.t_submit > max_wait; };
        std::stable_sort(order.begin(), order.end(), [&](const Request *a, const Request *b) {
            const bool ag = aged(a), bg = aged(b);
            if (ag != bg) return ag;
            if (ag) return false;  // both aged: arrival order (stable)
            return total_work(a) < total_work(b);
        });
    }
    std::vector<Request *> pick;
    std::vector<Request *> drop;  // leave the queue: admitted or rejected
    int64_t used = S->in_use;
    for (Request *r : order) {
        if ((int32_t)(S->active.size() + pick.size()) >= S->max_slots) break;
        if (r->footprint < 0) r->footprint = request_footprint(S->ctx, S->prec, *r);
        if (r->footprint > S->budget) {  // can never fit
            r->info.status = MRS_ENOMEM;
            r->info.t_admit = r->info.t_done = now_s();
            r->done = true;
            S->st.rejected++;
            drop.push_back(r);
            S->cv_done.notify_all();
            continue;
        }
        if (used + r->footprint > S->budget) continue;
        used += r->footprint;
        pick.push_back(r);
        drop.push_back(r);
    }
    if (!drop.empty()) {
        std::sort(drop.begin(), drop.end());
        S->queue.erase(std::remove_if(S->queue.begin(), S->queue.end(),
                                      [&](Request *r) { return std::binary_search(drop.begin(), drop.end(), r); }),
                       S->queue.end());
    }
    S->in_use = used;
    return pick;
}

// Device state of an admitted request: arrays from the cache, the inputs
// staged in pinned memory (spatial order, SoA) and copied on the upload
// stream; r->up_event fires when they are on the device.
mrs_status admit(mrs_server *S, Request *r) {
    mrs_context *ctx = S->ctx;
    const mrs_request &q = r->spec;
    const int64_t n = r->N;
    const bool ext = !r->f.empty();
    std::vector<int32_t> soff;
    std::vector<int64_t> perm;
    spatial_order(q.n_fil, r->off.data(), r->X.data(), soff, perm);
    std::unique_ptr<mrs_ensemble> E;
    mrs_status st = ensemble_alloc(ctx, q.n_fil, soff.data(), q.eps, q.mu, &q.rod, ext, E, &S->pool, false);
    if (st != MRS_OK) return st;
    E->perm = std::move(perm);
    // staging: X (3n), D (9n), [fext (3n), next (3n)], clock, offsets
    const size_t nd = (size_t)n * (12 + (ext ? 6 : 0)) + 1;
    const size_t bytes = nd * sizeof(double) + (size_t)(q.n_fil + 1) * sizeof(int32_t);
    if (S->pins.get(bytes, &r->pin_in.p, &r->pin_in.cap) != hipSuccess) {
        r->pin_in = PinBuf{};
        return fail(ctx, MRS_ENOMEM, "pinned staging (%zu bytes)", bytes);
    }
    double *h = static_cast<double *>(r->pin_in.p);
    aos_to_soa(r->X.data(), h, n, 3, E->perm);
    aos_to_soa(r->D.data(), h + 3 * n, n, 9, E->perm);
    if (ext) {
        aos_to_soa(r->f.data(), h + 12 * n, n, 3, E->perm);
        aos_to_soa(r->n.data(), h + 15 * n, n, 3, E->perm);
    }
    h[nd - 1] = 0.0;  // clock
    std::memcpy(h + nd, soff.data(), (size_t)(q.n_fil + 1) * sizeof(int32_t));
    hipStream_t u = S->up_stream;
    const size_t v3 = (size_t)n * 3 * sizeof(double);
    hipError_t he = hipMemcpyAsync(E->X.p, h, v3, hipMemcpyHostToDevice, u);
    if (he == hipSuccess) he = hipMemcpyAsync(E->D.p, h + 3 * n, 3 * v3, hipMemcpyHostToDevice, u);
    if (he == hipSuccess && ext) he = hipMemcpyAsync(E->fext.p, h + 12 * n, v3, hipMemcpyHostToDevice, u);
    if (he == hipSuccess && ext) he = hipMemcpyAsync(E->next.p, h + 15 * n, v3, hipMemcpyHostToDevice, u);
    if (he == hipSuccess) he = hipMemcpyAsync(E->clock.p, h + nd - 1, sizeof(double), hipMemcpyHostToDevice, u);
    if (he == hipSuccess)
        he = hipMemcpyAsync(E->off.p, h + nd, (size_t)(q.n_fil + 1) * sizeof(int32_t), hipMemcpyHostToDevice, u);
    if (he == hipSuccess) he = hipMemsetAsync(E->U.p, 0, v3, u);
    if (he == hipSuccess) he = hipMemsetAsync(E->W.p, 0, v3, u);
    if (he == hipSuccess && !(r->up_event = take_event(S))) he = hipErrorOutOfMemory;
    if (he == hipSuccess) he = hipEventRecord(r->up_event, u);
    ctx->ensembles.push_back(E.get());
    r->ens = E.release();
    if (he != hipSuccess) return fail(ctx, MRS_EDEVICE, "request upload: %s", hipGetErrorString(he));
    r->up_wait = true;
    std::vector<double>().swap(r->X);  // inputs now live on the device
    std::vector<double>().swap(r->D);
    std::vector<double>().swap(r->f);
    std::vector<double>().swap(r->n);
    return MRS_OK;
}

// Queue the copy of a finishing request's state and velocities to pinned
// memory after the tick's kernels (compute stream).
hipError_t queue_results(mrs_server *S, Request *r) {
    mrs_ensemble *E = r->ens;
    const size_t v3 = (size_t)r->N * 3 * sizeof(double);
    if (S->pins.get(6 * v3, &r->pin_out.p, &r->pin_out.cap) != hipSuccess) {
        r->pin_out = PinBuf{};
        return hipErrorOutOfMemory;
    }
    char *h = static_cast<char *>(r->pin_out.p);
    hipStream_t s = S->ctx->stream;
    hipError_t e = hipMemcpyAsync(h, E->X.p, v3, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + v3, E->D.p, 3 * v3, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + 4 * v3, E->U.p, v3, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + 5 * v3, E->W.p, v3, hipMemcpyDeviceToHost, s);
    return e;
}

// A request leaves the device: results (if any) reordered for the caller,
// device arrays and pinned buffers back to the caches.  No queued device
// work uses it any more.
void retire(mrs_server *S, Request *r, mrs_status status) {
    if (status == MRS_OK && r->ens && r->pin_out.p) {
        const int64_t n = r->N;
        const double *h = static_cast<const double *>(r->pin_out.p);
        r->Xo.resize((size_t)n * 3);
        r->Do.resize((size_t)n * 9);
        r->Uo.resize((size_t)n * 3);
        r->Wo.resize((size_t)n * 3);
        soa_to_aos(h, r->Xo.data(), n, 3, r->ens->perm);
        soa_to_aos(h + 3 * n, r->Do.data(), n, 9, r->ens->perm);
        soa_to_aos(h + 12 * n, r->Uo.data(), n, 3, r->ens->perm);
        soa_to_aos(h + 15 * n, r->Wo.data(), n, 3, r->ens->perm);
        status = check_host_finite(S->ctx, h, (size_t)n * 18, "result");  // MRS_ENUMERIC: results still returned
    }
    if (r->ens) {
        drop_plans(S, r->ens->uid);
        ensemble_detach(r->ens);
        r->ens = nullptr;
    }
    S->pins.put(r->pin_in.p, r->pin_in.cap);
    S->pins.put(r->pin_out.p, r->pin_out.cap);
    r->pin_in = r->pin_out = PinBuf{};
    give_event(S, r->up_event);
    r->up_event = nullptr;
    r->info.status = status;
    r->info.steps_done = r->steps_done;
    r->info.t_done = now_s();
}

// Retire the requests of the oldest queued tick once it has finished (wait:
// block until it has).  Returns false if there was none to retire.
bool complete_tick(mrs_server *S, bool wait) {
    if (S->in_flight.empty()) return false;
    Tick &T = S->in_flight.front();
    if (wait) (void)hipEventSynchronize(T.done);
    else if (hipEventQuery(T.done) != hipSuccess) return false;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, T.start, T.done);
    for (auto *r : T.finishing) retire(S, r, MRS_OK);
    S->ticks_completed = T.index + 1;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->st.busy_s += 1e-3 * ms;
        S->st.pairs += T.pairs;
        for (auto *r : T.finishing) {
            S->in_use -= r->footprint;
            r->done = true;
            S->st.completed++;
        }
        auto &A = S->active;
        for (auto *r : T.finishing) A.erase(std::remove(A.begin(), A.end(), r), A.end());
        if (!T.finishing.empty()) S->cv_done.notify_all();
    }
    give_event(S, T.start);
    give_event(S, T.done);
    S->in_flight.pop_front();
    return true;
}

// Every request still on the device ends with `status` once the device has
// drained; used when a tick cannot be queued.
void fail_all(mrs_server *S, mrs_status status) {
    (void)hipStreamSynchronize(S->ctx->stream);
    (void)hipStreamSynchronize(S->up_stream);
    while (complete_tick(S, true)) {
    }
    std::vector<Request *> act;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        act = S->active;
    }
    for (auto *r : act) retire(S, r, status);
    S->plans.clear();
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto *r : act) {
        S->in_use -= r->footprint;
        r->done = true;
        S->st.completed++;
    }
    S->active.clear();
    S->cv_done.notify_all();
}

// Queue one tick over the requests that still have units to launch; false
// if there were none.
bool queue_tick(mrs_server *S) {
    std::vector<Request *> cand;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto *r : S->active)
            if (!r->launched_all) cand.push_back(r);
    }
    if (cand.empty()) return false;
    const int64_t index = S->ticks_launched++;
    for (auto *r : cand)
        if (r->cost == 0) r->cost = (int64_t)evals_per_unit(r) * r->N * r->N;
    std::vector<Request *> run = pick_tick(S, cand);
    if (index + 1 == S->fail_tick) {  // forced failure: nothing queued, every request keeps its state
        std::lock_guard<std::mutex> lk(S->mu);
        S->st.ticks++;
        S->st.failed_ticks++;
        return true;
    }
    mrs_context *ctx = S->ctx;
    hipStream_t s = ctx->stream;
    TickPlan *TP = nullptr;
    mrs_status st = tick_plan(S, run, &TP);
    Tick T;
    T.index = index;
    hipError_t he = st == MRS_OK ? hipSuccess : hipErrorUnknown;
    for (auto *r : run)
        if (he == hipSuccess && r->up_wait) {
            he = hipStreamWaitEvent(s, r->up_event, 0);
            r->up_wait = false;
        }
    if (he == hipSuccess && !((T.start = take_event(S)) && (T.done = take_event(S)))) he = hipErrorOutOfMemory;
    if (he == hipSuccess) he = hipEventRecord(T.start, s);
    if (he == hipSuccess) he = launch_tick(S, *TP);
    if (he == hipSuccess) {
        TP->last_tick = index;
        for (auto *r : run) {
            T.pairs += r->cost;
            if (++r->steps_done >= units(r)) {
                r->launched_all = true;
                T.finishing.push_back(r);
                if ((he = queue_results(S, r)) != hipSuccess) break;
            }
        }
    }
    if (he == hipSuccess) he = hipEventRecord(T.done, s);
    if (he != hipSuccess) {
        give_event(S, T.start);
        give_event(S, T.done);
        if (st == MRS_OK) (void)fail(ctx, MRS_EDEVICE, "tick: %s", hipGetErrorString(he));
        fail_all(S, st != MRS_OK ? st : MRS_EDEVICE);
        return true;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->st.ticks++;
    }
    S->in_flight.push_back(std::move(T));
    return true;
}

void loop(mrs_server *S) {
    (void)hipSetDevice(S->ctx->device);
    for (;;) {
        std::vector<Request *> pick;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            pick = select_admissions(S);
            if (S->active.empty() && pick.empty() && S->in_flight.empty()) {
                if (S->stopping) break;
                S->cv_work.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        std::lock_guard<std::recursive_mutex> ctxlk(S->ctx->mu);
        for (auto *r : pick) {
            const mrs_status st = admit(S, r);
            r->info.t_admit = now_s();
            if (st != MRS_OK) {
                // nothing of it is queued on the compute stream; its uploads are drained
                (void)hipStreamSynchronize(S->up_stream);
                retire(S, r, st);
            }
            std::lock_guard<std::mutex> lk(S->mu);
            if (st == MRS_OK) {
                r->info.status = MRS_ENOTREADY;
                S->active.push_back(r);
                S->st.admitted++;
            } else {
                S->in_use -= r->footprint;
                r->done = true;
                S->st.rejected++;
                S->cv_done.notify_all();
            }
        }
        // retire what has finished, then keep kTicksInFlight ticks queued
        while (complete_tick(S, false)) {
        }
        bool queued = false;
        while ((int)S->in_flight.size() < kTicksInFlight && queue_tick(S)) queued = true;
        if (!queued && !S->in_flight.empty()) complete_tick(S, true);  // nothing more to queue: wait for the oldest
    }
}

mrs_status copy_out(Request *r, mrs_result_info *info, double *X, double *D, double *U, double *W) {
    if (info) *info = r->info;
    const size_t n = (size_t)r->N;
    // a non-finite result is still returned, with status MRS_ENUMERIC
    if (r->info.status == MRS_OK || r->info.status == MRS_ENUMERIC) {
        if (X) std::memcpy(X, r->Xo.data(), n * 3 * sizeof(double));
        if (D) std::memcpy(D, r->Do.data(), n * 9 * sizeof(double));
        if (U) std::memcpy(U, r->Uo.data(), n * 3 * sizeof(double));
        if (W) std::memcpy(W, r->Wo.data(), n * 3 * sizeof(double));
    }
    return (mrs_status)r->info.status;
}

bool finite_all(const double *p, size_t n) {
    for (size_t i = 0; i < n; i++)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

extern "C" {

mrs_status mrs_server_start(mrs_context *ctx, mrs_precision prec, int64_t hbm_budget_bytes, int32_t max_slots,
                            mrs_server **out) {
    if (!ctx || !out) return MRS_EINVAL;
    *out = nullptr;
    if (prec != MRS_FP64 && prec != MRS_FP32C) return fail(ctx, MRS_EINVAL, "unknown precision");
    if (hbm_budget_bytes <= 0 || max_slots < 1) return fail(ctx, MRS_EINVAL, "budget and slots must be positive");
    auto *S = new (std::nothrow) mrs_server();
    if (!S) return MRS_ENOMEM;
    S->ctx = ctx;
    S->prec = (int)prec;
    S->budget = hbm_budget_bytes;
    S->max_slots = max_slots;
    S->st.hbm_budget = hbm_budget_bytes;
    S->t_start = now_s();
    if (const char *v = std::getenv("MRS_DEBUG_FAIL_TICK")) S->fail_tick = std::atoll(v);
    (void)hipSetDevice(ctx->device);
    if (hipStreamCreateWithFlags(&S->up_stream, hipStreamNonBlocking) != hipSuccess) {
        delete S;
        return fail(ctx, MRS_EDEVICE, "upload stream");
    }
    S->th = std::thread(loop, S);
    *out = S;
    return MRS_OK;
}

mrs_status mrs_server_submit(mrs_server *S, const mrs_request *q, uint64_t *ticket) {
    if (!S || !q || !ticket) return MRS_EINVAL;
    if (q->kind != MRS_REQ_EVAL && q->kind != MRS_REQ_STEPS) return MRS_EINVAL;
    if (q->n_fil < 1 || !q->offsets || q->offsets[0] != 0 || !q->X || !q->D) return MRS_EINVAL;
    for (int32_t i = 0; i < q->n_fil; i++)
        if (q->offsets[i + 1] <= q->offsets[i]) return MRS_EINVAL;
    if (!(q->eps > 0) || !(q->mu > 0) || !std::isfinite(q->eps) || !std::isfinite(q->mu)) return MRS_EINVAL;
    if (q->kind == MRS_REQ_STEPS &&
        (q->nsteps < 1 || !std::isfinite(q->dt) ||
         (q->integ != MRS_EULER && q->integ != MRS_RK2 && q->integ != MRS_RK4)))
        return MRS_EINVAL;
    auto *r = new (std::nothrow) Request();
    if (!r) return MRS_ENOMEM;
    r->spec = *q;
    r->N = q->offsets[q->n_fil];
    const size_t n = (size_t)r->N;
    if (!finite_all(q->X, 3 * n) || !finite_all(q->D, 9 * n) || (q->f_ext && !finite_all(q->f_ext, 3 * n)) ||
        (q->n_ext && !finite_all(q->n_ext, 3 * n))) {
        delete r;
        return MRS_EINVAL;
    }
    r->off.assign(q->offsets, q->offsets + q->n_fil + 1);
    r->X.assign(q->X, q->X + 3 * n);
    r->D.assign(q->D, q->D + 9 * n);
    if (q->f_ext || q->n_ext) {
        r->f.assign(3 * n, 0.0);
        r->n.assign(3 * n, 0.0);
        if (q->f_ext) std::memcpy(r->f.data(), q->f_ext, 3 * n * sizeof(double));
        if (q->n_ext) std::memcpy(r->n.data(), q->n_ext, 3 * n * sizeof(double));
    }
    r->spec.offsets = nullptr;
    r->spec.X = r->spec.D = r->spec.f_ext = r->spec.n_ext = nullptr;
    if (q->f_ext || q->n_ext) r->spec.f_ext = r->spec.n_ext = reinterpret_cast<const double *>(1);  // flag only
    r->info.kind = q->kind;
    r->info.n = r->N;
    r->info.status = MRS_ENOTREADY;
    r->info.t_submit = now_s();
    r->footprint = -1;  // computed by the scheduler thread
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) {
        delete r;
        return MRS_EBUSY;
    }
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->table[r->ticket] = r;
    S->st.submitted++;
    S->queue.push_back(r);
    S->cv_work.notify_one();
    return MRS_OK;
}

mrs_status mrs_server_poll(mrs_server *S, uint64_t ticket, mrs_result_info *info, double *X, double *D, double *U,
                           double *W) {
    if (!S) return MRS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->table.find(ticket);
    if (it == S->table.end()) return MRS_EINVAL;
    Request *r = it->second;
    if (!r->done) {
        if (info) *info = r->info;
        return MRS_ENOTREADY;
    }
    mrs_status st = copy_out(r, info, X, D, U, W);
    S->table.erase(it);
    delete r;
    return st;
}

mrs_status mrs_server_wait(mrs_server *S, uint64_t ticket, double timeout_s, mrs_result_info *info, double *X,
                           double *D, double *U, double *W) {
    if (!S) return MRS_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(timeout_s, 0.0));
    for (;;) {
        auto it = S->table.find(ticket);
        if (it == S->table.end()) return MRS_EINVAL;
        Request *r = it->second;
        if (r->done) {
            mrs_status st = copy_out(r, info, X, D, U, W);
            S->table.erase(it);
            delete r;
            return st;
        }
        if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            if (info) *info = r->info;
            return MRS_ENOTREADY;
        }
    }
}

mrs_status mrs_server_set_tick_pairs(mrs_server *S, int64_t max_pairs) {
    if (!S || max_pairs < 0) return MRS_EINVAL;
    S->tick_pairs.store(max_pairs);
    return MRS_OK;
}

mrs_status mrs_server_set_admission(mrs_server *S, int32_t order, double max_wait_s) {
    if (!S || (order != MRS_ADMIT_ARRIVAL && order != MRS_ADMIT_LEAST_WORK) || !(max_wait_s >= 0.0))
        return MRS_EINVAL;
    S->admit_max_wait.store(max_wait_s);
    S->admit_order.store(order);
    S->cv_work.notify_one();
    return MRS_OK;
}

mrs_status mrs_server_stats_get(mrs_server *S, mrs_server_stats *out) {
    if (!S || !out) return MRS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->active = (int32_t)S->active.size();
    out->queued = (int32_t)S->queue.size();
    out->hbm_in_use = S->in_use;
    out->wall_s = now_s() - S->t_start;
    return MRS_OK;
}

mrs_status mrs_server_stop(mrs_server *S) {
    if (!S) return MRS_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
        for (auto *r : S->queue) {
            r->info.status = MRS_EBUSY;
            r->done = true;
        }
        S->queue.clear();
        S->cv_work.notify_all();
    }
    if (S->th.joinable()) S->th.join();
    (void)hipStreamSynchronize(S->ctx->stream);
    (void)hipStreamSynchronize(S->up_stream);
    for (auto &kv : S->table) delete kv.second;
    S->plans.clear();
    for (auto e : S->events) (void)hipEventDestroy(e);
    if (S->up_stream) (void)hipStreamDestroy(S->up_stream);
    delete S;
    return MRS_OK;
}

}  // extern "C"
