// Serving loop of the MRS filament library: continuous batching of
// independent ensemble requests on one device.
//
// A scheduler thread owns the context.  Each tick it
//   1. admits queued requests in arrival order (first fit) while a slot is
//      free and the request's device footprint fits the HBM budget; the
//      request's state is copied to the device and stays resident there;
//   2. launches ONE batched launch sequence that advances every admitted
//      request by one unit of work: an evaluation, one Euler step or one RK4
//      step (four stages; evaluation and Euler requests take part in the
//      first stage only);
//   3. retires finished requests (copies results to host, frees the slot).
// Requests arriving while a tick runs join at the next tick, so work of
// requests of different sizes and kinds overlaps inside the same kernels.
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

struct Request {
    uint64_t ticket = 0;
    mrs_request spec{};
    std::vector<int32_t> off;
    std::vector<double> X, D, f, n;
    mrs_ensemble *ens = nullptr;
    int64_t N = 0;
    int32_t steps_done = 0;
    int64_t footprint = -1;
    mrs_result_info info{};
    bool done = false;
    double credit = 0.0;  // pair budget earned and not yet spent (deficit round robin)
    int64_t cost = 0;     // pair interactions of one unit of work (eval or step)
    std::vector<double> Xo, Do, Uo, Wo;
};

// Work lists of one tick over the admitted set.
struct TickPlan {
    std::vector<uint64_t> key;  // ensemble uids of the admitted set, in order
    Plan all;       // stage 0 over every admitted request
    Plan rk[2];     // later stages of the RK4 (scheme 0) and RK2 (scheme 1) step requests
    std::vector<PointItem> pts_write, pts_euler, pts_rk0[2];
    DevBuf d_pts_write, d_pts_euler, d_pts_rk0[2];
    bool has_rk[2] = {false, false};
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
    std::vector<Request *> active;
    std::map<uint64_t, Request *> table;
    int64_t in_use = 0;
    uint64_t next_ticket = 1;
    bool stopping = false;
    mrs_server_stats st{};
    int64_t fail_tick = -1;
    std::atomic<int64_t> tick_pairs{0};  // 0 = no per-tick bound
    // tick plans of recently used request sets (small LRU)
    std::vector<std::unique_ptr<TickPlan>> plans;
    TickPlan *plan = nullptr;
};

namespace {

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

// Tick plan of the requests `run` (cached per set; the cache is small LRU).
mrs_status build_tick_plan(mrs_server *S, const std::vector<Request *> &run) {
    std::vector<uint64_t> key;
    for (auto *r : run) key.push_back(r->ens->uid);
    for (size_t i = 0; i < S->plans.size(); i++)
        if (S->plans[i]->key == key) {
            std::rotate(S->plans.begin(), S->plans.begin() + i, S->plans.begin() + i + 1);
            S->plan = S->plans.front().get();
            return MRS_OK;
        }
    auto T = std::make_unique<TickPlan>();
    T->key = key;
    T->all.prec = T->rk[0].prec = T->rk[1].prec = S->prec;
    for (size_t e = 0; e < run.size(); e++) {
        Request *r = run[e];
        Plan *single;
        mrs_status st = ensemble_plan(r->ens, S->prec, &single);
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
    if (S->plans.size() > kPlanCache) S->plans.pop_back();
    S->plan = S->plans.front().get();
    return MRS_OK;
}

// Forget cached plans that mention a retired request's ensemble.
void drop_plans(mrs_server *S, uint64_t uid) {
    for (auto it = S->plans.begin(); it != S->plans.end();) {
        const auto &k = (*it)->key;
        if (std::find(k.begin(), k.end(), uid) != k.end()) it = S->plans.erase(it);
        else ++it;
    }
    S->plan = nullptr;
}

int evals_per_unit(const Request *r) {
    return (r->spec.kind == MRS_REQ_STEPS && r->spec.integ != MRS_EULER) ? rk_stages(r->spec.integ) : 1;
}

// Requests that advance in this tick: all of them without a tick bound; with
// one, deficit round robin over the admitted requests.
std::vector<Request *> pick_tick(mrs_server *S) {
    const int64_t budget = S->tick_pairs.load();
    if (budget <= 0) return S->active;
    std::vector<Request *> run;
    const double quantum = (double)budget / (double)S->active.size();
    Request *best = nullptr;
    for (auto *r : S->active) {
        r->credit += quantum;
        if (r->credit >= (double)r->cost) run.push_back(r);
        if (!best || r->credit / (double)r->cost > best->credit / (double)best->cost) best = r;
    }
    if (run.empty()) run.push_back(best);  // always make progress
    for (auto *r : run) r->credit = std::max(0.0, r->credit - (double)r->cost);
    return run;
}

hipError_t launch_tick(mrs_server *S) {
    mrs_context *ctx = S->ctx;
    TickPlan &T = *S->plan;  // set by build_tick_plan
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
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

// Pick queued requests to admit (arrival order, first fit).  Caller holds S->mu.
std::vector<Request *> select_admissions(mrs_server *S) {
    std::vector<Request *> pick;
    int64_t used = S->in_use;
    for (auto it = S->queue.begin(); it != S->queue.end();) {
        if ((int32_t)(S->active.size() + pick.size()) >= S->max_slots) break;
        Request *r = *it;
        if (r->footprint < 0) r->footprint = request_footprint(S->ctx, S->prec, *r);
        if (r->footprint > S->budget) {  // can never fit
            r->info.status = MRS_ENOMEM;
            r->info.t_admit = r->info.t_done = now_s();
            r->done = true;
            S->st.rejected++;
            it = S->queue.erase(it);
            S->cv_done.notify_all();
            continue;
        }
        if (used + r->footprint > S->budget) {
            ++it;
            continue;
        }
        used += r->footprint;
        pick.push_back(r);
        it = S->queue.erase(it);
    }
    S->in_use = used;
    return pick;
}

// Copy the picked requests to the device.  Caller holds the context lock only.
void create_ensembles(mrs_server *S, std::vector<Request *> &pick) {
    for (auto *r : pick) {
        const mrs_request &q = r->spec;
        mrs_ensemble *ens = nullptr;
        mrs_status st = mrs_ensemble_create(S->ctx, q.n_fil, r->off.data(), r->X.data(), r->D.data(),
                                            r->f.empty() ? nullptr : r->f.data(),
                                            r->n.empty() ? nullptr : r->n.data(), q.eps, q.mu, &q.rod, &ens);
        r->info.t_admit = now_s();
        r->info.status = st == MRS_OK ? MRS_ENOTREADY : st;
        r->ens = ens;
        std::vector<double>().swap(r->X);  // inputs now live on the device
        std::vector<double>().swap(r->D);
        std::vector<double>().swap(r->f);
        std::vector<double>().swap(r->n);
    }
}

// Copy results of a finished request to host and free its device state;
// a result with a non-finite value completes with MRS_ENUMERIC.  Caller
// holds the context lock only.
void collect(Request *r, mrs_status status) {
    if (status == MRS_OK && r->ens) {
        r->Xo.resize((size_t)r->N * 3);
        r->Do.resize((size_t)r->N * 9);
        r->Uo.resize((size_t)r->N * 3);
        r->Wo.resize((size_t)r->N * 3);
        status = mrs_ensemble_get(r->ens, r->Xo.data(), r->Do.data(), r->Uo.data(), r->Wo.data());
    }
    if (r->ens) mrs_ensemble_destroy(r->ens);
    r->ens = nullptr;
    r->info.status = status;
    r->info.steps_done = r->steps_done;
    r->info.t_done = now_s();
}

void loop(mrs_server *S) {
    (void)hipSetDevice(S->ctx->device);
    int64_t tick = 0;
    for (;;) {
        std::vector<Request *> pick;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            pick = select_admissions(S);
            if (S->active.empty() && pick.empty()) {
                if (S->stopping) break;
                S->cv_work.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        std::lock_guard<std::recursive_mutex> ctxlk(S->ctx->mu);
        if (!pick.empty()) {
            create_ensembles(S, pick);
            std::lock_guard<std::mutex> lk(S->mu);
            for (auto *r : pick) {
                if (r->ens) {
                    S->active.push_back(r);
                    S->st.admitted++;
                } else {
                    S->in_use -= r->footprint;
                    r->info.t_done = now_s();
                    r->done = true;
                    S->st.rejected++;
                }
            }
            S->cv_done.notify_all();
        }
        if (S->active.empty()) continue;
        tick++;
        for (auto *r : S->active)
            if (r->cost == 0) r->cost = (int64_t)evals_per_unit(r) * r->N * r->N;
        std::vector<Request *> run = pick_tick(S);
        mrs_status st = build_tick_plan(S, run);
        const double t0 = now_s();
        hipError_t he = hipSuccess;
        bool failed = false;
        if (st == MRS_OK) {
            if (tick == S->fail_tick) failed = true;  // forced failure: nothing launched, state unchanged
            else he = launch_tick(S);
        }
        const double t1 = now_s();
        if (failed) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->st.ticks++;
            S->st.failed_ticks++;
            continue;  // every request retries this tick from its step-boundary state
        }
        std::vector<Request *> keep, finished;
        int64_t pairs = 0;
        const bool ok = st == MRS_OK && he == hipSuccess;
        for (auto *r : S->active) {
            if (!ok) {
                finished.push_back(r);
                continue;
            }
            if (std::find(run.begin(), run.end(), r) == run.end()) {  // did not run this tick
                keep.push_back(r);
                continue;
            }
            pairs += r->cost;
            const bool fin = r->spec.kind == MRS_REQ_EVAL || ++r->steps_done >= r->spec.nsteps;
            (fin ? finished : keep).push_back(r);
        }
        for (auto *r : finished) {
            if (r->ens) drop_plans(S, r->ens->uid);
            collect(r, ok ? MRS_OK : (st != MRS_OK ? st : MRS_EDEVICE));
        }
        if (!ok) {
            S->plans.clear();
            S->plan = nullptr;
        }
        std::lock_guard<std::mutex> lk(S->mu);
        S->st.ticks++;
        S->st.busy_s += t1 - t0;
        S->st.pairs += pairs;
        for (auto *r : finished) {
            S->in_use -= r->footprint;
            r->done = true;
            S->st.completed++;
        }
        S->active.swap(keep);
        if (!finished.empty()) S->cv_done.notify_all();
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
    if (const char *v = std::getenv("MRS_DEBUG_FAIL_TICK")) S->fail_tick = std::atoll(v);
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

mrs_status mrs_server_stats_get(mrs_server *S, mrs_server_stats *out) {
    if (!S || !out) return MRS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->active = (int32_t)S->active.size();
    out->queued = (int32_t)S->queue.size();
    out->hbm_in_use = S->in_use;
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
    for (auto &kv : S->table) delete kv.second;
    S->plans.clear();
    delete S;
    return MRS_OK;
}

}  // extern "C"
