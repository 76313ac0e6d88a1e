// Autotuner of the pair kernel: times candidate work decompositions on a
// seeded synthetic filament ensemble and keeps the fastest per size class.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mrs_runtime.h"

using namespace mrs;

namespace {

// Seeded synthetic filaments (straight, 128 points, spacing 1/128, random
// directions) at the density of 100 filaments in a box of side 10, with
// loads in [-1, 1]: same near-pair structure as the configured workloads.
void synth_cloud(int64_t n, std::vector<double> &X, std::vector<double> &f, std::vector<double> &t, double &eps) {
    uint64_t state = 0x9E3779B97F4A7C15ull;
    auto rnd = [&]() {  // splitmix64 -> [0, 1)
        state += 0x9E3779B97F4A7C15ull;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (z >> 11) * (1.0 / 9007199254740992.0);
    };
    const int M = 128;
    const double ds = 1.0 / M;
    eps = 1.5 * ds;
    const int64_t F = (n + M - 1) / M;
    const double box = 10.0 * std::cbrt((double)F / 100.0);
    X.resize(3 * n);
    f.resize(3 * n);
    t.resize(3 * n);
    double base[3] = {0, 0, 0}, dir[3] = {1, 0, 0};
    for (int64_t i = 0; i < n; i++) {
        if (i % M == 0) {
            for (int c = 0; c < 3; c++) base[c] = box * rnd();
            double nn = 0;
            for (int c = 0; c < 3; c++) { dir[c] = 2 * rnd() - 1; nn += dir[c] * dir[c]; }
            nn = std::sqrt(std::max(nn, 1e-12));
            for (int c = 0; c < 3; c++) dir[c] /= nn;
        }
        const double s = (i % M) * ds;
        for (int c = 0; c < 3; c++) {
            X[3 * i + c] = base[c] + s * dir[c];
            f[3 * i + c] = 2 * rnd() - 1;
            t[3 * i + c] = 2 * rnd() - 1;
        }
    }
}

bool valid_cfg(const mrs_pair_config *c) {
    return c && (c->mode == PAIR_TILE || c->mode == PAIR_SPLIT || c->mode == PAIR_QUAD) &&
           (c->targets_per_lane == 1 || c->targets_per_lane == 2) &&
           c->chunks >= 0 && (c->schedule == SCHED_GRID || c->schedule == SCHED_PERSISTENT);
}

}  // namespace

extern "C" {

mrs_status mrs_tune_get(mrs_context *ctx, int64_t n, mrs_precision prec, mrs_pair_config *out) {
    if (!ctx || !out || n < 1 || (prec != MRS_FP64 && prec != MRS_FP32C)) return MRS_EINVAL;
    PairCfg c = choose_cfg(ctx, n, (int)prec);
    out->mode = c.mode;
    out->targets_per_lane = c.tpl;
    out->chunks = c.K;
    out->schedule = c.sched;
    return MRS_OK;
}

mrs_status mrs_tune_set(mrs_context *ctx, int64_t n, mrs_precision prec, const mrs_pair_config *cfg) {
    if (!ctx || n < 1 || (prec != MRS_FP64 && prec != MRS_FP32C) || !valid_cfg(cfg)) return MRS_EINVAL;
    PairCfg c;
    c.mode = cfg->mode;
    c.tpl = cfg->targets_per_lane;
    c.K = cfg->chunks;
    c.sched = cfg->schedule;
    ctx->tune[{(int)prec, size_bucket(n)}] = c;
    return MRS_OK;
}

mrs_status mrs_autotune(mrs_context *ctx, int64_t n, mrs_precision prec, int32_t reps, mrs_pair_config *best,
                        double *best_ms) {
    if (!ctx || n < 1 || n > (1 << 24) || (prec != MRS_FP64 && prec != MRS_FP32C)) return MRS_EINVAL;
    reps = std::max(1, std::min(reps, 20));
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    std::vector<double> X, f, t;
    double eps;
    synth_cloud(n, X, f, t, eps);
    DevBuf io;
    const size_t b = (size_t)n * 3 * sizeof(double);
    if (io.reserve(5 * b) != hipSuccess) return fail(ctx, MRS_ENOMEM, "autotune buffers");
    double *dX = io.as<double>(), *df = dX + 3 * n, *dt = df + 3 * n, *dU = dt + 3 * n, *dW = dU + 3 * n;
    if (hipMemcpy(dX, X.data(), b, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(df, f.data(), b, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dt, t.data(), b, hipMemcpyHostToDevice) != hipSuccess)
        return fail(ctx, MRS_EDEVICE, "autotune upload");

    std::vector<PairCfg> cands;
    if (n <= 8192) {
        PairCfg c;
        c.mode = PAIR_SPLIT;
        cands.push_back(c);
    }
    for (int tpl : {1, 2}) {
        const int64_t tiles = (n + (int64_t)kBlock * tpl - 1) / ((int64_t)kBlock * tpl);
        std::vector<int> Ks;
        for (int per_cu : {1, 2, 4, 8, 16, 32}) {
            int64_t K = ((int64_t)ctx->n_cu * per_cu + tiles - 1) / tiles;
            K = std::max<int64_t>(1, std::min<int64_t>(K, (n + kKahanBlock - 1) / kKahanBlock));
            if (std::find(Ks.begin(), Ks.end(), (int)K) == Ks.end()) Ks.push_back((int)K);
        }
        for (int K : Ks) {
            PairCfg c;
            c.mode = PAIR_TILE;
            c.tpl = tpl;
            c.K = K;
            cands.push_back(c);
        }
    }
    const auto key = std::make_pair((int)prec, size_bucket(n));
    const bool had = ctx->tune.count(key) > 0;
    const PairCfg saved = had ? ctx->tune[key] : PairCfg();
    const bool prof_was = ctx->prof_on;
    std::vector<mrs::ProfRec> prof_saved;
    prof_saved.swap(ctx->prof);
    double best_t = 1e300;
    PairCfg best_c;
    mrs_status st = MRS_OK;
    for (const PairCfg &c : cands) {
        ctx->tune[key] = c;
        std::vector<double> times;
        for (int r = 0; r <= reps && st == MRS_OK; r++) {  // first run is a warm-up
            ctx->prof_on = true;
            st = mrs_eval_device(ctx, n, dX, df, dt, eps, 1.0, prec, dU, dW, ctx->stream);
            ctx->prof_on = false;
            if (st != MRS_OK) break;
            int64_t launches = 0;
            double ms = 0;
            st = mrs_profile_query(ctx, "pairs", &launches, &ms);
            for (auto &p : ctx->prof) {
                ctx->event_pool.push_back(p.start);
                ctx->event_pool.push_back(p.stop);
            }
            ctx->prof.clear();
            if (r > 0) times.push_back(ms);
        }
        if (st != MRS_OK) break;
        std::sort(times.begin(), times.end());
        const double med = times[times.size() / 2];
        if (med < best_t) {
            best_t = med;
            best_c = c;
        }
    }
    ctx->prof_on = prof_was;
    ctx->prof.swap(prof_saved);
    if (st != MRS_OK) {
        if (had) ctx->tune[key] = saved;
        else ctx->tune.erase(key);
        (void)hipStreamSynchronize(ctx->stream);
        return st;
    }
    ctx->tune[key] = best_c;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, MRS_EDEVICE, "autotune sync");
    if (best) {
        best->mode = best_c.mode;
        best->targets_per_lane = best_c.tpl;
        best->chunks = best_c.K;
        best->schedule = best_c.sched;
    }
    if (best_ms) *best_ms = best_t;
    return MRS_OK;
}

}  // extern "C"
