// Autotuner of the pair kernel: times candidate work decompositions on a
// seeded synthetic filament ensemble and keeps the fastest per size class.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <ctime>
#include <vector>

#include <unistd.h>

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

bool same_cfg(const PairCfg &a, const PairCfg &b) {
    return a.mode == b.mode && a.tpl == b.tpl && a.K == b.K && a.sched == b.sched;
}

PairCfg stored(int mode, int tpl, int K, int sched) {
    PairCfg c;
    c.mode = mode;
    c.tpl = tpl;
    c.K = K;
    c.sched = sched;
    return c;
}

// The automatic configuration as a table entry: chunks = 0 keeps the
// automatic chunking, tail split included, so storing it changes nothing.
PairCfg automatic_entry(int64_t n, int prec, int n_cu) {
    const PairCfg a = choose_cfg_for(nullptr, n, prec, n_cu);
    return stored(a.mode, a.tpl, a.mode == PAIR_SPLIT ? 1 : 0, a.sched);
}

// Candidates for n points; the first is the automatic configuration.
std::vector<PairCfg> candidates(int64_t n, int prec, int n_cu) {
    std::vector<PairCfg> out;
    auto add = [&](const PairCfg &c) {
        for (const PairCfg &o : out)
            if (same_cfg(o, c)) return;
        out.push_back(c);
    };
    add(automatic_entry(n, prec, n_cu));
    if (n <= 8192) add(stored(PAIR_SPLIT, 1, 1, SCHED_GRID));
    // chunk counts that give 1 ... 64 blocks per compute unit
    auto ks = [&](int64_t tile) {
        const int64_t tiles = (n + tile - 1) / tile;
        std::vector<int> out_k;
        for (int per_cu : {1, 2, 4, 8, 16, 32, 64}) {
            int64_t K = ((int64_t)n_cu * per_cu + tiles - 1) / tiles;
            K = std::max<int64_t>(1, std::min<int64_t>(K, (n + kKahanBlock - 1) / kKahanBlock));
            if (std::find(out_k.begin(), out_k.end(), (int)K) == out_k.end()) out_k.push_back((int)K);
        }
        return out_k;
    };
    for (int tpl : {1, 2}) {
        add(stored(PAIR_TILE, tpl, 0, SCHED_GRID));
        add(stored(PAIR_TILE, tpl, 0, SCHED_PERSISTENT));
        for (int K : ks((int64_t)kBlock * tpl)) add(stored(PAIR_TILE, tpl, K, SCHED_GRID));
    }
    if (prec == MRS_FP32C) {
        add(stored(PAIR_QUAD, 1, 0, SCHED_GRID));
        add(stored(PAIR_QUAD, 1, 0, SCHED_PERSISTENT));
        const std::vector<int> kq = ks(64);
        for (size_t i = 0; i < kq.size(); i += 2) add(stored(PAIR_QUAD, 1, kq[i], SCHED_GRID));
    }
    return out;
}

// Seconds since the epoch (stamp of a tuning table).
long long now_s() { return (long long)std::time(nullptr); }

mrs_status save_table(mrs_context *ctx, const char *path) {
    // written beside the table and renamed over it, so that a reader never
    // sees half a table (one temporary name per process)
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    FILE *fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return fail(ctx, MRS_EINVAL, "cannot write %s", tmp.c_str());
    std::fprintf(fp, "mrs-pair-tuning 1 %s %d %lld\n", ctx->arch.c_str(), ctx->n_cu, now_s());
    std::fprintf(fp, "# precision size_class mode targets_per_lane chunks schedule tuned_ms automatic_ms\n");
    for (auto &kv : ctx->tune) {
        const PairCfg &c = kv.second;
        auto t = ctx->tune_ms.find(kv.first);
        std::fprintf(fp, "%d %d %d %d %d %d %.6f %.6f\n", kv.first.first, kv.first.second, c.mode, c.tpl, c.K,
                     c.sched, t != ctx->tune_ms.end() ? t->second.first : -1.0,
                     t != ctx->tune_ms.end() ? t->second.second : -1.0);
    }
    const bool ok = std::fflush(fp) == 0 && !std::ferror(fp);
    std::fclose(fp);
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(ctx, MRS_EINVAL, "cannot write %s", path);
    }
    return MRS_OK;
}

// missing_ok: a file that does not exist loads nothing and is no error.
mrs_status load_table(mrs_context *ctx, const char *path, bool missing_ok) {
    FILE *fp = std::fopen(path, "r");
    if (!fp) return missing_ok ? MRS_OK : fail(ctx, MRS_EINVAL, "cannot read %s", path);
    char line[512], arch[128];
    int version = 0, n_cu = 0;
    long long stamp = 0;
    mrs_status st = MRS_OK;
    if (!std::fgets(line, sizeof line, fp) ||
        std::sscanf(line, "mrs-pair-tuning %d %127s %d %lld", &version, arch, &n_cu, &stamp) != 4 || version != 1) {
        st = fail(ctx, MRS_EINVAL, "%s: not a tuning table", path);
    } else if (ctx->arch != arch || ctx->n_cu != n_cu) {
        st = fail(ctx, MRS_EINVAL, "%s: tuned on %s with %d compute units, this device is %s with %d", path, arch,
                  n_cu, ctx->arch.c_str(), ctx->n_cu);
    }
    std::map<std::pair<int, int>, PairCfg> entries;
    std::map<std::pair<int, int>, std::pair<double, double>> times;
    int lineno = 1;
    while (st == MRS_OK && std::fgets(line, sizeof line, fp)) {
        lineno++;
        if (line[0] == '#' || line[0] == '\n') continue;
        int prec, bucket;
        mrs_pair_config c;
        double tms, dms;
        if (std::sscanf(line, "%d %d %d %d %d %d %lf %lf", &prec, &bucket, &c.mode, &c.targets_per_lane, &c.chunks,
                        &c.schedule, &tms, &dms) != 8 ||
            (prec != MRS_FP64 && prec != MRS_FP32C) || bucket < 0 || bucket > 40 || !valid_cfg(&c)) {
            st = fail(ctx, MRS_EINVAL, "%s:%d: bad entry", path, lineno);
            break;
        }
        entries[{prec, bucket}] = stored(c.mode, c.targets_per_lane, c.chunks, c.schedule);
        times[{prec, bucket}] = {tms, dms};
    }
    std::fclose(fp);
    if (st != MRS_OK) return st;
    for (auto &kv : entries) ctx->tune[kv.first] = kv.second;
    for (auto &kv : times) ctx->tune_ms[kv.first] = kv.second;
    return MRS_OK;
}

// Device time of one mrs_eval_device call: the sum of its kernels' event
// times (the host work between launches is not counted).
mrs_status time_eval(mrs_context *ctx, int64_t n, const double *dX, const double *df, const double *dt, double eps,
                     int prec, double *dU, double *dW, double *ms) {
    ctx->prof_on = true;
    mrs_status st = mrs_eval_device(ctx, n, dX, df, dt, eps, 1.0, (mrs_precision)prec, dU, dW, ctx->stream);
    ctx->prof_on = false;
    if (st != MRS_OK) return st;
    int64_t launches = 0;
    st = mrs_profile_query(ctx, "", &launches, ms);
    for (auto &p : ctx->prof) {
        ctx->event_pool.push_back(p.start);
        ctx->event_pool.push_back(p.stop);
    }
    ctx->prof.clear();
    return st;
}

double median(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    return v.empty() ? 1e300 : v[v.size() / 2];
}

}  // namespace

namespace mrs {

// Largest ensemble tuned on first use: a tuning pass takes about 60
// evaluations, 7 s in FP64 at 256,000 points; larger size classes keep the
// table or the automatic configuration unless mrs_autotune is called.
constexpr int64_t kFirstUseMaxPoints = 1 << 18;

mrs_status tune_if_unseen(mrs_context *ctx, int64_t n, int prec) {
    if (ctx->tune_first_use <= 0 || n > kFirstUseMaxPoints ||
        ctx->tune.count({prec, size_bucket(std::max<int64_t>(n, 1))}))
        return MRS_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return MRS_OK;
    return mrs_autotune(ctx, n, (mrs_precision)prec, ctx->tune_first_use, nullptr, nullptr);
}

}  // namespace mrs

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
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    const auto key = std::make_pair((int)prec, size_bucket(n));
    ctx->tune[key] = stored(cfg->mode, cfg->targets_per_lane, cfg->chunks, cfg->schedule);
    ctx->tune_ms.erase(key);
    return MRS_OK;
}

mrs_status mrs_tune_save(mrs_context *ctx, const char *path) {
    if (!ctx || !path || !*path) return MRS_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    return save_table(ctx, path);
}

mrs_status mrs_tune_load(mrs_context *ctx, const char *path) {
    if (!ctx || !path || !*path) return MRS_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    return load_table(ctx, path, false);
}

mrs_status mrs_tune_on_first_use(mrs_context *ctx, int32_t reps, const char *table_path) {
    if (!ctx || reps < 0 || reps > 20) return MRS_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (table_path && *table_path) {
        mrs_status st = load_table(ctx, table_path, true);
        if (st != MRS_OK) return st;
        // written once now, so that a path that cannot be written is
        // refused here and not by a later evaluation that tunes
        if ((st = save_table(ctx, table_path)) != MRS_OK) return st;
        ctx->tune_path = table_path;
    } else {
        ctx->tune_path.clear();
    }
    ctx->tune_first_use = reps;
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

    const std::vector<PairCfg> cands = candidates(n, (int)prec, ctx->n_cu);
    const auto key = std::make_pair((int)prec, size_bucket(n));
    const bool had = ctx->tune.count(key) > 0;
    const PairCfg saved = had ? ctx->tune[key] : PairCfg();
    const bool prof_was = ctx->prof_on;
    const std::string sel_was = ctx->prof_sel;
    ctx->prof_sel.clear();
    std::vector<mrs::ProfRec> prof_saved;
    prof_saved.swap(ctx->prof);
    std::vector<std::vector<double>> times(cands.size());
    mrs_status st = MRS_OK;
    // run candidate i `runs` more times (after one untimed warm-up run)
    auto run = [&](size_t i, int runs) {
        ctx->tune[key] = cands[i];
        for (int r = times[i].empty() ? -1 : 0; r < runs && st == MRS_OK; r++) {
            double ms = 0;
            st = time_eval(ctx, n, dX, df, dt, eps, (int)prec, dU, dW, &ms);
            if (st == MRS_OK && r >= 0) times[i].push_back(ms);
        }
    };
    // first pass: every candidate once; second pass: the fastest quarter (at least
    // four) and the automatic configuration `reps` more times, interleaved
    // so that slow drifts of the clock touch every candidate alike
    for (size_t i = 0; i < cands.size() && st == MRS_OK; i++) run(i, 1);
    std::vector<size_t> order(cands.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t c) { return times[a][0] < times[c][0]; });
    const size_t keep = std::min(order.size(), std::max<size_t>(4, order.size() / 4));
    std::vector<size_t> final_set(order.begin(), order.begin() + keep);
    if (std::find(final_set.begin(), final_set.end(), (size_t)0) == final_set.end()) final_set.push_back(0);
    for (auto i : final_set) times[i].clear();
    for (int r = 0; r < reps && st == MRS_OK; r++)
        for (size_t i : final_set) run(i, 1);
    ctx->prof_on = prof_was;
    ctx->prof_sel = sel_was;
    ctx->prof.swap(prof_saved);
    if (st != MRS_OK) {
        if (had) ctx->tune[key] = saved;
        else ctx->tune.erase(key);
        (void)hipStreamSynchronize(ctx->stream);
        return st;
    }
    // the automatic configuration (index 0) stays unless a candidate beats
    // its median by more than 1%
    size_t pick = 0;
    const double auto_ms = median(times[0]);
    for (size_t i : final_set)
        if (median(times[i]) < median(times[pick]) && median(times[i]) < 0.99 * auto_ms) pick = i;
    ctx->tune[key] = cands[pick];
    ctx->tune_ms[key] = {median(times[pick]), auto_ms};
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, MRS_EDEVICE, "autotune sync");
    if (!ctx->tune_path.empty()) {
        st = save_table(ctx, ctx->tune_path.c_str());
        if (st != MRS_OK) return st;
    }
    if (best) {
        best->mode = cands[pick].mode;
        best->targets_per_lane = cands[pick].tpl;
        best->chunks = cands[pick].K;
        best->schedule = cands[pick].sched;
    }
    if (best_ms) *best_ms = median(times[pick]);
    return MRS_OK;
}

}  // extern "C"
