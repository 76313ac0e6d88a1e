// Parareal (Sec. II.D) on one device: the fine propagations of the slices run
// as batched launch sequences; the coarse sweep and the correction of Eq.
// serial_correct run on the device; slice-boundary states stay resident.
//
// Two schedules compute the same iterates bit for bit.  The regular one
// (mrs_parareal) runs the fine propagations of an iteration as one batch
// after the serial sweep that feeds them.  The pipelined one
// (mrs_parareal_pipelined, Sec. II.D's pipelined scheduling) splits the
// slices into groups: a group's fine batch starts on a stream of its own as
// soon as the sweep has produced its start states, and the next sweep corrects
// each slice as soon as its group is done, so the serial coarse work overlaps
// the fine work.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mrs_runtime.h"

using namespace mrs;

namespace {

// Slice-boundary states: n_states states of 12 N doubles each (X SoA then D SoA).
struct States {
    DevBuf buf;
    int64_t N = 0;
    double *X(int n) const { return buf.as<double>() + (size_t)n * 12 * N; }
    double *D(int n) const { return X(n) + 3 * N; }
};

hipError_t copy_state(double *dX, double *dD, const double *sX, const double *sD, int64_t N, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(dX, sX, (size_t)N * 3 * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dD, sD, (size_t)N * 9 * sizeof(double), hipMemcpyDeviceToDevice, s);
    return e;
}

// max over points of |a_i - b_i| / |a_i| (positions, SoA, host copies)
double rel_increment(const std::vector<double> &a, const std::vector<double> &b, int64_t N) {
    double worst = 0.0;
    for (int64_t i = 0; i < N; i++) {
        double num = 0.0, den = 0.0;
        for (int c = 0; c < 3; c++) {
            const double d = a[(size_t)c * N + i] - b[(size_t)c * N + i];
            num += d * d;
            den += a[(size_t)c * N + i] * a[(size_t)c * N + i];
        }
        const double r = den > 0.0 ? std::sqrt(num / den) : std::sqrt(num);
        worst = std::max(worst, r);
    }
    return worst;
}

// Device events of one solve, destroyed with it.
struct Events {
    std::vector<hipEvent_t> ev;
    ~Events() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    bool create(size_t n) {
        ev.assign(n, nullptr);
        for (auto &e : ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return false;
        return true;
    }
};

// What both schedules share: arguments, the coarse worker W[0] and one fine
// worker W[n] per slice (clones of the ensemble, kept with it between calls
// so that their batch plans and graphs are reused), the slice boundary
// times, the state buffers and events.  Destruction waits for the streams.
struct Solve {
    mrs_context *ctx = nullptr;
    mrs_ensemble *E = nullptr;
    int32_t ns = 0, fsteps = 0, csteps = 0;
    mrs_integrator fi = MRS_RK4;
    double fdt = 0.0, cdt = 0.0;
    mrs_precision prec = MRS_FP64;
    int el = 0;
    int64_t N = 0;
    std::vector<double> T;  // T[n]: time at the start of slice n
    States st[6];
    Events ev[3];
    std::vector<mrs_ensemble *> W;

    ~Solve() {
        if (ctx) {
            (void)hipStreamSynchronize(ctx->stream);
            for (auto a : ctx->aux_stream)
                if (a) (void)hipStreamSynchronize(a);
        }
    }

    mrs_status init(mrs_ensemble *ens, int32_t n_slices, mrs_integrator integ, double dt, int32_t fine_steps,
                    int32_t coarse_steps, int32_t max_iter, double tol, mrs_precision p, int include_elastic) {
        E = ens;
        ctx = E->ctx;
        if (n_slices < 1 || fine_steps < 1 || coarse_steps < 1 || max_iter < 1 || max_iter > n_slices)
            return fail(ctx, MRS_EINVAL, "need n_slices, fine_steps, coarse_steps >= 1 and 1 <= max_iter <= n_slices");
        if (!std::isfinite(dt) || !std::isfinite(tol) || tol < 0.0) return fail(ctx, MRS_EINVAL, "bad dt or tol");
        if (integ != MRS_EULER && integ != MRS_RK2 && integ != MRS_RK4) return fail(ctx, MRS_EINVAL, "unknown integrator");
        if (p != MRS_FP64 && p != MRS_FP32C) return fail(ctx, MRS_EINVAL, "unknown precision");
        ns = n_slices;
        fi = integ;
        fdt = dt;
        fsteps = fine_steps;
        csteps = coarse_steps;
        cdt = fdt * fsteps / csteps;
        prec = p;
        el = include_elastic ? 1 : 0;
        N = E->N;
        numeric_reset(ctx);
        mrs_status wst = ensemble_workers(E, ns + 1, W);
        if (wst != MRS_OK) return wst;
        // slice boundary times, accumulated step by step exactly as the
        // device clock of a serial fine run accumulates them
        T.assign(ns + 1, 0.0);
        if (hipMemcpy(&T[0], E->clock.p, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal clock read");
        for (int n = 1; n <= ns; n++) {
            T[n] = T[n - 1];
            for (int k = 0; k < fsteps; k++) T[n] += fdt;
        }
        return MRS_OK;
    }

    // The first n_states state buffers, (ns + 1) states each.
    mrs_status alloc(int n_states) {
        for (int i = 0; i < n_states; i++) {
            st[i].N = N;
            if (st[i].buf.reserve((size_t)(ns + 1) * 12 * N * sizeof(double)) != hipSuccess)
                return fail(ctx, MRS_ENOMEM, "parareal state buffers");
        }
        return MRS_OK;
    }

    hipError_t set_clock(mrs_ensemble *w, int n, hipStream_t s) {
        return hipMemcpyAsync(w->clock.p, &T[n], sizeof(double), hipMemcpyHostToDevice, s);
    }

    // G: coarse propagation of slice n0 from (X, D) into (oX, oD), queued on s.
    mrs_status coarse(const double *X, const double *D, int n0, double *oX, double *oD, hipStream_t s) {
        mrs_ensemble *C = W[0];
        if (copy_state(C->X.as<double>(), C->D.as<double>(), X, D, N, s) != hipSuccess ||
            set_clock(C, n0, s) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal copy");
        mrs_status r = ensemble_enqueue(C, MRS_EULER, cdt, csteps, prec, el, s);
        if (r != MRS_OK) return r;
        if (copy_state(oX, oD, C->X.as<double>(), C->D.as<double>(), N, s) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal copy");
        return MRS_OK;
    }

    // X = Fv + Gn - Go with re-orthonormalised frames (Eq. serial_correct), slice n.
    mrs_status correct(const States &Fv, const States &Gn, const States &Go, const States &V, int n, hipStream_t s) {
        hipError_t he = timed(ctx, "parareal_correct", s, [&] {
            return launch_parareal_correct((int)N, Fv.X(n), Fv.D(n), Gn.X(n), Gn.D(n), Go.X(n), Go.D(n), V.X(n),
                                           V.D(n), s);
        });
        if (he != hipSuccess) return fail(ctx, MRS_EDEVICE, "parareal correction: %s", hipGetErrorString(he));
        return MRS_OK;
    }

    // Relative increment of slice boundary n between two iterates (waits for s).
    mrs_status increment(const double *Xnew, const double *Xold, std::vector<double> &ha, std::vector<double> &hb,
                         hipStream_t s, double *inc) {
        if (hipMemcpyAsync(ha.data(), Xnew, ha.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(hb.data(), Xold, hb.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal increment copy");
        *inc = std::max(*inc, rel_increment(ha, hb, N));
        return MRS_OK;
    }

    // The result: the last boundary state and its time into the ensemble.
    // MRS_ENUMERIC when a propagation produced a non-finite value (flag of
    // the reduction kernels, cleared by init) or an increment was not finite.
    mrs_status finish(const States &U, hipStream_t s, bool finite_increments) {
        if (copy_state(E->X.as<double>(), E->D.as<double>(), U.X(ns), U.D(ns), N, s) != hipSuccess ||
            set_clock(E, ns, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal result copy");
        mrs_status st = numeric_check(ctx);
        if (st == MRS_OK && !finite_increments) st = fail(ctx, MRS_ENUMERIC, "non-finite Parareal increment");
        return st;
    }
};

}  // namespace

extern "C" mrs_status mrs_parareal(mrs_ensemble *E, int32_t ns, mrs_integrator fi, double fdt, int32_t fsteps,
                                   int32_t csteps, int32_t max_iter, double tol, mrs_precision prec,
                                   int include_elastic, double *history, int32_t *iters) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    Solve S;
    mrs_status st = S.init(E, ns, fi, fdt, fsteps, csteps, max_iter, tol, prec, include_elastic);
    if (st != MRS_OK) return st;
    hipStream_t s = ctx->stream;
    const int64_t N = S.N;
    // U: current iterate, V: next iterate, Go / Gn: coarse values, Fv: fine values
    if ((st = S.alloc(5)) != MRS_OK) return st;
    States &U = S.st[0], &V = S.st[1], &Go = S.st[2], &Gn = S.st[3], &Fv = S.st[4];

    // iteration 0: serial coarse sweep (Eq. initial)
    if (copy_state(U.X(0), U.D(0), E->X.as<double>(), E->D.as<double>(), N, s) != hipSuccess)
        return fail(ctx, MRS_EDEVICE, "parareal copy");
    for (int n = 1; n <= ns; n++) {
        if ((st = S.coarse(U.X(n - 1), U.D(n - 1), n - 1, Go.X(n), Go.D(n), s)) != MRS_OK) return st;
        if (copy_state(U.X(n), U.D(n), Go.X(n), Go.D(n), N, s) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal copy");
    }
    std::vector<double> ha((size_t)3 * N), hb((size_t)3 * N);
    int done = 0;
    bool finite_inc = true;
    for (int k = 1; k <= max_iter; k++) {
        // fine propagations of slices k..ns from the previous iterate, batched (Eq. intermediate)
        std::vector<mrs_ensemble *> batch;
        for (int n = k; n <= ns; n++) {
            if (copy_state(S.W[n]->X.as<double>(), S.W[n]->D.as<double>(), U.X(n - 1), U.D(n - 1), N, s) !=
                    hipSuccess ||
                S.set_clock(S.W[n], n - 1, s) != hipSuccess)
                return fail(ctx, MRS_EDEVICE, "parareal copy");
            batch.push_back(S.W[n]);
        }
        st = batch_enqueue(ctx, (int32_t)batch.size(), batch.data(), fi, fdt, fsteps, prec, S.el, 1, s);
        if (st != MRS_OK) return st;
        for (int n = k; n <= ns; n++)
            if (copy_state(Fv.X(n), Fv.D(n), S.W[n]->X.as<double>(), S.W[n]->D.as<double>(), N, s) != hipSuccess)
                return fail(ctx, MRS_EDEVICE, "parareal copy");
        // slices before k are converged; slice k takes its fine value
        for (int n = 0; n < k; n++)
            if (copy_state(V.X(n), V.D(n), U.X(n), U.D(n), N, s) != hipSuccess)
                return fail(ctx, MRS_EDEVICE, "parareal copy");
        if (copy_state(V.X(k), V.D(k), Fv.X(k), Fv.D(k), N, s) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal copy");
        // serial correction (Eq. serial_correct)
        for (int n = k + 1; n <= ns; n++) {
            if ((st = S.coarse(V.X(n - 1), V.D(n - 1), n - 1, Gn.X(n), Gn.D(n), s)) != MRS_OK) return st;
            if ((st = S.correct(Fv, Gn, Go, V, n, s)) != MRS_OK) return st;
        }
        // relative increment over the slice boundaries that changed (Eq. true_err, second form)
        double inc = 0.0;
        for (int n = k; n <= ns; n++)
            if ((st = S.increment(V.X(n), U.X(n), ha, hb, s, &inc)) != MRS_OK) return st;
        std::swap(U.buf.p, V.buf.p);
        std::swap(U.buf.bytes, V.buf.bytes);
        std::swap(Go.buf.p, Gn.buf.p);
        std::swap(Go.buf.bytes, Gn.buf.bytes);
        if (history) history[k - 1] = inc;
        done = k;
        finite_inc = finite_inc && std::isfinite(inc);
        if (!(inc > tol)) break;
    }
    if (iters) *iters = done;
    return S.finish(U, s, finite_inc);
}

extern "C" mrs_status mrs_parareal_pipelined(mrs_ensemble *E, int32_t ns, mrs_integrator fi, double fdt,
                                             int32_t fsteps, int32_t csteps, int32_t max_iter, double tol,
                                             mrs_precision prec, int include_elastic, int32_t group,
                                             double *history, int32_t *iters) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ns >= 1 && (group < 0 || group > ns)) return fail(ctx, MRS_EINVAL, "group must be in [0, n_slices]");
    Solve S;
    mrs_status st = S.init(E, ns, fi, fdt, fsteps, csteps, max_iter, tol, prec, include_elastic);
    if (st != MRS_OK) return st;
    const int g = group > 0 ? group : std::max(1, (ns + 3) / 4);
    // sweeps (coarse propagation, correction) on the context's stream; the
    // fine groups on up to three more, group j on stream j % n_sf, so that
    // groups of one iteration run side by side and a slice's fine worker is
    // always used from one stream
    hipStream_t sc = ctx->stream, sf[3];
    const int n_groups = (ns + g - 1) / g, n_sf = std::min(3, n_groups);
    for (int i = 0; i < n_sf; i++)
        if (!(sf[i] = aux_stream(ctx, i))) return fail(ctx, MRS_EDEVICE, "fine streams");
    auto fine_stream = [&](int b) { return sf[((b - 1) / g) % n_sf]; };
    const int64_t N = S.N;
    // iterate k lives in It[k % 2], the coarse values G(X^k_{n-1}) of sweep k
    // in Gc[k % 2], the fine values F(X^{k-1}_{n-1}) in Fv[k % 2]
    if ((st = S.alloc(6)) != MRS_OK) return st;
    States *It = S.st, *Gc = S.st + 2, *Fv = S.st + 4;
    // state_ready[n]: boundary n of the current sweep is final (on sc);
    // fine_done[k % 2][b]: the fine group of iteration k ending at slice b is done
    Events &state_ready = S.ev[0], *fine_done = S.ev + 1;
    if (!state_ready.create(ns + 1) || !fine_done[0].create(ns + 1) || !fine_done[1].create(ns + 1))
        return fail(ctx, MRS_EDEVICE, "parareal events");
    // groups are aligned: slices (j - 1) g + 1 .. j g, clipped to [k, ns] in iteration k
    auto group_end = [&](int n) { return std::min(ns, ((n + g - 1) / g) * g); };

    // Queues the fine group [a, b] of iteration k: start states from iterate
    // k - 1 (final once state_ready[b - 1] of sweep k - 1 has fired).
    auto launch_group = [&](int k, int a, int b) -> mrs_status {
        hipStream_t fs = fine_stream(b);
        if (hipStreamWaitEvent(fs, state_ready.ev[b - 1], 0) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal wait");
        const States &P = It[(k - 1) & 1];
        for (int n = a; n <= b; n++)
            if (copy_state(S.W[n]->X.as<double>(), S.W[n]->D.as<double>(), P.X(n - 1), P.D(n - 1), N, fs) !=
                    hipSuccess ||
                S.set_clock(S.W[n], n - 1, fs) != hipSuccess)
                return fail(ctx, MRS_EDEVICE, "parareal copy");
        mrs_status r = batch_enqueue(ctx, b - a + 1, S.W.data() + a, fi, fdt, fsteps, prec, S.el, 1, fs);
        if (r != MRS_OK) return r;
        for (int n = a; n <= b; n++)
            if (copy_state(Fv[k & 1].X(n), Fv[k & 1].D(n), S.W[n]->X.as<double>(), S.W[n]->D.as<double>(), N,
                           fs) != hipSuccess)
                return fail(ctx, MRS_EDEVICE, "parareal copy");
        if (hipEventRecord(fine_done[k & 1].ev[b], fs) != hipSuccess) return fail(ctx, MRS_EDEVICE, "parareal event");
        return MRS_OK;
    };
    // Fine groups of iteration kn are launched in slice order once their
    // start states are final and iteration kn is certain to run; next_a is
    // the first slice of the next group not launched yet.
    int next_a = 0;
    auto launch_ready = [&](int kn, int last_final) -> mrs_status {
        while (next_a <= ns && group_end(next_a) - 1 <= last_final) {
            const int b = group_end(next_a);
            mrs_status r = launch_group(kn, next_a, b);
            if (r != MRS_OK) return r;
            next_a = b + 1;
        }
        return MRS_OK;
    };

    // sweep 0: serial coarse sweep (Eq. initial); iteration 1 always runs
    States &I0 = It[0];
    if (copy_state(I0.X(0), I0.D(0), E->X.as<double>(), E->D.as<double>(), N, sc) != hipSuccess ||
        hipEventRecord(state_ready.ev[0], sc) != hipSuccess)
        return fail(ctx, MRS_EDEVICE, "parareal copy");
    next_a = 1;
    if ((st = launch_ready(1, 0)) != MRS_OK) return st;
    for (int n = 1; n <= ns; n++) {
        if ((st = S.coarse(I0.X(n - 1), I0.D(n - 1), n - 1, Gc[0].X(n), Gc[0].D(n), sc)) != MRS_OK)
            return st;
        if (copy_state(I0.X(n), I0.D(n), Gc[0].X(n), Gc[0].D(n), N, sc) != hipSuccess ||
            hipEventRecord(state_ready.ev[n], sc) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal copy");
        if ((st = launch_ready(1, n)) != MRS_OK) return st;
    }
    std::vector<double> ha((size_t)3 * N), hb((size_t)3 * N);
    int done = 0;
    bool finite_inc = true;
    for (int k = 1; k <= max_iter; k++) {
        States &V = It[k & 1];
        const States &U = It[(k - 1) & 1];
        const bool more = k + 1 <= max_iter;  // iteration k + 1 may run
        next_a = k + 1;
        // slices before k are converged; slice k takes its fine value
        for (int n = 0; n < k; n++)
            if (copy_state(V.X(n), V.D(n), U.X(n), U.D(n), N, sc) != hipSuccess)
                return fail(ctx, MRS_EDEVICE, "parareal copy");
        if (hipStreamWaitEvent(sc, fine_done[k & 1].ev[group_end(k)], 0) != hipSuccess ||
            copy_state(V.X(k), V.D(k), Fv[k & 1].X(k), Fv[k & 1].D(k), N, sc) != hipSuccess ||
            hipEventRecord(state_ready.ev[k], sc) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal copy");
        // relative increment (Eq. true_err, second form), accumulated slice by
        // slice; once it exceeds tol, iteration k + 1 is certain and its fine
        // groups start as their states become final
        double inc = 0.0;
        if ((st = S.increment(V.X(k), U.X(k), ha, hb, sc, &inc)) != MRS_OK) return st;
        if (more && inc > tol && (st = launch_ready(k + 1, k)) != MRS_OK) return st;
        // serial correction (Eq. serial_correct), each slice once its fine group is done
        for (int n = k + 1; n <= ns; n++) {
            if ((st = S.coarse(V.X(n - 1), V.D(n - 1), n - 1, Gc[k & 1].X(n), Gc[k & 1].D(n), sc)) != MRS_OK)
                return st;
            if (hipStreamWaitEvent(sc, fine_done[k & 1].ev[group_end(n)], 0) != hipSuccess)
                return fail(ctx, MRS_EDEVICE, "parareal wait");
            if ((st = S.correct(Fv[k & 1], Gc[k & 1], Gc[(k - 1) & 1], V, n, sc)) != MRS_OK) return st;
            if (hipEventRecord(state_ready.ev[n], sc) != hipSuccess)
                return fail(ctx, MRS_EDEVICE, "parareal event");
            if ((st = S.increment(V.X(n), U.X(n), ha, hb, sc, &inc)) != MRS_OK) return st;
            if (more && inc > tol && (st = launch_ready(k + 1, n)) != MRS_OK) return st;
        }
        if (history) history[k - 1] = inc;
        done = k;
        finite_inc = finite_inc && std::isfinite(inc);
        if (!(inc > tol)) break;
    }
    for (int i = 0; i < n_sf; i++)
        if (hipStreamSynchronize(sf[i]) != hipSuccess) return fail(ctx, MRS_EDEVICE, "parareal fine stream");
    if (iters) *iters = done;
    return S.finish(It[done & 1], sc, finite_inc);
}
