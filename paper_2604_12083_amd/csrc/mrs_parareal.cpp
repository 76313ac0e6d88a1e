// Parareal (Sec. II.D) on one device: the fine propagations of all slices of
// an iteration run as one batched launch sequence; the coarse sweep and the
// correction of Eq. serial_correct run on the device; slice-boundary states
// stay resident.
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

}  // namespace

extern "C" mrs_status mrs_parareal(mrs_ensemble *E, int32_t ns, mrs_integrator fi, double fdt, int32_t fsteps,
                                   int32_t csteps, int32_t max_iter, double tol, mrs_precision prec,
                                   int include_elastic, double *history, int32_t *iters) {
    if (!E) return MRS_EINVAL;
    mrs_context *ctx = E->ctx;
    if (ns < 1 || fsteps < 1 || csteps < 1 || max_iter < 1 || max_iter > ns)
        return fail(ctx, MRS_EINVAL, "need n_slices, fine_steps, coarse_steps >= 1 and 1 <= max_iter <= n_slices");
    if (!std::isfinite(fdt) || !std::isfinite(tol) || tol < 0.0) return fail(ctx, MRS_EINVAL, "bad dt or tol");
    if (fi != MRS_EULER && fi != MRS_RK2 && fi != MRS_RK4) return fail(ctx, MRS_EINVAL, "unknown integrator");
    if (prec != MRS_FP64 && prec != MRS_FP32C) return fail(ctx, MRS_EINVAL, "unknown precision");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    hipStream_t s = ctx->stream;
    const int64_t N = E->N;
    const double cdt = fdt * fsteps / csteps;
    const int el = include_elastic ? 1 : 0;

    // U: current iterate, V: next iterate, Go / Gn: coarse values, Fv: fine values
    States U, V, Go, Gn, Fv;
    for (States *st : {&U, &V, &Go, &Gn, &Fv}) {
        st->N = N;
        if (st->buf.reserve((size_t)(ns + 1) * 12 * N * sizeof(double)) != hipSuccess)
            return fail(ctx, MRS_ENOMEM, "parareal state buffers");
    }
    std::vector<mrs_ensemble *> W(ns + 1, nullptr);  // W[n]: fine worker of slice n; W[0]: coarse worker
    mrs_status st = MRS_OK;
    auto cleanup = [&]() {
        for (auto *w : W)
            if (w) mrs_ensemble_destroy(w);
    };
    for (int n = 0; n <= ns && st == MRS_OK; n++) st = ensemble_clone(E, &W[n]);
    if (st != MRS_OK) {
        cleanup();
        return st;
    }
    mrs_ensemble *C = W[0];
    // slice boundary times T[n], accumulated step by step exactly as the
    // device clock of a serial fine run accumulates them
    std::vector<double> T(ns + 1);
    if (hipMemcpy(&T[0], E->clock.p, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
        cleanup();
        return fail(ctx, MRS_EDEVICE, "parareal clock read");
    }
    for (int n = 1; n <= ns; n++) {
        T[n] = T[n - 1];
        for (int k = 0; k < fsteps; k++) T[n] += fdt;
    }
    auto set_clock = [&](mrs_ensemble *w, int n) {
        return hipMemcpyAsync(w->clock.p, &T[n], sizeof(double), hipMemcpyHostToDevice, s);
    };
    auto coarse = [&](const double *X, const double *D, int n0, double *oX, double *oD) -> mrs_status {
        if (copy_state(C->X.as<double>(), C->D.as<double>(), X, D, N, s) != hipSuccess ||
            set_clock(C, n0) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal copy");
        mrs_status r = mrs_ensemble_step(C, MRS_EULER, cdt, csteps, prec, el);
        if (r != MRS_OK) return r;
        if (copy_state(oX, oD, C->X.as<double>(), C->D.as<double>(), N, s) != hipSuccess)
            return fail(ctx, MRS_EDEVICE, "parareal copy");
        return MRS_OK;
    };

    // iteration 0: serial coarse sweep (Eq. initial)
    if (copy_state(U.X(0), U.D(0), E->X.as<double>(), E->D.as<double>(), N, s) != hipSuccess) {
        cleanup();
        return fail(ctx, MRS_EDEVICE, "parareal copy");
    }
    for (int n = 1; n <= ns && st == MRS_OK; n++) {
        st = coarse(U.X(n - 1), U.D(n - 1), n - 1, Go.X(n), Go.D(n));
        if (st == MRS_OK && copy_state(U.X(n), U.D(n), Go.X(n), Go.D(n), N, s) != hipSuccess)
            st = fail(ctx, MRS_EDEVICE, "parareal copy");
    }
    std::vector<double> ha((size_t)3 * N), hb((size_t)3 * N);
    int done = 0;
    for (int k = 1; k <= max_iter && st == MRS_OK; k++) {
        // fine propagations of slices k..ns from the previous iterate, batched (Eq. intermediate)
        std::vector<mrs_ensemble *> batch;
        for (int n = k; n <= ns; n++) {
            if (copy_state(W[n]->X.as<double>(), W[n]->D.as<double>(), U.X(n - 1), U.D(n - 1), N, s) != hipSuccess ||
                set_clock(W[n], n - 1) != hipSuccess) {
                st = fail(ctx, MRS_EDEVICE, "parareal copy");
                break;
            }
            batch.push_back(W[n]);
        }
        if (st != MRS_OK) break;
        st = mrs_batch_step(ctx, (int32_t)batch.size(), batch.data(), fi, fdt, fsteps, prec, el, 1);
        if (st != MRS_OK) break;
        for (int n = k; n <= ns; n++)
            if (copy_state(Fv.X(n), Fv.D(n), W[n]->X.as<double>(), W[n]->D.as<double>(), N, s) != hipSuccess)
                st = fail(ctx, MRS_EDEVICE, "parareal copy");
        // slices before k are converged; slice k takes its fine value
        for (int n = 0; n < k && st == MRS_OK; n++)
            if (copy_state(V.X(n), V.D(n), U.X(n), U.D(n), N, s) != hipSuccess) st = fail(ctx, MRS_EDEVICE, "copy");
        if (st == MRS_OK && copy_state(V.X(k), V.D(k), Fv.X(k), Fv.D(k), N, s) != hipSuccess)
            st = fail(ctx, MRS_EDEVICE, "parareal copy");
        for (int n = 1; n <= k && st == MRS_OK; n++)
            if (copy_state(Gn.X(n), Gn.D(n), Go.X(n), Go.D(n), N, s) != hipSuccess) st = fail(ctx, MRS_EDEVICE, "copy");
        // serial correction (Eq. serial_correct)
        for (int n = k + 1; n <= ns && st == MRS_OK; n++) {
            st = coarse(V.X(n - 1), V.D(n - 1), n - 1, Gn.X(n), Gn.D(n));
            if (st != MRS_OK) break;
            hipError_t he = timed(ctx, "parareal_correct", s, [&] {
                return launch_parareal_correct((int)N, Fv.X(n), Fv.D(n), Gn.X(n), Gn.D(n), Go.X(n), Go.D(n), V.X(n),
                                               V.D(n), s);
            });
            if (he != hipSuccess) st = fail(ctx, MRS_EDEVICE, "parareal correction: %s", hipGetErrorString(he));
        }
        if (st != MRS_OK) break;
        // relative increment over the slice boundaries that changed (Eq. true_err, second form)
        double inc = 0.0;
        for (int n = k; n <= ns && st == MRS_OK; n++) {
            if (hipMemcpyAsync(ha.data(), V.X(n), ha.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(hb.data(), U.X(n), hb.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = fail(ctx, MRS_EDEVICE, "parareal increment copy");
                break;
            }
            inc = std::max(inc, rel_increment(ha, hb, N));
        }
        if (st != MRS_OK) break;
        std::swap(U.buf.p, V.buf.p);
        std::swap(U.buf.bytes, V.buf.bytes);
        std::swap(Go.buf.p, Gn.buf.p);
        std::swap(Go.buf.bytes, Gn.buf.bytes);
        if (history) history[k - 1] = inc;
        done = k;
        if (!(inc > tol)) break;
    }
    if (st == MRS_OK) {
        if (copy_state(E->X.as<double>(), E->D.as<double>(), U.X(ns), U.D(ns), N, s) != hipSuccess ||
            set_clock(E, ns) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            st = fail(ctx, MRS_EDEVICE, "parareal result copy");
    }
    if (iters) *iters = done;
    cleanup();
    return st;
}
