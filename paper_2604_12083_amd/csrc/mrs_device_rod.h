// Device code of the rod mechanics and of the element-wise step used by the
// kernels of mrs_kernels.hip: source records, rotations and the principal
// square root by quaternions (Sec. III.B.1, Eq. halfangle), the rod segment
// and node forces (Sec. II.B, Eqs. mid_triad, F_comp_discrete,
// N_comp_discrete, discrete_f, discrete_n; Alg. 1), and the step epilogue
// (Eqs. newx, newD; Sec. III.A).
#pragma once

#include <hip/hip_runtime.h>

#include "mrs_internal.h"

namespace mrs {

// The functions below are inlined into several kernels; with contraction off
// inside them, every kernel rounds each operation the same way, so the same
// inputs give the same bits whichever kernel evaluates them (explicit fma()
// calls stay fused).
#define FP_STRICT _Pragma("clang fp contract(off)")

// ------------------------------------------------------- source records

// FP32C position coordinate: x / eps split into hi + lo (the record form;
// the block descriptors take their boxes from the same split).
__device__ __forceinline__ void split_pos(double x, double inv_eps, float &h, float &l) {
    FP_STRICT;
    const double sx = x * inv_eps;
    h = (float)sx;
    l = (float)(sx - (double)h);
}

__device__ __forceinline__ RecF32 make_rec_f32(double x, double y, double z, double fx, double fy,
                                               double fz, double nx, double ny, double nz,
                                               double inv_eps) {
    FP_STRICT;
    float hx, hy, hz, lx, ly, lz;
    split_pos(x, inv_eps, hx, lx);
    split_pos(y, inv_eps, hy, ly);
    split_pos(z, inv_eps, hz, lz);
    const double ie2 = inv_eps * inv_eps;
    RecF32 r;
    r.a = make_float4(hx, hy, hz, (float)(fx * inv_eps));
    r.b = make_float4(lx, ly, lz, (float)(fy * inv_eps));
    r.c = make_float4((float)(fz * inv_eps), (float)(nx * ie2), (float)(ny * ie2), (float)(nz * ie2));
    return r;
}

__device__ __forceinline__ void store_rec(int prec, void *rec, int i, double x, double y, double z,
                                          double fx, double fy, double fz, double nx, double ny,
                                          double nz, double inv_eps) {
    FP_STRICT;
    if (prec == 1) {
        reinterpret_cast<RecF32 *>(rec)[i] = make_rec_f32(x, y, z, fx, fy, fz, nx, ny, nz, inv_eps);
    } else {
        RecF64 r;
        r.x = x; r.y = y; r.z = z;
        r.fx = fx; r.fy = fy; r.fz = fz;
        r.nx = nx; r.ny = ny; r.nz = nz;
        r.pad = 0.0;
        reinterpret_cast<RecF64 *>(rec)[i] = r;
    }
}

// ------------------------------------------------------------- rotations

// Unit quaternion (w, x, y, z), w >= 0, of a proper rotation A (row-major),
// by Shepperd's choice of the largest of 4w^2 = 1 + tr A, 4x^2 = 1 + A00 - A11
// - A22, and so on, which keeps the division well conditioned at every angle.
__device__ __forceinline__ void rot_to_quat(const double *A, double *q) {
    FP_STRICT;
    const double tr = A[0] + A[4] + A[8];
    double w, x, y, z;
    if (tr >= A[0] && tr >= A[4] && tr >= A[8]) {
        w = 0.5 * sqrt(1.0 + tr);
        const double s = 0.25 / w;
        x = (A[7] - A[5]) * s;
        y = (A[2] - A[6]) * s;
        z = (A[3] - A[1]) * s;
    } else if (A[0] >= A[4] && A[0] >= A[8]) {
        x = 0.5 * sqrt(fmax(1.0 + A[0] - A[4] - A[8], 0.0));
        const double s = 0.25 / x;
        w = (A[7] - A[5]) * s;
        y = (A[1] + A[3]) * s;
        z = (A[2] + A[6]) * s;
    } else if (A[4] >= A[8]) {
        y = 0.5 * sqrt(fmax(1.0 - A[0] + A[4] - A[8], 0.0));
        const double s = 0.25 / y;
        w = (A[2] - A[6]) * s;
        x = (A[1] + A[3]) * s;
        z = (A[5] + A[7]) * s;
    } else {
        z = 0.5 * sqrt(fmax(1.0 - A[0] - A[4] + A[8], 0.0));
        const double s = 0.25 / z;
        w = (A[3] - A[1]) * s;
        x = (A[2] + A[6]) * s;
        y = (A[5] + A[7]) * s;
    }
    if (w < 0.0) { w = -w; x = -x; y = -y; z = -z; }
    q[0] = w; q[1] = x; q[2] = y; q[3] = z;
}

// Quaternion of the principal square root: rotation by half the angle about
// the same axis, (1 + w, x, y, z) normalised.
__device__ __forceinline__ void quat_half(const double *q, double *h) {
    FP_STRICT;
    const double w = 1.0 + q[0];
    const double inv = 1.0 / sqrt(w * w + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    h[0] = w * inv; h[1] = q[1] * inv; h[2] = q[2] * inv; h[3] = q[3] * inv;
}

// v <- q v q*, for a unit quaternion q = (w, u): t = 2 u x v, v' = v + w t + u x t.
__device__ __forceinline__ void quat_rotate(const double *q, const double *v, double *o) {
    FP_STRICT;
    const double tx = 2.0 * (q[2] * v[2] - q[3] * v[1]);
    const double ty = 2.0 * (q[3] * v[0] - q[1] * v[2]);
    const double tz = 2.0 * (q[1] * v[1] - q[2] * v[0]);
    o[0] = v[0] + q[0] * tx + (q[2] * tz - q[3] * ty);
    o[1] = v[1] + q[0] * ty + (q[3] * tx - q[1] * tz);
    o[2] = v[2] + q[0] * tz + (q[1] * ty - q[2] * tx);
}

// Rotation quaternion of the rotation vector v (angle |v| about v/|v|).
__device__ __forceinline__ void quat_from_rotvec(double vx, double vy, double vz, double *q) {
    FP_STRICT;
    const double th = sqrt(vx * vx + vy * vy + vz * vz);
    double s, c;
    sincos(0.5 * th, &s, &c);
    const double k = th > 0.0 ? s / th : 0.5;
    q[0] = c; q[1] = k * vx; q[2] = k * vy; q[3] = k * vz;
}

__device__ __forceinline__ void quat_to_matrix(const double *q, double *S) {
    FP_STRICT;
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    S[0] = 1.0 - 2.0 * (y * y + z * z); S[1] = 2.0 * (x * y - w * z);       S[2] = 2.0 * (x * z + w * y);
    S[3] = 2.0 * (x * y + w * z);       S[4] = 1.0 - 2.0 * (x * x + z * z); S[5] = 2.0 * (y * z - w * x);
    S[6] = 2.0 * (x * z - w * y);       S[7] = 2.0 * (y * z + w * x);       S[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Frame re-orthonormalisation: D3 <- D3/|D3|, D1 <- unit(D1 - (D1.D3) D3), D2 <- D3 x D1.
__device__ __forceinline__ void reorthonormalize(double *d) {
    FP_STRICT;
    double *d1 = d, *d2 = d + 3, *d3 = d + 6;
    const double i3 = 1.0 / sqrt(d3[0] * d3[0] + d3[1] * d3[1] + d3[2] * d3[2]);
    d3[0] *= i3; d3[1] *= i3; d3[2] *= i3;
    const double p = d1[0] * d3[0] + d1[1] * d3[1] + d1[2] * d3[2];
    d1[0] -= p * d3[0]; d1[1] -= p * d3[1]; d1[2] -= p * d3[2];
    const double i1 = 1.0 / sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);
    d1[0] *= i1; d1[1] *= i1; d1[2] *= i1;
    d2[0] = d3[1] * d1[2] - d3[2] * d1[1];
    d2[1] = d3[2] * d1[0] - d3[0] * d1[2];
    d2[2] = d3[0] * d1[1] - d3[1] * d1[0];
}

// Explicit Runge-Kutta schemes whose stage s + 1 depends on stage s only:
// weights w_s and the node c_{s+1} of the next stage.  Scheme 0 is the
// classical RK4, scheme 1 the midpoint RK2.
static __constant__ double kRkWeight[2][4] = {{1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0}, {0.0, 1.0, 0.0, 0.0}};
static __constant__ double kRkNextNode[2][3] = {{0.5, 0.5, 1.0}, {0.5, 0.0, 0.0}};

// Preferred strain-twist of a segment at arclength s and time t: the
// intrinsic vector plus, for a swimmer, (0, -k^2 A sin(k s + f t), 0)
// (Sec. IV).
__device__ __forceinline__ void preferred_strain(const EnsDesc &E, double s, double t, double *om) {
    FP_STRICT;
    om[0] = E.om0[0];
    om[1] = E.om0[1];
    om[2] = E.om0[2];
    if (E.has_wave) om[1] += -E.wave[1] * E.wave[1] * E.wave[0] * sin(E.wave[1] * s + E.wave[2] * t);
}

// F and N of the segment between nodes ka and kb = ka + 1 (SoA state of N
// points) at arclength s_mid (its midpoint) and time t.
__device__ __forceinline__ void rod_segment(const EnsDesc &E, const double *__restrict__ X,
                                            const double *__restrict__ D, int N, int ka, int kb,
                                            double s_mid, double t, double *F, double *Nv, double *dX) {
    FP_STRICT;
    double Da[9], Db[9];
#pragma unroll
    for (int k = 0; k < 9; k++) {
        Da[k] = D[(size_t)k * N + ka];
        Db[k] = D[(size_t)k * N + kb];
    }
    // A = sum_j D^j_b (D^j_a)^T maps frame a onto frame b.
    double A[9];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++)
            A[3 * r + c] = Db[r] * Da[c] + Db[3 + r] * Da[3 + c] + Db[6 + r] * Da[6 + c];
    double q[4], h[4], Dh[9];
    rot_to_quat(A, q);
    quat_half(q, h);
#pragma unroll
    for (int i = 0; i < 3; i++) quat_rotate(h, Da + 3 * i, Dh + 3 * i);
#pragma unroll
    for (int c = 0; c < 3; c++) dX[c] = X[(size_t)c * N + kb] - X[(size_t)c * N + ka];
    const double ids = 1.0 / E.ds;
    F[0] = F[1] = F[2] = 0.0;
    Nv[0] = Nv[1] = Nv[2] = 0.0;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const double str = (dX[0] * Dh[3 * j] + dX[1] * Dh[3 * j + 1] + dX[2] * Dh[3 * j + 2]) * ids -
                           (j == 2 ? 1.0 : 0.0);
        const double Fj = E.b[j] * str;
        F[0] += Fj * Dh[3 * j]; F[1] += Fj * Dh[3 * j + 1]; F[2] += Fj * Dh[3 * j + 2];
    }
    double om[3];
    preferred_strain(E, s_mid, t, om);
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int j = (i + 1) % 3, l = (i + 2) % 3;
        const double kap = ((Db[3 * j] - Da[3 * j]) * Dh[3 * l] + (Db[3 * j + 1] - Da[3 * j + 1]) * Dh[3 * l + 1] +
                            (Db[3 * j + 2] - Da[3 * j + 2]) * Dh[3 * l + 2]) * ids - om[i];
        const double Ni = E.a[i] * kap;
        Nv[0] += Ni * Dh[3 * i]; Nv[1] += Ni * Dh[3 * i + 1]; Nv[2] += Ni * Dh[3 * i + 2];
    }
}

// Rod forces of one filament (nodes k0 .. k0 + M - 1 of an SoA state of N
// points; Sec. II.B, Alg. 1): for every node, the point force and torque on
// the fluid, g = F_{k+1/2} - F_{k-1/2} + external, m = N_{k+1/2} - N_{k-1/2}
// + (dX_{k+1/2} x F_{k+1/2} + dX_{k-1/2} x F_{k-1/2}) / 2 + external, written
// as source records into rec[point].  BLOCK threads walk the filament in
// chunks of BLOCK - 1 nodes: thread t computes segment c0 - 1 + t into LDS,
// then node c0 + t combines its two neighbouring segments (a node's result
// does not depend on the chunking).  Every thread of the block must call it.
template <int BLOCK>
__device__ __forceinline__ void rod_filament(int prec, int stage_state, int elastic, int scheme, int stage,
                                             double dt, const EnsDesc &E, int fil, void *rec) {
    FP_STRICT;
    __shared__ double sF[3][BLOCK], sN[3][BLOCK], sX[3][BLOCK];
    const int N = E.N;
    const double *__restrict__ X = stage_state ? E.Xs : E.X;
    const double *__restrict__ D = stage_state ? E.Ds : E.D;
    const int k0 = E.off[fil];
    const int M = E.off[fil + 1] - k0;
    const int tid = threadIdx.x;
    if (elastic < 0) elastic = E.elastic;
    // waveform time of this stage: step start + c_stage dt
    double t = 0.0;
    if (E.has_wave) {
        if (dt != dt) dt = E.dt;
        t = *E.clock + (stage > 0 ? kRkNextNode[scheme][stage - 1] : 0.0) * dt;
    }
    for (int c0 = 0; c0 < M; c0 += BLOCK - 1) {
        // this thread's node: its external loads and position, loaded before
        // the segment work so that the two memory latencies overlap
        const int k = c0 + tid;
        const bool node = tid < BLOCK - 1 && k < M;
        const int p = k0 + (node ? k : 0);
        double g[3] = {0.0, 0.0, 0.0}, m[3] = {0.0, 0.0, 0.0}, xp[3] = {0.0, 0.0, 0.0};
        if (node) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                if (E.fext) g[c] = E.fext[(size_t)c * N + p];
                if (E.next) m[c] = E.next[(size_t)c * N + p];
                if (E.has_lj) g[c] += E.flj[(size_t)c * N + p];
                xp[c] = X[(size_t)c * N + p];
            }
        }
        if (elastic) {
            const int s = c0 - 1 + tid;
            double F[3] = {0.0, 0.0, 0.0}, Nv[3] = {0.0, 0.0, 0.0}, dX[3] = {0.0, 0.0, 0.0};
            if (s >= 0 && s <= M - 2)
                rod_segment(E, X, D, N, k0 + s, k0 + s + 1, (s + 0.5) * E.ds, t, F, Nv, dX);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                sF[c][tid] = F[c];
                sN[c][tid] = Nv[c];
                sX[c][tid] = dX[c];
            }
            __syncthreads();
        }
        if (node) {
            if (elastic) {
                // segment k+1/2 sits at LDS slot tid + 1, segment k-1/2 at slot tid
                const double Fp[3] = {sF[0][tid + 1], sF[1][tid + 1], sF[2][tid + 1]};
                const double Fm[3] = {sF[0][tid], sF[1][tid], sF[2][tid]};
                const double Xp[3] = {sX[0][tid + 1], sX[1][tid + 1], sX[2][tid + 1]};
                const double Xm[3] = {sX[0][tid], sX[1][tid], sX[2][tid]};
                const double cp[3] = {Xp[1] * Fp[2] - Xp[2] * Fp[1], Xp[2] * Fp[0] - Xp[0] * Fp[2],
                                      Xp[0] * Fp[1] - Xp[1] * Fp[0]};
                const double cm[3] = {Xm[1] * Fm[2] - Xm[2] * Fm[1], Xm[2] * Fm[0] - Xm[0] * Fm[2],
                                      Xm[0] * Fm[1] - Xm[1] * Fm[0]};
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    g[c] += Fp[c] - Fm[c];
                    m[c] += (sN[c][tid + 1] - sN[c][tid]) + 0.5 * (cp[c] + cm[c]);
                }
            }
            store_rec(prec, rec, p, xp[0], xp[1], xp[2], g[0], g[1], g[2], m[0], m[1], m[2], E.inv_eps);
            if (E.g_out) {
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    E.g_out[3 * (size_t)p + c] = g[c];
                    E.m_out[3 * (size_t)p + c] = m[c];
                }
            }
        }
        if (elastic) __syncthreads();
    }
}

__device__ __forceinline__ void rotate_frame(const double *din, double *__restrict__ Dout, int N, int i,
                                             double vx, double vy, double vz, bool reorth) {
    FP_STRICT;
    double q[4], d[9];
    quat_from_rotvec(vx, vy, vz, q);
#pragma unroll
    for (int k = 0; k < 3; k++) quat_rotate(q, din + 3 * k, d + 3 * k);
    if (reorth) reorthonormalize(d);
#pragma unroll
    for (int k = 0; k < 9; k++) Dout[(size_t)k * N + i] = d[k];
}

// Raises the ensemble's non-finite flag when any of v[0..n) is not finite
// (an ordinary vector store from the lanes that see one).
__device__ __forceinline__ void check_finite(const EnsDesc &E, const double *v, int n) {
    bool ok = true;
    for (int k = 0; k < n; k++) ok = ok && isfinite(v[k]);
    if (!ok && E.nonfinite) *E.nonfinite = 1;
}


// Epilogue of point i once its split-K sum acc (6 values, before scaling)
// is known: U = cU acc[0..2], Omega = cW acc[3..5], the non-finite check, and
// the element-wise part of the step (Eqs. newx, newD): EPI_WRITE stores U,
// Omega; EPI_EULER also moves X += dt U and rotates the frame by dt Omega
// (re-orthonormalised); EPI_RK_STAGE accumulates the weighted stage sums and
// builds the next stage state from the step-start state (xv, dv); EPI_RK_FINAL
// finishes the step from the weighted sums (uav, wav: the sums so far).
//
// Frames under RK4 follow Runge-Kutta-Munthe-Kaas: stage s's frame is
// exp(theta_s) D with theta_s = c_s dt k_{s-1}, and the angular velocity
// Omega found there enters the stage sums and the next stage frame as
// k_s = dexp^{-1}_{theta_s}(Omega) = Omega - theta_s x Omega / 2 +
// theta_s x (theta_s x Omega) / 12 (the series of the inverse derivative of
// the exponential map on so(3), cut after the terms a fourth-order method
// needs; k_0 = Omega).  kv holds k_{s-1} (stage > 0); E.Ks receives k_s.
// RK2 (midpoint) needs no correction for its order and uses Omega as is.
template <int EPI>
__device__ __forceinline__ void epilogue_point(const EnsDesc &E, int N, int i, const double *acc, const double *xv,
                                               const double *dv, const double *uav, const double *wav,
                                               const double *kv, int stage, int scheme, double dt) {
    FP_STRICT;
    const double U[3] = {acc[0] * E.cU, acc[1] * E.cU, acc[2] * E.cU};
    const double W[3] = {acc[3] * E.cW, acc[4] * E.cW, acc[5] * E.cW};
    const double UW[6] = {U[0], U[1], U[2], W[0], W[1], W[2]};
    check_finite(E, UW, 6);
    if (EPI == EPI_WRITE) {
        if (E.aos_io) {
#pragma unroll
            for (int c = 0; c < 3; c++) { E.U[3 * (size_t)i + c] = U[c]; E.W[3 * (size_t)i + c] = W[c]; }
        } else {
#pragma unroll
            for (int c = 0; c < 3; c++) { E.U[(size_t)c * N + i] = U[c]; E.W[(size_t)c * N + i] = W[c]; }
        }
        return;
    }
    if (EPI == EPI_EULER) {
        double xn[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            xn[c] = xv[c] + dt * U[c];
            E.U[(size_t)c * N + i] = U[c];
            E.W[(size_t)c * N + i] = W[c];
            E.X[(size_t)c * N + i] = xn[c];
        }
        check_finite(E, xn, 3);
        rotate_frame(dv, E.D, N, i, dt * W[0], dt * W[1], dt * W[2], true);
        return;
    }
    // Runge-Kutta stage `stage` of `scheme`, evaluated at the stage state.
    const double wgt = kRkWeight[scheme][stage];
    double k[3] = {W[0], W[1], W[2]};
    if (scheme == 0 && stage > 0) {
        const double c_dt = kRkNextNode[scheme][stage - 1] * dt;
        const double th[3] = {c_dt * kv[0], c_dt * kv[1], c_dt * kv[2]};
        const double t1[3] = {th[1] * W[2] - th[2] * W[1], th[2] * W[0] - th[0] * W[2], th[0] * W[1] - th[1] * W[0]};
        const double t2[3] = {th[1] * t1[2] - th[2] * t1[1], th[2] * t1[0] - th[0] * t1[2],
                              th[0] * t1[1] - th[1] * t1[0]};
#pragma unroll
        for (int c = 0; c < 3; c++) k[c] = W[c] - 0.5 * t1[c] + t2[c] / 12.0;
    }
    double ua[3], wa[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (stage == 0) {
            E.U[(size_t)c * N + i] = U[c];
            E.W[(size_t)c * N + i] = W[c];
            ua[c] = wgt * U[c];
            wa[c] = wgt * k[c];
        } else {
            ua[c] = uav[c] + wgt * U[c];
            wa[c] = wav[c] + wgt * k[c];
        }
    }
    if (EPI == EPI_RK_STAGE) {
        const double h = kRkNextNode[scheme][stage] * dt;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            E.Ua[(size_t)c * N + i] = ua[c];
            E.Wa[(size_t)c * N + i] = wa[c];
            E.Xs[(size_t)c * N + i] = xv[c] + h * U[c];
            if (scheme == 0) E.Ks[(size_t)c * N + i] = k[c];
        }
        rotate_frame(dv, E.Ds, N, i, h * k[0], h * k[1], h * k[2], false);
    } else {
        double xn[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            xn[c] = xv[c] + dt * ua[c];
            E.X[(size_t)c * N + i] = xn[c];
        }
        check_finite(E, xn, 3);
        rotate_frame(dv, E.D, N, i, dt * wa[0], dt * wa[1], dt * wa[2], true);
    }
}

}  // namespace mrs

#undef FP_STRICT
