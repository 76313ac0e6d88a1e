// HIP kernels (gfx950) of the MRS filament path other than the pair sum.
//
//   k_pack_aos        n x 3 caller arrays -> source records
//   k_rod_forces      per segment: A = sum_j D^j_{k+1} (D^j_k)^T, its principal
//                     square root, mid frame, F and N (Sec. II.B, Eqs.
//                     mid_triad, F_comp_discrete, N_comp_discrete; Alg. 1);
//                     per node: the point force and torque on the fluid
//                     (Eqs. discrete_f, discrete_n) written straight into the
//                     pair kernel's source records
//   k_reduce<EPI>     fixed-order FP64 sum of the split-K partials, scaling,
//                     and the element-wise step epilogue (Eqs. newx, newD)
//   k_parareal_correct  Parareal correction of one slice boundary
//   k_rotsqrt         batched principal 3x3 rotation square root
//
// Source records: FP32C positions in units of eps (rho = x/eps) split
// hi + lo, forces f/eps and torques n/eps^2; FP64 records hold x, f, n.
#include <hip/hip_runtime.h>

#include "mrs_internal.h"

namespace mrs {

// ------------------------------------------------------- source records

__device__ __forceinline__ RecF32 make_rec_f32(double x, double y, double z, double fx, double fy,
                                               double fz, double nx, double ny, double nz,
                                               double inv_eps) {
    const double sx = x * inv_eps, sy = y * inv_eps, sz = z * inv_eps;
    const float hx = (float)sx, hy = (float)sy, hz = (float)sz;
    const float lx = (float)(sx - (double)hx), ly = (float)(sy - (double)hy), lz = (float)(sz - (double)hz);
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
    const double w = 1.0 + q[0];
    const double inv = 1.0 / sqrt(w * w + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    h[0] = w * inv; h[1] = q[1] * inv; h[2] = q[2] * inv; h[3] = q[3] * inv;
}

// v <- q v q*, for a unit quaternion q = (w, u): t = 2 u x v, v' = v + w t + u x t.
__device__ __forceinline__ void quat_rotate(const double *q, const double *v, double *o) {
    const double tx = 2.0 * (q[2] * v[2] - q[3] * v[1]);
    const double ty = 2.0 * (q[3] * v[0] - q[1] * v[2]);
    const double tz = 2.0 * (q[1] * v[1] - q[2] * v[0]);
    o[0] = v[0] + q[0] * tx + (q[2] * tz - q[3] * ty);
    o[1] = v[1] + q[0] * ty + (q[3] * tx - q[1] * tz);
    o[2] = v[2] + q[0] * tz + (q[1] * ty - q[2] * tx);
}

// Rotation quaternion of the rotation vector v (angle |v| about v/|v|).
__device__ __forceinline__ void quat_from_rotvec(double vx, double vy, double vz, double *q) {
    const double th = sqrt(vx * vx + vy * vy + vz * vz);
    double s, c;
    sincos(0.5 * th, &s, &c);
    const double k = th > 0.0 ? s / th : 0.5;
    q[0] = c; q[1] = k * vx; q[2] = k * vy; q[3] = k * vz;
}

__device__ __forceinline__ void quat_to_matrix(const double *q, double *S) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    S[0] = 1.0 - 2.0 * (y * y + z * z); S[1] = 2.0 * (x * y - w * z);       S[2] = 2.0 * (x * z + w * y);
    S[3] = 2.0 * (x * y + w * z);       S[4] = 1.0 - 2.0 * (x * x + z * z); S[5] = 2.0 * (y * z - w * x);
    S[6] = 2.0 * (x * z - w * y);       S[7] = 2.0 * (y * z + w * x);       S[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Frame re-orthonormalisation: D3 <- D3/|D3|, D1 <- unit(D1 - (D1.D3) D3), D2 <- D3 x D1.
__device__ __forceinline__ void reorthonormalize(double *d) {
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

__global__ __launch_bounds__(kBlock) void k_rotsqrt(int64_t count, const double *__restrict__ R,
                                                    double *__restrict__ S) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    double A[9], q[4], h[4], o[9];
    for (int k = 0; k < 9; k++) A[k] = R[9 * i + k];
    rot_to_quat(A, q);
    quat_half(q, h);
    quat_to_matrix(h, o);
    for (int k = 0; k < 9; k++) S[9 * i + k] = o[k];
}

// ------------------------------------------------------------ pack / rod

__global__ __launch_bounds__(kBlock) void k_pack_aos(int prec, const EnsDesc *__restrict__ desc) {
    const EnsDesc &E = desc[0];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= E.N) return;
    const double *X = E.Xin_aos, *f = E.fext, *n = E.next;
    store_rec(prec, E.rec, i, X[3 * i], X[3 * i + 1], X[3 * i + 2], f[3 * i], f[3 * i + 1],
              f[3 * i + 2], n[3 * i], n[3 * i + 1], n[3 * i + 2], E.inv_eps);
}

// F and N of the segment between nodes ka and kb = ka + 1 (SoA state of N points).
// Explicit Runge-Kutta schemes whose stage s + 1 depends on stage s only:
// weights w_s and the node c_{s+1} of the next stage.  Scheme 0 is the
// classical RK4, scheme 1 the midpoint RK2.
__constant__ double kRkWeight[2][4] = {{1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0}, {0.0, 1.0, 0.0, 0.0}};
__constant__ double kRkNextNode[2][3] = {{0.5, 0.5, 1.0}, {0.5, 0.0, 0.0}};

// Preferred strain-twist of a segment at arclength s and time t: the
// intrinsic vector plus, for a swimmer, (0, -k^2 A sin(k s + f t), 0)
// (Sec. IV).
__device__ __forceinline__ void preferred_strain(const EnsDesc &E, double s, double t, double *om) {
    om[0] = E.om0[0];
    om[1] = E.om0[1];
    om[2] = E.om0[2];
    if (E.has_wave) om[1] += -E.wave[1] * E.wave[1] * E.wave[0] * sin(E.wave[1] * s + E.wave[2] * t);
}

// Segment ka -> kb = ka + 1 at arclength s_mid (its midpoint) and time t.
__device__ __forceinline__ void rod_segment(const EnsDesc &E, const double *__restrict__ X,
                                            const double *__restrict__ D, int N, int ka, int kb,
                                            double s_mid, double t, double *F, double *Nv, double *dX) {
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

// One block per filament; the filament is walked in chunks of kBlock - 1
// nodes.  Thread t computes segment c0 - 1 + t into LDS, then node c0 + t
// combines its two neighbouring segments.
__global__ __launch_bounds__(kBlock) void k_rod_forces(int prec, int stage_state, int elastic, int scheme,
                                                       int stage, double dt, const EnsDesc *__restrict__ desc,
                                                       const RodItem *__restrict__ items) {
    __shared__ double sF[3][kBlock], sN[3][kBlock], sX[3][kBlock];
    const RodItem it = items[blockIdx.x];
    const EnsDesc &E = desc[it.ens];
    const int N = E.N;
    const double *__restrict__ X = stage_state ? E.Xs : E.X;
    const double *__restrict__ D = stage_state ? E.Ds : E.D;
    const int k0 = E.off[it.fil];
    const int M = E.off[it.fil + 1] - k0;
    const int tid = threadIdx.x;
    if (elastic < 0) elastic = E.elastic;
    // waveform time of this stage: step start + c_stage dt
    double t = 0.0;
    if (E.has_wave) {
        if (dt != dt) dt = E.dt;
        t = *E.clock + (stage > 0 ? kRkNextNode[scheme][stage - 1] : 0.0) * dt;
    }
    for (int c0 = 0; c0 < M; c0 += kBlock - 1) {
        // this thread's node: its external loads and position, loaded before
        // the segment work so that the two memory latencies overlap
        const int k = c0 + tid;
        const bool node = tid < kBlock - 1 && k < M;
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
            store_rec(prec, E.rec, p, xp[0], xp[1], xp[2], g[0], g[1], g[2], m[0], m[1], m[2], E.inv_eps);
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

// ------------------------------------------------------------ Lennard-Jones

__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

static_assert(kLjBlockPoints <= 64, "an LJ source block fits one wave, one point per lane");

// Value of v in lane l (l wave-uniform), read into scalar registers.
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Box of every LJ source block (at most kLjBlockPoints consecutive points of
// one filament) of the (stage) positions: one wave per block.
__global__ __launch_bounds__(kBlock) void k_lj_boxes(int stage_state, const EnsDesc *__restrict__ desc,
                                                     const PointItem *__restrict__ items) {
    const PointItem it = items[blockIdx.x];
    const EnsDesc &E = desc[it.ens];
    const int b = it.p0 + (int)(threadIdx.x >> 6);
    if (b >= E.n_ljblk) return;  // wave-uniform
    const int N = E.N;
    const double *__restrict__ X = stage_state ? E.Xs : E.X;
    const int k = E.lj_blk[3 * b] + (int)(threadIdx.x & 63);
    const bool real = k < E.lj_blk[3 * b + 1];
    double lo[3], hi[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const double v = real ? X[(size_t)c * N + k] : 0.0;
        lo[c] = wave_min_d(real ? v : INFINITY);
        hi[c] = wave_max_d(real ? v : -INFINITY);
    }
    if ((threadIdx.x & 63) == 0) {
        double *bx = E.lj_box + 6 * (size_t)b;
#pragma unroll
        for (int c = 0; c < 3; c++) { bx[c] = lo[c]; bx[3 + c] = hi[c]; }
    }
}

// Lennard-Jones force on every point (Sec. IV): the sum over points of other
// filaments closer than r_c of 24 e (2 (sig/r)^12 - (sig/r)^6) (x_i - x_j)/r^2.
// A block owns 64 points (one per lane); its kLjWaves waves split the LJ
// source blocks (wave w takes every kLjWaves-th staged box), visit a block
// only when one of their lanes lies within r_c of its box, and their partial
// forces are added in wave order.  Sixteen waves keep the chain of boxes a
// wave visits short when there are few target blocks (25 swimmers of 51
// points: 20 blocks).  The block also writes the LJ mask of its 64 points: the
// FP32C pair kernels evaluate those sources in FP64, since the equal and
// opposite contact forces largely cancel at a distance and FP32 terms would
// leave their rounding behind.
constexpr int kLjWaves = 16;
constexpr int kLjStage = 256;  // LJ source-block boxes staged in LDS per pass

__global__ __launch_bounds__(64 * kLjWaves) void k_lj_forces(int stage_state, const EnsDesc *__restrict__ desc,
                                                             const PointItem *__restrict__ items) {
    constexpr int kWaves = kLjWaves;
    __shared__ double sBox[kLjStage][6];
    __shared__ int sBlk[kLjStage][3];
    __shared__ double sPart[kWaves][3][64];
    const PointItem it = items[blockIdx.x];
    const EnsDesc &E = desc[it.ens];
    const int N = E.N;
    const double *__restrict__ X = stage_state ? E.Xs : E.X;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i = it.p0 + lane;
    const bool real = i < N;
    const int ii = real ? i : N - 1;
    const double x0 = X[ii], x1 = X[(size_t)N + ii], x2 = X[2 * (size_t)N + ii];
    const int fi = E.fil[ii];
    const double rc = E.lj_rc, rc2 = rc * rc, sig2 = E.lj_sig * E.lj_sig, c24 = 24.0 * E.lj_e;
    double acc[3] = {0.0, 0.0, 0.0};
    const int nblk = E.n_ljblk;
    for (int b0 = 0; b0 < nblk; b0 += kLjStage) {
        __syncthreads();
        if (tid < kLjStage && b0 + tid < nblk) {
#pragma unroll
            for (int c = 0; c < 6; c++) sBox[tid][c] = E.lj_box[6 * (size_t)(b0 + tid) + c];
#pragma unroll
            for (int c = 0; c < 3; c++) sBlk[tid][c] = E.lj_blk[3 * (b0 + tid) + c];
        }
        __syncthreads();
        const int cnt = min(kLjStage, nblk - b0);
        for (int bb = w; bb < cnt; bb += kWaves) {
            double gap2 = 0.0;
            const double xs[3] = {x0, x1, x2};
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const double g = fmax(0.0, fmax(sBox[bb][c] - xs[c], xs[c] - sBox[bb][3 + c]));
                gap2 += g * g;
            }
            const bool near = real && gap2 < rc2 && sBlk[bb][2] != fi;
            if (!__any(near ? 1 : 0)) continue;  // wave-uniform
            // the wave loads the block's points once (lane = point, coalesced)
            // and broadcasts them from lane registers: no dependent global
            // load per source point
            const int j0 = sBlk[bb][0], jn = sBlk[bb][1] - j0;  // jn <= kLjBlockPoints = 64
            double y0 = 0.0, y1 = 0.0, y2 = 0.0;
            if (lane < jn) {
                y0 = X[j0 + lane];
                y1 = X[(size_t)N + j0 + lane];
                y2 = X[2 * (size_t)N + j0 + lane];
            }
            // r < r_c is tested as r^2 < r_c^2 and 1/r^2 is one reciprocal
            // refined twice (the force vanishes at r_c = 2^(1/6) sigma, so a
            // decision that differs from r < r_c by a rounding changes no
            // force); four sources per iteration keep independent chains in
            // flight
#pragma unroll 4
            for (int jj = 0; jj < jn; jj++) {
                const double r0 = x0 - readlane_d(y0, jj), r1 = x1 - readlane_d(y1, jj), r2 = x2 - readlane_d(y2, jj);
                const double rr2 = fma(r2, r2, fma(r1, r1, r0 * r0));
                if (!near || !(rr2 < rc2)) continue;
                double inv = __builtin_amdgcn_rcp(rr2);
                inv = fma(inv, fma(-rr2, inv, 1.0), inv);
                inv = fma(inv, fma(-rr2, inv, 1.0), inv);
                const double s2 = sig2 * inv, s6 = s2 * s2 * s2;
                const double cf = c24 * fma(2.0 * s6, s6, -s6) * inv;
                acc[0] = fma(cf, r0, acc[0]);
                acc[1] = fma(cf, r1, acc[1]);
                acc[2] = fma(cf, r2, acc[2]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; c++) sPart[w][c][lane] = acc[c];
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        double v = sPart[0][c][lane];
#pragma unroll
        for (int q = 1; q < kWaves; q++) v += sPart[q][c][lane];
        acc[c] = v;
    }
    if (real) {
#pragma unroll
        for (int c = 0; c < 3; c++) E.flj[(size_t)c * N + i] = acc[c];
    }
    const bool pushed = real && (acc[0] != 0.0 || acc[1] != 0.0 || acc[2] != 0.0);
    const uint64_t mask = __ballot(pushed ? 1 : 0);
    if (lane == 0 && it.p0 < N) E.lj_mask[it.p0 / kLjMaskPoints] = mask;
}

// ------------------------------------------------------- reduce + epilogue

__device__ __forceinline__ void rotate_frame(const double *din, double *__restrict__ Dout, int N, int i,
                                             double vx, double vy, double vz, bool reorth) {
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

// One block per kReducePoints points: the waves each sum a fixed share of
// the split-K chunks for the block's points (lane = point), the parts are
// combined through LDS in wave order, and wave 0 runs the epilogue.
template <int EPI>
__global__ __launch_bounds__(kReduceThreads) void k_reduce(int stage, int scheme, double dt,
                                                   const EnsDesc *__restrict__ desc,
                                                   const PointItem *__restrict__ items) {
    __shared__ double sPart[kReduceThreads / 64][6][64];
    const PointItem it = items[blockIdx.x];
    const EnsDesc &E = desc[it.ens];
    const int N = E.N;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = it.p0 + lane;
    const int K = E.K;
    const int k0 = (K * w) / (kReduceThreads / 64), k1 = (K * (w + 1)) / (kReduceThreads / 64);
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // wave 0 loads the state its epilogue updates before the partial sums,
    // so that the two memory latencies overlap
    double xv[3] = {0.0, 0.0, 0.0}, dv[9], uav[3] = {0.0, 0.0, 0.0}, wav[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 9; k++) dv[k] = 0.0;
    if (EPI != EPI_WRITE && w == 0 && i < N) {
#pragma unroll
        for (int c = 0; c < 3; c++) xv[c] = E.X[(size_t)c * N + i];
#pragma unroll
        for (int k = 0; k < 9; k++) dv[k] = E.D[(size_t)k * N + i];
        if (EPI != EPI_EULER && stage > 0) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                uav[c] = E.Ua[(size_t)c * N + i];
                wav[c] = E.Wa[(size_t)c * N + i];
            }
        }
    }
    if (i < N) {
        const double *__restrict__ part = E.part;
        // unrolled so that several chunks' loads are in flight; the sum
        // order (k ascending) is unchanged
#pragma unroll 4
        for (int k = k0; k < k1; k++)
#pragma unroll
            for (int c = 0; c < 6; c++) acc[c] += part[((size_t)k * 6 + c) * N + i];
    }
#pragma unroll
    for (int c = 0; c < 6; c++) sPart[w][c][lane] = acc[c];
    __syncthreads();
    if (w != 0 || i >= N) return;
#pragma unroll
    for (int c = 0; c < 6; c++) {
        double v = sPart[0][c][lane];
#pragma unroll
        for (int q = 1; q < kReduceThreads / 64; q++) v += sPart[q][c][lane];
        acc[c] = v;
    }
    if (dt != dt) dt = E.dt;  // NaN: per-ensemble step size
    // the step's last epilogue advances the ensemble clock (one writer)
    if ((EPI == EPI_EULER || EPI == EPI_RK_FINAL) && i == 0 && E.clock) *E.clock += dt;
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
    double ua[3], wa[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (stage == 0) {
            E.U[(size_t)c * N + i] = U[c];
            E.W[(size_t)c * N + i] = W[c];
            ua[c] = wgt * U[c];
            wa[c] = wgt * W[c];
        } else {
            ua[c] = uav[c] + wgt * U[c];
            wa[c] = wav[c] + wgt * W[c];
        }
    }
    if (EPI == EPI_RK_STAGE) {
        const double h = kRkNextNode[scheme][stage] * dt;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            E.Ua[(size_t)c * N + i] = ua[c];
            E.Wa[(size_t)c * N + i] = wa[c];
            E.Xs[(size_t)c * N + i] = xv[c] + h * U[c];
        }
        rotate_frame(dv, E.Ds, N, i, h * W[0], h * W[1], h * W[2], false);
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

// ------------------------------------------------------ Parareal correction

// X = Xf + Xg - Xo and D = reorth(Df + Dg - Do) for every point (SoA state).
__global__ __launch_bounds__(kBlock) void k_parareal_correct(int N, const double *__restrict__ Xf,
                                                             const double *__restrict__ Df,
                                                             const double *__restrict__ Xg,
                                                             const double *__restrict__ Dg,
                                                             const double *__restrict__ Xo,
                                                             const double *__restrict__ Do,
                                                             double *__restrict__ X, double *__restrict__ D) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const size_t k = (size_t)c * N + i;
        X[k] = Xf[k] + Xg[k] - Xo[k];
    }
    double d[9];
#pragma unroll
    for (int c = 0; c < 9; c++) {
        const size_t k = (size_t)c * N + i;
        d[c] = Df[k] + Dg[k] - Do[k];
    }
    reorthonormalize(d);
#pragma unroll
    for (int c = 0; c < 9; c++) D[(size_t)c * N + i] = d[c];
}

// ------------------------------------------------------------ clock probe

// One wave spins until `cycles` shader-clock ticks (s_memtime) have passed,
// or `max_iter` reads, and writes the shader ticks and the constant
// reference-clock ticks (s_memrealtime) that elapsed.
__global__ __launch_bounds__(64) void k_clock_probe(int64_t cycles, int64_t max_iter, uint64_t *out) {
    const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    uint64_t t = t0;
    for (int64_t i = 0; i < max_iter && t - t0 < (uint64_t)cycles; i++) t = __builtin_amdgcn_s_memtime();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
        out[0] = t - t0;
        out[1] = r1 - r0;
    }
}

hipError_t launch_clock_probe(int64_t cycles, uint64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_clock_probe, dim3(1), dim3(64), 0, s, cycles, (int64_t)1 << 26, out);
    return hipGetLastError();
}

// --------------------------------------------------------- launch wrappers

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_pack_aos(int prec, const EnsDesc *d_desc, const EnsDesc &h_desc, hipStream_t s) {
    if (h_desc.N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_aos, dim3(blocks_for(h_desc.N)), dim3(kBlock), 0, s, prec, d_desc);
    return hipGetLastError();
}

hipError_t launch_rod_forces(int prec, int stage_state, int elastic, int scheme, int stage, double dt,
                             const EnsDesc *d_desc, const RodItem *d_items, int n_items, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rod_forces, dim3(n_items), dim3(kBlock), 0, s, prec, stage_state, elastic, scheme,
                       stage, dt, d_desc, d_items);
    return hipGetLastError();
}

hipError_t launch_lj(int stage_state, const EnsDesc *d_desc, const PointItem *d_box_items, int n_box_items,
                     const PointItem *d_items, int n_items, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lj_boxes, dim3(n_box_items), dim3(kBlock), 0, s, stage_state, d_desc, d_box_items);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lj_forces, dim3(n_items), dim3(64 * kLjWaves), 0, s, stage_state, d_desc, d_items);
    return hipGetLastError();
}

hipError_t launch_reduce(int epi, int stage, int scheme, double dt, const EnsDesc *d_desc,
                         const PointItem *d_items, int n_items, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    const dim3 g(n_items), b(kReduceThreads);
    switch (epi) {
        case EPI_EULER: hipLaunchKernelGGL(k_reduce<EPI_EULER>, g, b, 0, s, stage, scheme, dt, d_desc, d_items); break;
        case EPI_RK_STAGE: hipLaunchKernelGGL(k_reduce<EPI_RK_STAGE>, g, b, 0, s, stage, scheme, dt, d_desc, d_items); break;
        case EPI_RK_FINAL: hipLaunchKernelGGL(k_reduce<EPI_RK_FINAL>, g, b, 0, s, stage, scheme, dt, d_desc, d_items); break;
        default: hipLaunchKernelGGL(k_reduce<EPI_WRITE>, g, b, 0, s, stage, scheme, dt, d_desc, d_items); break;
    }
    return hipGetLastError();
}

hipError_t launch_parareal_correct(int N, const double *Xf, const double *Df, const double *Xg, const double *Dg,
                                  const double *Xo, const double *Do, double *X, double *D, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_parareal_correct, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, Xf, Df, Xg, Dg, Xo, Do, X, D);
    return hipGetLastError();
}

hipError_t launch_rotsqrt(int64_t count, const double *R, double *S, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rotsqrt, dim3(blocks_for(count)), dim3(kBlock), 0, s, count, R, S);
    return hipGetLastError();
}

}  // namespace mrs
