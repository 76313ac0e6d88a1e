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

#include "mrs_device_pairs.h"
#include "mrs_device_rod.h"
#include "mrs_internal.h"

namespace mrs {

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

// Descriptor of source block b from the positions X (SoA, or AoS with
// aos), one wave: the same hi/lo split as the records (split_pos).
__device__ __forceinline__ void block_desc_from_x(const EnsDesc &E, const double *__restrict__ X, bool aos, int b) {
    const int N = E.N;
    const int i = b * kDescPoints + (int)(threadIdx.x & 63);
    const bool real = i < N;
    float h[3] = {0.f, 0.f, 0.f}, l[3] = {0.f, 0.f, 0.f};
    if (real) {
#pragma unroll
        for (int c = 0; c < 3; c++) split_pos(aos ? X[3 * (size_t)i + c] : X[(size_t)c * N + i], E.inv_eps, h[c], l[c]);
    }
    src_block_desc(E.wanch, E.blk, b, i, real, h[0], h[1], h[2], l[0], l[1], l[2]);
}

// One thread per point; with FP32C block descriptors (E.blk set) every wave
// (64 consecutive points, block-aligned) also writes its block's descriptor.
__global__ __launch_bounds__(kBlock) void k_pack_aos(int prec, const EnsDesc *__restrict__ desc) {
    const EnsDesc &E = desc[0];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const double *X = E.Xin_aos, *f = E.fext, *n = E.next;
    if (i < E.N)
        store_rec(prec, E.rec, i, X[3 * i], X[3 * i + 1], X[3 * i + 2], f[3 * i], f[3 * i + 1],
                  f[3 * i + 2], n[3 * i], n[3 * i + 1], n[3 * i + 2], E.inv_eps);
    const int b = i / kDescPoints;  // wave-uniform
    if (prec == 1 && E.blk && b * kDescPoints < E.N) block_desc_from_x(E, X, true, b);
}

// One block per filament (rod_filament), or one wave per source-block
// descriptor (RodItem with fil < 0): the descriptors depend only on the
// positions, so they are written beside the filaments' records.
__global__ __launch_bounds__(kBlock) void k_rod_forces(int prec, int stage_state, int elastic, int scheme,
                                                       int stage, double dt, const EnsDesc *__restrict__ desc,
                                                       const RodItem *__restrict__ items) {
    const RodItem it = items[blockIdx.x];
    const EnsDesc &E = desc[it.ens];
    if (it.fil < 0) {  // the whole block takes this branch
        const int b = (-1 - it.fil) * (kBlock / 64) + (int)(threadIdx.x >> 6);
        if (b * kDescPoints < E.N) block_desc_from_x(E, stage_state ? E.Xs : E.X, false, b);
        return;
    }
    rod_filament<kBlock>(prec, stage_state, elastic, scheme, stage, dt, E, it.fil, E.rec);
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
    double kv[3] = {0.0, 0.0, 0.0};
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
                if (scheme == 0) kv[c] = E.Ks[(size_t)c * N + i];
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
    epilogue_point<EPI>(E, N, i, acc, xv, dv, uav, wav, kv, stage, scheme, dt);
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
