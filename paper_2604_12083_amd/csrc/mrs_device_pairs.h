// Device arithmetic of the all-pairs MRS sum (Sec. II.C, Eqs. velocity_field,
// angular_velocity_field, superposition) used by the pair kernels: the
// reciprocal square roots, the pair contributions in FP32 (units of eps) and
// FP64, compensated addition and wave-wide reductions.  The kernel functions
// are listed at the top of mrs_pairs.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "mrs_internal.h"

namespace mrs {

__device__ __forceinline__ float rsq_f32(float x) { return __builtin_amdgcn_rsqf(x); }

// Hardware reciprocal square root refined by one third-order step
// q <- q (1 + e/2 + 3 e^2/8), e = 1 - x q^2, which takes the hardware
// estimate to double precision.
__device__ __forceinline__ double rsq_f64(double x) {
    double q = __builtin_amdgcn_rsq(x);
    double e = fma(-x, q * q, 1.0);
    double p = fma(0.375, e, 0.5);
    return fma(q * e, p, q);
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float x) {
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Pairs closer than rho = r/eps < 4 (R^2 = rho^2 + 1 < 17) carry the largest
// terms of every sum; the FP32C kernels evaluate them in FP64 (on the exact
// hi/lo difference) and every other pair in FP32.
constexpr float kNearR2 = 17.0f;

// R^2 = rho^2 + 1 of a target (th + tl) and a source (sh + sl), in FP32.
// Both the hot loop and the near-pair rescan use this one function, so they
// take the same near/far decision bit for bit.
__device__ __forceinline__ float sep_f32(float thx, float thy, float thz, float tlx, float tly,
                                         float tlz, float shx, float shy, float shz, float slx,
                                         float sly, float slz, float &rx, float &ry, float &rz) {
    rx = (thx - shx) + (tlx - slx);
    ry = (thy - shy) + (tly - sly);
    rz = (thz - shz) + (tlz - slz);
    return fmaf(rz, rz, fmaf(ry, ry, fmaf(rx, rx, 1.0f)));
}

// Contribution of one source at separation r (R2 = |r|^2 + 1) to p[0..5] =
// (8 pi mu U, 8 pi mu eps Omega) of one target, in units of eps.  With MASK a
// near pair adds exactly zero; without it the caller guarantees that no pair
// is near.
template <bool MASK>
__device__ __forceinline__ void pair_core_f32(float rx, float ry, float rz, float R2, float fx,
                                              float fy, float fz, float nx, float ny, float nz,
                                              float *p) {
    const float q = (MASK && R2 < kNearR2) ? 0.0f : rsq_f32(R2);
    const float q2 = q * q, q3 = q2 * q, q5 = q3 * q2, q7 = q5 * q2;
    const float h1 = q + q3;
    const float t = 1.5f * q5;
    const float h3 = q3 + t;
    const float u = 3.75f * q7;
    const float h5 = u + t;
    const float h4 = fmaf(-0.5f, h3, u);
    const float fr = fmaf(fz, rz, fmaf(fy, ry, fx * rx));
    const float nr = fmaf(nz, rz, fmaf(ny, ry, nx * rx));
    const float a = q3 * fr, b = h5 * nr;
    // H3 (n x r) = n x g and H3 (f x r) = f x g with g = H3 r
    const float gx = h3 * rx, gy = h3 * ry, gz = h3 * rz;
    p[0] = fmaf(-nz, gy, fmaf(ny, gz, fmaf(a, rx, fmaf(h1, fx, p[0]))));
    p[1] = fmaf(-nx, gz, fmaf(nz, gx, fmaf(a, ry, fmaf(h1, fy, p[1]))));
    p[2] = fmaf(-ny, gx, fmaf(nx, gy, fmaf(a, rz, fmaf(h1, fz, p[2]))));
    p[3] = fmaf(-fz, gy, fmaf(fy, gz, fmaf(b, rx, fmaf(h4, nx, p[3]))));
    p[4] = fmaf(-fx, gz, fmaf(fz, gx, fmaf(b, ry, fmaf(h4, ny, p[4]))));
    p[5] = fmaf(-fy, gx, fmaf(fx, gy, fmaf(b, rz, fmaf(h4, nz, p[5]))));
}

// The same for a source record (a = hi + fx, b = lo + fy, c = fz, n); returns R^2.
template <bool MASK>
__device__ __forceinline__ float pair_f32(float thx, float thy, float thz, float tlx, float tly,
                                          float tlz, const float4 A, const float4 B,
                                          const float4 C, float *p) {
    float rx, ry, rz;
    const float R2 = sep_f32(thx, thy, thz, tlx, tly, tlz, A.x, A.y, A.z, B.x, B.y, B.z, rx, ry, rz);
    pair_core_f32<MASK>(rx, ry, rz, R2, A.w, B.w, C.x, C.y, C.z, C.w, p);
    return R2;
}

// Same in FP64 for the separation r = x_target - X_source:
// p += (8 pi mu U, 8 pi mu Omega) in unscaled units (e2 = eps^2, c375e2 =
// 3.75 eps^2), or the eps-unit form with e2 = 1, c375e2 = 3.75.
__device__ __forceinline__ void pair_f64_r(double rx, double ry, double rz, double fx, double fy,
                                           double fz, double nx, double ny, double nz, double e2,
                                           double c375e2, double *p) {
    const double R2 = fma(rz, rz, fma(ry, ry, fma(rx, rx, e2)));
    const double q = rsq_f64(R2);
    const double q2 = q * q, q3 = q2 * q, q5 = q3 * q2, q7 = q5 * q2;
    const double h1 = fma(e2, q3, q);
    const double t = 1.5 * q5;
    const double h3 = fma(e2, t, q3);
    const double u = c375e2 * q7;
    const double h5 = t + u;
    const double h4 = fma(-0.5, h3, e2 * u);
    const double fr = fma(fz, rz, fma(fy, ry, fx * rx));
    const double nr = fma(nz, rz, fma(ny, ry, nx * rx));
    const double a = q3 * fr, b = h5 * nr;
    const double gx = h3 * rx, gy = h3 * ry, gz = h3 * rz;  // see pair_f32
    p[0] = fma(-nz, gy, fma(ny, gz, fma(a, rx, fma(h1, fx, p[0]))));
    p[1] = fma(-nx, gz, fma(nz, gx, fma(a, ry, fma(h1, fy, p[1]))));
    p[2] = fma(-ny, gx, fma(nx, gy, fma(a, rz, fma(h1, fz, p[2]))));
    p[3] = fma(-fz, gy, fma(fy, gz, fma(b, rx, fma(h4, nx, p[3]))));
    p[4] = fma(-fx, gz, fma(fz, gx, fma(b, ry, fma(h4, ny, p[4]))));
    p[5] = fma(-fy, gx, fma(fx, gy, fma(b, rz, fma(h4, nz, p[5]))));
}

__device__ __forceinline__ void pair_f64(double tx, double ty, double tz, double x, double y,
                                         double z, double fx, double fy, double fz, double nx,
                                         double ny, double nz, double e2, double c375e2,
                                         double *p) {
    pair_f64_r(tx - x, ty - y, tz - z, fx, fy, fz, nx, ny, nz, e2, c375e2, p);
}

// FP64 evaluation of a near pair from FP32 hi/lo positions: the hi and lo
// differences are exact in FP64, the loads are the record's FP32 values.
__device__ __forceinline__ void near_pair_f64(float thx, float thy, float thz, float tlx, float tly,
                                              float tlz, float shx, float shy, float shz, float slx,
                                              float sly, float slz, float fx, float fy, float fz,
                                              float nx, float ny, float nz, double *p) {
    const double rx = ((double)thx - (double)shx) + ((double)tlx - (double)slx);
    const double ry = ((double)thy - (double)shy) + ((double)tly - (double)sly);
    const double rz = ((double)thz - (double)shz) + ((double)tlz - (double)slz);
    pair_f64_r(rx, ry, rz, fx, fy, fz, nx, ny, nz, 1.0, 3.75, p);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Source blocks of the FP32C tiled kernels.  Boxes are taken over the hi
// parts of the positions and then widened by 2^-23 of their largest
// coordinate magnitude on every side, which covers the lo parts
// (|lo| <= 2^-24 |hi|), so box tests hold for the exact positions.
constexpr float kBoxWiden = 1.0f / 8388608.0f;  // 2^-23

// Widens a hi-part box [lo, hi] to contain the exact positions.
__device__ __forceinline__ void widen_box(float *lo, float *hi) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const float m = fmaxf(fabsf(lo[k]), fabsf(hi[k])) * kBoxWiden;
        lo[k] -= m;
        hi[k] += m;
    }
}

// Descriptor of the aligned 64-point block b of an ensemble, computed by one
// wave whose lane l holds point 64 b + l (real: below N) with position hi + lo
// (the record's split): the widened box of the real points' hi parts, its
// centre c, the squared half-diagonal, and every real point's anchored
// position w = (hi - c) + lo.  The tiled pair kernels read these instead of
// reducing every staged block again (the same values for every target tile).
// A block's box and centre depend on its real points only, in any order.
__device__ __forceinline__ void src_block_desc(float4 *__restrict__ wanch, float *__restrict__ blk, int b, int i,
                                               bool real, float hx, float hy, float hz, float lx, float ly,
                                               float lz) {
    float lo[3], hi[3], ctr[3], hd2 = 0.0f;
    lo[0] = wave_min(real ? hx : INFINITY); lo[1] = wave_min(real ? hy : INFINITY);
    lo[2] = wave_min(real ? hz : INFINITY);
    hi[0] = wave_max(real ? hx : -INFINITY); hi[1] = wave_max(real ? hy : -INFINITY);
    hi[2] = wave_max(real ? hz : -INFINITY);
    widen_box(lo, hi);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        ctr[k] = 0.5f * (lo[k] + hi[k]);
        const float h = 0.5f * (hi[k] - lo[k]);
        hd2 = fmaf(h, h, hd2);
    }
    if (real) wanch[i] = make_float4((hx - ctr[0]) + lx, (hy - ctr[1]) + ly, (hz - ctr[2]) + lz, 0.0f);
    if ((threadIdx.x & 63) == 0) {
        float *d = blk + (size_t)kDescFloats * b;
#pragma unroll
        for (int k = 0; k < 3; k++) { d[k] = lo[k]; d[3 + k] = hi[k]; d[6 + k] = ctr[k]; }
        d[9] = hd2;
    }
}

// wave_sum of M values at once, level by level, so that the M exchanges of
// a level are in flight together; each value is added exactly as wave_sum
// adds it (same partners, same order), so the bits are the same.
template <int M>
__device__ __forceinline__ void wave_sum_n(double *v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double o[M];
#pragma unroll
        for (int k = 0; k < M; k++) o[k] = __shfl_xor(v[k], off, 64);
#pragma unroll
        for (int k = 0; k < M; k++) v[k] += o[k];
    }
}

}  // namespace mrs
