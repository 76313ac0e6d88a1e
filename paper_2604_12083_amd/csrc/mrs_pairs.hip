// HIP kernels (gfx950) of the all-pairs MRS sum (Sec. II.C, Eqs.
// velocity_field, angular_velocity_field, superposition).
//
//   k_pairs_tile_*    one lane per target (T targets per lane), sources
//                     staged through LDS and broadcast to the wave, split-K
//                     over source chunks
//   k_pairs_split     small-ensemble form: a wave owns a few targets, its lanes
//                     stride over the sources and the sums are combined with
//                     wave shuffles
//
// Kernel functions.  With R^2 = r^2 + eps^2, Q = 1/R and H_i the kernel
// functions of the blob phi_eps (Sec. II.C), 8 pi H_i are
//   H1: Q + eps^2 Q^3            H2: Q^3
//   H3: Q^3 + 1.5 eps^2 Q^5      H4: 3.75 eps^4 Q^7 - 0.75 eps^2 Q^5 - 0.5 Q^3
//   H5: 1.5 Q^5 + 3.75 eps^2 Q^7
// The FP32C form works in units of eps (rho = r/eps, f~ = f/eps,
// n~ = n/eps^2), where the same expressions hold with eps = 1 and
// U = sum/(8 pi mu), Omega = sum/(8 pi mu eps); this keeps every FP32
// intermediate far from overflow and folds all constants into one FP64
// scale per target.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mrs_device_pairs.h"
#include "mrs_internal.h"

namespace mrs {

// ----------------------------------------------------------------- pairs

// Squared distance between the boxes [lo0, hi0] and [lo1, hi1] (0 if they overlap).
__device__ __forceinline__ float box_gap2(const float *lo0, const float *hi0, const float *lo1, const float *hi1) {
    float d2 = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const float g = fmaxf(0.0f, fmaxf(lo0[c] - hi1[c], lo1[c] - hi0[c]));
        d2 = fmaf(g, g, d2);
    }
    return d2;
}

// A wave whose target box is farther than this (squared, in units of eps)
// from a source block's box has no near pair in it (rho >= 4).  The boxes
// are the widened hi-part boxes of the block descriptors (src_block_desc),
// which contain the exact positions at any distance from the origin.
constexpr float kFarBoxGap2 = 17.0f;

// Anchored far blocks.  Relative to the centre c of a 64-source block's box,
// a source sits at w = (sh - c) + sl (stored with the block descriptors) and
// a target at u = (th - c) + tl, and r = u - w costs 3 instead of 9
// operations.  Each of u and w takes two FP32 roundings (at most 2^-24 of
// its magnitude each), and r one more; with the gap between the boxes larger
// than the block's half-diagonal, |w| < |r| and |u| < 2 |r|, so r keeps a
// relative error below 7 x 2^-24 < 2^-21, against 2^-23 for the exact hi/lo
// difference of the other paths.  (A gap of 4 half-diagonals, |w| <= |r|/4,
// sent more blocks down the exact-separation path and was 2.6% slower on
// 1,000 swimmers of 51 points, 3.4% on 16 batched 3,200-point slices;
// MI355X, interleaved A/B, 12,800 points even.)
constexpr float kAnchorGapRatio2 = 1.0f;

// Block descriptors and contact masks are written before the pair launch and
// only read by it, so the kernel reads them through the constant address
// space: the loads are wave-uniform and go through the scalar cache into
// scalar registers.
typedef __attribute__((address_space(4))) const float desc_float;
typedef __attribute__((address_space(4))) const uint64_t mask_word;
__device__ __forceinline__ const desc_float *desc_at(const float *blk, int64_t b) {
    return (const desc_float *)(blk + (size_t)kDescFloats * b);
}

// Persistent schedule.  The grid holds as many blocks as the device keeps
// resident; each block claims the next item of the work list from a counter
// (queue[0], an ordinary vector atomic from one lane) until the list is
// exhausted, so blocks that run ahead take more items and the device stays
// full until the last items, which the work list makes the shortest.  Every
// item still writes its own partial slot: results do not depend on which
// block ran which item.  The last block to leave (queue[1] counts them)
// resets both counters, so the next launch (or graph replay) starts at zero.
__device__ __forceinline__ int claim_item(uint32_t *queue, int *sNext) {
    __syncthreads();  // the previous item is finished and sNext has been read
    if (threadIdx.x == 0) *sNext = (int)atomicAdd(queue, 1u);
    __syncthreads();
    return *sNext;
}

__device__ __forceinline__ void leave_queue(uint32_t *queue) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(queue + 1, 1u) == gridDim.x - 1) {
            atomicExch(queue, 0u);
            atomicExch(queue + 1, 0u);
        }
    }
}

// Orders a wave's own LDS writes before its later reads (and its reads
// before later writes) without waiting for the other waves of the block.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Blocks per CU the register budget must allow: 5 with one target per lane
// (<= 102 VGPRs), 3 with two (<= 170).  PERSIST: items claimed from the queue;
// otherwise block b runs item b.
//
// QUAD (one target per lane): the block's four waves share the item's 64
// targets and split its sources, wave w taking the 64-source blocks w, w + 4,
// ... of the item; each wave stages and uses only its own blocks (no block
// barrier in the loop), and the four waves' sums are added in wave order at
// the end of the item.  A wave's share of an item is a quarter of the
// item's pairs, so the waves that run last on a SIMD hold short work.
template <int T, bool PERSIST, bool QUAD>
__global__ __launch_bounds__(kBlock, T == 1 ? 5 : 3) void k_pairs_tile_f32(const EnsDesc *__restrict__ desc,
                                                           const PairItem *__restrict__ items, int n_items,
                                                           uint32_t *queue) {
    static_assert(!QUAD || T == 1, "four-wave source split: one target per lane");
    // staged sources: sW = (w, fx) with w the anchored position, sF = (fy, fz,
    // nx, ny), sN = (nz, lo), sH = (hi, 0)
    __shared__ float4 sW[kSrcTile], sF[kSrcTile], sN[kSrcTile], sH[kSrcTile];
    __shared__ double sNear[6][T][kBlock];  // FP64 near-pair sums, one slot per lane and target
    static_assert(kSrcTile / kKahanBlock == kBlock / 64 && kKahanBlock == kDescPoints,
                  "one source block (one descriptor) per wave");
    __shared__ int sNext;
    int idx = PERSIST ? claim_item(queue, &sNext) : (int)blockIdx.x;
    while (idx < n_items) {
    const PairItem it = items[idx];
    const EnsDesc &E = desc[it.ens];
    const RecF32 *__restrict__ rec = reinterpret_cast<const RecF32 *>(E.rec);
    const int tid = threadIdx.x;
    // target slot of this lane: the block's lanes (tiled) or the wave's (QUAD)
    const int tl = QUAD ? (tid & 63) : tid;
    float thx[T], thy[T], thz[T], tlx[T], tly[T], tlz[T];
    float s[T][6], c[T][6];
    // box of this wave's targets: the descriptors of the blocks they lie in
    // (tiles start on block boundaries; lanes past the tile repeat its last
    // target, which lies in the block of the last real lane)
    float tlo[3] = {INFINITY, INFINITY, INFINITY}, thi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int t = 0; t < T; t++) {
        const int li = min(tl + t * kBlock, it.ntgt - 1);
        const RecF32 r = rec[it.tgt0 + li];
        thx[t] = r.a.x; thy[t] = r.a.y; thz[t] = r.a.z;
        tlx[t] = r.b.x; tly[t] = r.b.y; tlz[t] = r.b.z;
        const int wb = (it.tgt0 + min((tl & ~63) + t * kBlock, it.ntgt - 1)) / kDescPoints;  // wave-uniform
        const desc_float *d = desc_at(E.blk, wb);
#pragma unroll
        for (int k = 0; k < 3; k++) { tlo[k] = fminf(tlo[k], d[k]); thi[k] = fmaxf(thi[k], d[3 + k]); }
#pragma unroll
        for (int k = 0; k < 6; k++) { s[t][k] = 0.0f; c[t][k] = 0.0f; sNear[k][t][tid] = 0.0; }
    }
    for (int base = 0; base < it.nsrc; base += kSrcTile) {
        if (QUAD) {
            if (base + (tid & ~63) >= it.nsrc) break;  // wave-uniform: this wave has no block left
            wave_sync();
        } else {
            __syncthreads();
        }
        // this wave stages source block tid / 64 (its anchored positions
        // from the descriptors); padding lanes stage zero loads
        const int j = base + tid;
        const bool real = j < it.nsrc;
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, cc = a, w = a;
        if (real) {
            const RecF32 r = rec[it.src0 + j];
            a = r.a; b = r.b; cc = r.c;
            w = E.wanch[it.src0 + j];
        }
        // a source with contact forces enters the FP32 sums with zero loads;
        // the FP64 pass evaluates it with its own loads
        bool contact = false;
        if (E.lj_mask && real) {
            const int jg = it.src0 + j;
            contact = (E.lj_mask[jg / kLjMaskPoints] >> (jg % kLjMaskPoints)) & 1;
        }
        sW[tid] = make_float4(w.x, w.y, w.z, contact ? 0.0f : a.w);
        sF[tid] = contact ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(b.w, cc.x, cc.y, cc.z);
        sN[tid] = make_float4(contact ? 0.0f : cc.w, b.x, b.y, b.z);
        sH[tid] = make_float4(a.x, a.y, a.z, 0.0f);
        if (QUAD) wave_sync();
        else __syncthreads();
        const int cnt = min(kSrcTile, it.nsrc - base);
        // QUAD: only the block this wave staged
        const int sb0 = QUAD ? (tid & ~63) : 0;
        const int sb1 = QUAD ? sb0 + kKahanBlock : cnt;
        for (int sb = sb0; sb < sb1; sb += kKahanBlock) {
            // Issue priority of this wave: the 64-source blocks of the item
            // still to do after this one (3 or more: highest).  A SIMD
            // issues its oldest wave first among equals, so without this
            // the waves that start last wait behind older ones and then
            // finish the launch alone; preferring the waves with the most
            // work left evens out when a SIMD's waves finish (measured on
            // MI355X: -1.2% at 12,800 points, -1.5% for 16 batched 3,200-
            // point slices, +0.5% for 1,000 swimmers, 256,000 points even).
            {
                const int left = (it.nsrc - base - sb - 1) / kKahanBlock;  // wave-uniform
                if (left >= 3) __builtin_amdgcn_s_setprio(3);
                else if (left == 2) __builtin_amdgcn_s_setprio(2);
                else if (left == 1) __builtin_amdgcn_s_setprio(1);
                else __builtin_amdgcn_s_setprio(0);
            }
            float p[T][6];
            // bit j of near[t]: source sb + j is near target t (masked path only)
            uint64_t near[T];
#pragma unroll
            for (int t = 0; t < T; t++) {
                near[t] = 0;
#pragma unroll
                for (int k = 0; k < 6; k++) p[t][k] = 0.0f;
            }
            // descriptor of this source block (wave-uniform)
            float bx[10];
            {
                const desc_float *bd = desc_at(E.blk, (it.src0 + base + sb) / kDescPoints);
#pragma unroll
                for (int k = 0; k < 10; k++) bx[k] = bd[k];
            }
            const float gap2 = box_gap2(tlo, thi, bx, bx + 3);
            // sources of this block that carry contact forces (wave-uniform)
            const uint64_t ljm = E.lj_mask ? ((const mask_word *)E.lj_mask)[(it.src0 + base + sb) / kLjMaskPoints] : 0;
            if (gap2 > kFarBoxGap2 && gap2 > kAnchorGapRatio2 * bx[9]) {
                // wave-uniform: no near pair, separation from the block's anchor
                float ux[T], uy[T], uz[T];
#pragma unroll
                for (int t = 0; t < T; t++) {
                    ux[t] = (thx[t] - bx[6]) + tlx[t];
                    uy[t] = (thy[t] - bx[7]) + tly[t];
                    uz[t] = (thz[t] - bx[8]) + tlz[t];
                }
                // four sources per iteration: 51.5 instead of 52 VALU
                // instructions per pair (LDS address and loop counter) and
                // 2-3% faster on MI355X; still 96 VGPRs, no spills
#pragma unroll 4
                for (int jj = sb; jj < sb + kKahanBlock; jj++) {
                    const float4 W = sW[jj], F = sF[jj], Nn = sN[jj];
#pragma unroll
                    for (int t = 0; t < T; t++) {
                        const float rx = ux[t] - W.x, ry = uy[t] - W.y, rz = uz[t] - W.z;
                        const float R2 = fmaf(rz, rz, fmaf(ry, ry, fmaf(rx, rx, 1.0f)));
                        pair_core_f32<false>(rx, ry, rz, R2, W.w, F.x, F.y, F.z, F.w, Nn.x, p[t]);
                    }
                }
            } else if (gap2 > kFarBoxGap2) {
                // wave-uniform: no near pair, exact hi/lo separation
#pragma unroll 2
                for (int jj = sb; jj < sb + kKahanBlock; jj++) {
                    const float4 W = sW[jj], F = sF[jj], Nn = sN[jj], H = sH[jj];
#pragma unroll
                    for (int t = 0; t < T; t++) {
                        float rx, ry, rz;
                        const float R2 = sep_f32(thx[t], thy[t], thz[t], tlx[t], tly[t], tlz[t], H.x, H.y, H.z,
                                                 Nn.y, Nn.z, Nn.w, rx, ry, rz);
                        pair_core_f32<false>(rx, ry, rz, R2, W.w, F.x, F.y, F.z, F.w, Nn.x, p[t]);
                    }
                }
            } else {
#pragma unroll 2
                for (int jj = sb; jj < sb + kKahanBlock; jj++) {
                    const float4 W = sW[jj], F = sF[jj], Nn = sN[jj], H = sH[jj];
#pragma unroll
                    for (int t = 0; t < T; t++) {
                        float rx, ry, rz;
                        const float R2 = sep_f32(thx[t], thy[t], thz[t], tlx[t], tly[t], tlz[t], H.x, H.y, H.z,
                                                 Nn.y, Nn.z, Nn.w, rx, ry, rz);
                        pair_core_f32<true>(rx, ry, rz, R2, W.w, F.x, F.y, F.z, F.w, Nn.x, p[t]);
                        near[t] |= (uint64_t)(R2 < kNearR2) << (jj - sb);
                    }
                }
            }
            // the sources with contact forces join the FP64 pass for every target
#pragma unroll
            for (int t = 0; t < T; t++) near[t] |= ljm;
#pragma unroll
            for (int t = 0; t < T; t++)
#pragma unroll
                for (int k = 0; k < 6; k++) kahan_add(s[t][k], c[t][k], p[t][k]);
            // the pairs masked above, in FP64 on the exact hi/lo difference:
            // each lane walks only its own near sources
#pragma unroll
            for (int t = 0; t < T; t++) {
                uint64_t m = near[t];
                if (m) {
                    double pn[6];
#pragma unroll
                    for (int k = 0; k < 6; k++) pn[k] = sNear[k][t][tid];
                    do {
                        const int jj = sb + __builtin_ctzll(m);
                        m &= m - 1;
                        const float4 W = sW[jj], F = sF[jj], Nn = sN[jj], H = sH[jj];
                        float fx = W.w, fy = F.x, fz = F.y, nx = F.z, ny = F.w, nz = Nn.x;
                        if ((ljm >> (jj - sb)) & 1) {  // staged with zero loads: take them from the record
                            const RecF32 r = rec[it.src0 + base + jj];
                            fx = r.a.w; fy = r.b.w; fz = r.c.x; nx = r.c.y; ny = r.c.z; nz = r.c.w;
                        }
                        near_pair_f64(thx[t], thy[t], thz[t], tlx[t], tly[t], tlz[t], H.x, H.y, H.z, Nn.y, Nn.z,
                                      Nn.w, fx, fy, fz, nx, ny, nz, pn);
                    } while (m);
#pragma unroll
                    for (int k = 0; k < 6; k++) sNear[k][t][tid] = pn[k];
                }
            }
        }
    }
    const int N = E.N;
    if (QUAD) {
        // the four waves' sums for the same targets, added in wave order
#pragma unroll
        for (int k = 0; k < 6; k++) sNear[k][0][tid] += (double)s[0][k] - (double)c[0][k];
        __syncthreads();
        if (tid < 64 && tid < it.ntgt) {
#pragma unroll
            for (int k = 0; k < 6; k++) {
                double v = sNear[k][0][tid];
#pragma unroll
                for (int w = 1; w < kBlock / 64; w++) v += sNear[k][0][w * 64 + tid];
                E.part[((size_t)it.chunk * 6 + k) * N + it.tgt0 + tid] = v;
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < T; t++) {
            const int li = tid + t * kBlock;
            if (li < it.ntgt) {
#pragma unroll
                for (int k = 0; k < 6; k++)
                    E.part[((size_t)it.chunk * 6 + k) * N + it.tgt0 + li] =
                        ((double)s[t][k] - (double)c[t][k]) + sNear[k][t][tid];
            }
        }
    }
    if (!PERSIST) break;
    idx = claim_item(queue, &sNext);
    }
    if (PERSIST) leave_queue(queue);
}

template <int T, bool PERSIST>
__global__ __launch_bounds__(kBlock) void k_pairs_tile_f64(const EnsDesc *__restrict__ desc,
                                                           const PairItem *__restrict__ items, int n_items,
                                                           uint32_t *queue) {
    __shared__ double2 s0[kSrcTile], s1[kSrcTile], s2[kSrcTile], s3[kSrcTile], s4[kSrcTile];
    __shared__ int sNext;
    int idx = PERSIST ? claim_item(queue, &sNext) : (int)blockIdx.x;
    while (idx < n_items) {
    const PairItem it = items[idx];
    const EnsDesc &E = desc[it.ens];
    const RecF64 *__restrict__ rec = reinterpret_cast<const RecF64 *>(E.rec);
    const int tid = threadIdx.x;
    const double e2 = E.eps * E.eps, c375e2 = 3.75 * e2;
    double tx[T], ty[T], tz[T], acc[T][6];
#pragma unroll
    for (int t = 0; t < T; t++) {
        const int li = min(tid + t * kBlock, it.ntgt - 1);
        const RecF64 &r = rec[it.tgt0 + li];
        tx[t] = r.x; ty[t] = r.y; tz[t] = r.z;
#pragma unroll
        for (int k = 0; k < 6; k++) acc[t][k] = 0.0;
    }
    const double2 *__restrict__ rw = reinterpret_cast<const double2 *>(rec);
    for (int base = 0; base < it.nsrc; base += kSrcTile) {
        __syncthreads();
        const int j = base + tid;
        double2 w0 = make_double2(0.0, 0.0), w1 = w0, w2 = w0, w3 = w0, w4 = w0;
        if (j < it.nsrc) {
            const double2 *src = rw + (size_t)(it.src0 + j) * 5;
            w0 = src[0]; w1 = src[1]; w2 = src[2]; w3 = src[3]; w4 = src[4];
        }
        s0[tid] = w0; s1[tid] = w1; s2[tid] = w2; s3[tid] = w3; s4[tid] = w4;
        __syncthreads();
        const int cnt = min(kSrcTile, it.nsrc - base);
#pragma unroll 2
        for (int jj = 0; jj < cnt; jj++) {
            const double2 a = s0[jj], b = s1[jj], cc = s2[jj], d = s3[jj], e = s4[jj];
#pragma unroll
            for (int t = 0; t < T; t++)
                pair_f64(tx[t], ty[t], tz[t], a.x, a.y, b.x, b.y, cc.x, cc.y, d.x, d.y, e.x, e2, c375e2, acc[t]);
        }
    }
    const int N = E.N;
#pragma unroll
    for (int t = 0; t < T; t++) {
        const int li = tid + t * kBlock;
        if (li < it.ntgt) {
#pragma unroll
            for (int k = 0; k < 6; k++) E.part[((size_t)it.chunk * 6 + k) * N + it.tgt0 + li] = acc[t][k];
        }
    }
    if (!PERSIST) break;
    idx = claim_item(queue, &sNext);
    }
    if (PERSIST) leave_queue(queue);
}

// Small-ensemble pair kernel: each wave owns kSplitTargetsPerWave targets and
// its 64 lanes stride over the item's sources; per-lane sums are combined in
// FP64 with a butterfly of wave shuffles in a fixed order.
// Sources staged through LDS per round by the whole block (its waves share
// them): FP32C rounds are the 1,024-source compensated chunks of the loop
// below (48 KB), FP64 rounds 256 sources (20 KB).  A lane reads its sources
// in the same order as straight from the records, so the staging changes no
// result; it replaces one dependent global load per lane and 64 sources by
// one per round.
constexpr int kSplitPerLane = 16;  // FP32C: sources per lane between compensated updates
constexpr int kSplitRoundF32 = 64 * kSplitPerLane, kSplitRoundF64 = kBlock;

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_pairs_split(const EnsDesc *__restrict__ desc,
                                                        const PairItem *__restrict__ items) {
    constexpr int TW = kSplitTargetsPerWave;
    static_assert(sizeof(RecF32) == 48 && sizeof(RecF64) == 80, "record layouts");
    __shared__ float4 sBuf[PREC == 1 ? 3 * kSplitRoundF32 : 5 * kSplitRoundF64];
    const PairItem it = items[blockIdx.x];
    const EnsDesc &E = desc[it.ens];
    const int tid = threadIdx.x, lane = tid & 63;
    const int tb = (tid >> 6) * TW;
    // a wave without targets still stages sources and meets every barrier
    const bool active = tb < it.ntgt;  // wave-uniform
    double out[TW][6];
    if (PREC == 1) {
        const RecF32 *__restrict__ rec = reinterpret_cast<const RecF32 *>(E.rec);
        RecF32 *sRec = reinterpret_cast<RecF32 *>(sBuf);
        float thx[TW], thy[TW], thz[TW], tlx[TW], tly[TW], tlz[TW], s[TW][6], c[TW][6];
        double pn[TW][6];
#pragma unroll
        for (int t = 0; t < TW; t++) {
            const RecF32 r = rec[it.tgt0 + min(tb + t, it.ntgt - 1)];
            thx[t] = r.a.x; thy[t] = r.a.y; thz[t] = r.a.z;
            tlx[t] = r.b.x; tly[t] = r.b.y; tlz[t] = r.b.z;
#pragma unroll
            for (int k = 0; k < 6; k++) { s[t][k] = 0.f; c[t][k] = 0.f; pn[t][k] = 0.0; }
        }
        for (int j0 = 0; j0 < it.nsrc; j0 += kSplitRoundF32) {
            const int cnt = min(kSplitRoundF32, it.nsrc - j0);
            __syncthreads();
            for (int q = tid; q < cnt; q += kBlock) sRec[q] = rec[it.src0 + j0 + q];
            __syncthreads();
            if (!active) continue;
            float p[TW][6];
            float rmin = kNearR2;
#pragma unroll
            for (int t = 0; t < TW; t++)
#pragma unroll
                for (int k = 0; k < 6; k++) p[t][k] = 0.f;
            for (int j = lane; j < cnt; j += 64) {
                const int jg = it.src0 + j0 + j;
                if (E.lj_mask && ((E.lj_mask[jg / kLjMaskPoints] >> (jg % kLjMaskPoints)) & 1)) {
                    rmin = 0.0f;  // a source with contact forces: FP64 below
                    continue;
                }
                const RecF32 r = sRec[j];
#pragma unroll
                for (int t = 0; t < TW; t++)
                    rmin = fminf(rmin, pair_f32<true>(thx[t], thy[t], thz[t], tlx[t], tly[t], tlz[t], r.a, r.b, r.c, p[t]));
            }
#pragma unroll
            for (int t = 0; t < TW; t++)
#pragma unroll
                for (int k = 0; k < 6; k++) kahan_add(s[t][k], c[t][k], p[t][k]);
            if (rmin < kNearR2) {  // near pairs and contact-force blocks of this lane's sources: FP64
                for (int j = lane; j < cnt; j += 64) {
                    const RecF32 r = sRec[j];
                    const int jg = it.src0 + j0 + j;
                    const bool strong = E.lj_mask && ((E.lj_mask[jg / kLjMaskPoints] >> (jg % kLjMaskPoints)) & 1);
#pragma unroll
                    for (int t = 0; t < TW; t++) {
                        float rx, ry, rz;
                        if (strong || sep_f32(thx[t], thy[t], thz[t], tlx[t], tly[t], tlz[t], r.a.x, r.a.y, r.a.z, r.b.x,
                                              r.b.y, r.b.z, rx, ry, rz) < kNearR2)
                            near_pair_f64(thx[t], thy[t], thz[t], tlx[t], tly[t], tlz[t], r.a.x, r.a.y, r.a.z, r.b.x,
                                          r.b.y, r.b.z, r.a.w, r.b.w, r.c.x, r.c.y, r.c.z, r.c.w, pn[t]);
                    }
                }
            }
        }
        if (!active) return;  // no barrier follows
#pragma unroll
        for (int t = 0; t < TW; t++)
#pragma unroll
            for (int k = 0; k < 6; k++) out[t][k] = ((double)s[t][k] - (double)c[t][k]) + pn[t][k];
        wave_sum_n<6 * TW>(&out[0][0]);
    } else {
        const RecF64 *__restrict__ rec = reinterpret_cast<const RecF64 *>(E.rec);
        RecF64 *sRec = reinterpret_cast<RecF64 *>(sBuf);
        const double e2 = E.eps * E.eps, c375e2 = 3.75 * e2;
        double tx[TW], ty[TW], tz[TW], acc[TW][6];
#pragma unroll
        for (int t = 0; t < TW; t++) {
            const RecF64 &r = rec[it.tgt0 + min(tb + t, it.ntgt - 1)];
            tx[t] = r.x; ty[t] = r.y; tz[t] = r.z;
#pragma unroll
            for (int k = 0; k < 6; k++) acc[t][k] = 0.0;
        }
        for (int j0 = 0; j0 < it.nsrc; j0 += kSplitRoundF64) {
            const int cnt = min(kSplitRoundF64, it.nsrc - j0);
            __syncthreads();
            for (int q = tid; q < cnt; q += kBlock) sRec[q] = rec[it.src0 + j0 + q];
            __syncthreads();
            if (!active) continue;
            for (int j = lane; j < cnt; j += 64) {
                const RecF64 r = sRec[j];
#pragma unroll
                for (int t = 0; t < TW; t++)
                    pair_f64(tx[t], ty[t], tz[t], r.x, r.y, r.z, r.fx, r.fy, r.fz, r.nx, r.ny, r.nz, e2, c375e2, acc[t]);
            }
        }
        if (!active) return;  // no barrier follows
#pragma unroll
        for (int t = 0; t < TW; t++)
#pragma unroll
            for (int k = 0; k < 6; k++) out[t][k] = acc[t][k];
        wave_sum_n<6 * TW>(&out[0][0]);
    }
    if (lane < 6) {
        const int N = E.N;
#pragma unroll
        for (int t = 0; t < TW; t++) {
            if (tb + t < it.ntgt) {
                double v = out[t][0];
#pragma unroll
                for (int k = 1; k < 6; k++) v = (lane == k) ? out[t][k] : v;
                E.part[((size_t)it.chunk * 6 + lane) * N + it.tgt0 + tb + t] = v;
            }
        }
    }
}

// --------------------------------------------------------- launch wrapper

template <int T, bool PERSIST>
static void launch_tile(int prec, dim3 g, dim3 b, hipStream_t s, const EnsDesc *d_desc, const PairItem *d_items,
                        int n_items, uint32_t *queue) {
    if (prec == 1)
        hipLaunchKernelGGL((k_pairs_tile_f32<T, PERSIST, false>), g, b, 0, s, d_desc, d_items, n_items, queue);
    else hipLaunchKernelGGL((k_pairs_tile_f64<T, PERSIST>), g, b, 0, s, d_desc, d_items, n_items, queue);
}

// Resident blocks per CU of a tiled pair kernel (persistent schedule).
int pairs_resident_blocks(int prec, int tpl) {
    static int cache[2][3] = {{0, 0, 0}, {0, 0, 0}};
    int &c = cache[prec == 1][tpl == 2 ? 2 : 1];
    if (c > 0) return c;
    int nb = 0;
    hipError_t e;
    if (prec == 1)
        e = tpl == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pairs_tile_f32<2, true, false>, kBlock, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pairs_tile_f32<1, true, false>, kBlock, 0);
    else
        e = tpl == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pairs_tile_f64<2, true>, kBlock, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pairs_tile_f64<1, true>, kBlock, 0);
    c = (e == hipSuccess && nb > 0) ? nb : 1;
    return c;
}

hipError_t launch_pairs(int prec, int mode, int tpl, const EnsDesc *d_desc, const PairItem *d_items,
                        int n_items, hipStream_t s, uint32_t *queue, int resident) {
    if (n_items == 0) return hipSuccess;
    const dim3 b(kBlock);  // the pair kernels index LDS by threadIdx.x < kBlock
    if (mode == PAIR_SPLIT) {
        const dim3 g(n_items);
        if (prec == 1) hipLaunchKernelGGL(k_pairs_split<1>, g, b, 0, s, d_desc, d_items);
        else hipLaunchKernelGGL(k_pairs_split<0>, g, b, 0, s, d_desc, d_items);
    } else if (mode == PAIR_QUAD) {  // FP32C only (the plan never makes FP64 QUAD items)
        if (queue && resident > 0)
            hipLaunchKernelGGL((k_pairs_tile_f32<1, true, true>), dim3((unsigned)std::min(n_items, resident)), b, 0, s,
                               d_desc, d_items, n_items, queue);
        else
            hipLaunchKernelGGL((k_pairs_tile_f32<1, false, true>), dim3(n_items), b, 0, s, d_desc, d_items, n_items,
                               nullptr);
    } else if (queue && resident > 0) {
        const dim3 g((unsigned)std::min(n_items, resident));
        if (tpl == 2) launch_tile<2, true>(prec, g, b, s, d_desc, d_items, n_items, queue);
        else launch_tile<1, true>(prec, g, b, s, d_desc, d_items, n_items, queue);
    } else {
        const dim3 g(n_items);
        if (tpl == 2) launch_tile<2, false>(prec, g, b, s, d_desc, d_items, n_items, nullptr);
        else launch_tile<1, false>(prec, g, b, s, d_desc, d_items, n_items, nullptr);
    }
    return hipGetLastError();
}

}  // namespace mrs
