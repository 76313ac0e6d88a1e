// Internal types shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrs {

// Threads per block of every kernel on the path (4 wave64s).
constexpr int kBlock = 256;
// Sources staged in LDS per tile of the tiled pair kernel.
constexpr int kSrcTile = 256;
// Sources summed in plain FP32 before one compensated (Kahan) update.
constexpr int kKahanBlock = 64;
// Targets per wave in the small-N pair kernel (lanes split the sources).
// One: the kernel is latency-bound, and four times the waves shorten each
// wave's chain (MI355X: 64 points 10.2 -> 6.6 us FP32C, 8.2 -> 6.3 us FP64;
// 960 points 27.7 -> 15.0 us and 19.1 -> 11.8 us; same results, since each
// target's sum is formed the same way).
constexpr int kSplitTargetsPerWave = 1;
constexpr int kSplitTargetsPerBlock = kSplitTargetsPerWave * (kBlock / 64);

// Source record of the FP32C pair kernel, 48 bytes, read as three float4:
//   a = (xh, yh, zh, fx)  b = (xl, yl, zl, fy)  c = (fz, nx, ny, nz)
// with positions scaled by 1/eps and split hi + lo, forces scaled by 1/eps
// and torques by 1/eps^2.
struct alignas(16) RecF32 {
    float4 a, b, c;
};

// Source record of the FP64 pair kernel, 80 bytes (five 16-byte words).
struct alignas(16) RecF64 {
    double x, y, z, fx, fy, fz, nx, ny, nz, pad;
};

// Source-block descriptor of the FP32C tiled pair kernels (one per aligned
// 64-point block), padded to 64 bytes.
constexpr int kDescFloats = 16;
constexpr int kDescPoints = 64;

// Bytes of a record buffer for n points in either precision: FP64 records,
// or FP32C records followed by the anchored positions and the block
// descriptors.
inline size_t rec_buffer_bytes(int64_t n) {
    const size_t f64 = (size_t)n * sizeof(RecF64);
    const size_t f32 = (size_t)n * (sizeof(RecF32) + sizeof(float4)) +
                       (size_t)((n + kDescPoints - 1) / kDescPoints) * kDescFloats * sizeof(float);
    return f64 > f32 ? f64 : f32;
}

// Everything a kernel needs to know about one ensemble.  Arrays are SoA:
// component c of point i of an N-point vector field lives at [c * N + i];
// director i, component c of point k at [(3 i + c) * N + k].
struct EnsDesc {
    int32_t N;
    int32_t n_fil;
    int32_t K;         // source chunks of the split-K pair kernel
    int32_t aos_io;    // 1: X/f/n inputs and U/W outputs are n x 3 row-major
    const int32_t *off;
    double *X, *D;     // state (SoA)
    double *Xs, *Ds;   // RK stage state (SoA)
    double *U, *W;     // velocities (SoA, or AoS when aos_io)
    double *Ua, *Wa;   // RK weighted sums (SoA)
    double *Ks;        // RK4: the last stage's corrected angular velocity k (SoA)
    const double *fext, *next;  // external loads (SoA, or AoS when aos_io), may be null
    const double *Xin_aos;      // AoS positions when aos_io
    void *rec;         // source records (RecF32 or RecF64), N entries
    // FP32C tiled pair kernels: per point its position relative to the centre
    // of its aligned 64-point block (anchored form), and per block the
    // descriptor (kDescFloats floats: widened hi-part box lo[3], hi[3],
    // centre[3], squared half-diagonal); both follow the records in the same
    // buffer (set_records) and are written with them (k_rod_forces
    // descriptor items, k_pack_aos)
    float4 *wanch;
    float *blk;
    double *part;      // split-K partial sums [K][6][N]
    double *g_out, *m_out;  // optional AoS copies of the rod loads (tests)
    double eps, inv_eps, mu;
    double cU, cW;     // 1/(8 pi mu) and the Omega scale of the record form
    double a[3], b[3], om0[3], ds;
    double dt;         // step size used when a launch passes dt = NaN
    int32_t elastic;   // rod forces on/off used when a launch passes elastic < 0
    // swimming (Sec. IV): waveform (A, k, f) added to the preferred
    // strain-twist, Lennard-Jones repulsion between filaments
    int32_t has_wave, has_lj;
    int32_t n_ljblk;        // source blocks of the LJ pass (with LJ)
    double wave[3];
    double lj_sig, lj_e, lj_rc;
    double *clock;          // time at the start of the current step (one double)
    const int32_t *fil;     // filament of each point (with LJ)
    double *flj;            // LJ force on each point [3][N] (with LJ)
    const int32_t *lj_blk;  // per LJ source block: first point, end, filament (with LJ)
    double *lj_box;         // per LJ source block: lo[3], hi[3] of its positions (with LJ)
    uint64_t *lj_mask;      // per aligned 64-point block: bit j set when point 64 b + j
                            // feels a LJ force (with LJ)
    int32_t *nonfinite;     // set to 1 (plain vector store) by the reduction when a
                            // result it writes is not finite; may be null
};

// Source blocks of the Lennard-Jones pass hold at most this many consecutive
// points of one filament; the LJ mask covers aligned blocks of 64 points.
constexpr int kLjBlockPoints = 64;
constexpr int kLjMaskPoints = 64;

// One block of a pair kernel: targets [tgt0, tgt0 + ntgt) against sources
// [src0, src0 + nsrc) of ensemble `ens`, written to split-K chunk `chunk`.
struct PairItem {
    int32_t ens, tgt0, ntgt, src0, nsrc, chunk;
};

// One block of the rod-force kernel: filament `fil` of ensemble `ens`; or,
// with fil = -1 - g (FP32C tiled configurations), the source-block
// descriptors of blocks kBlock / 64 * g ... of ensemble `ens`, one per wave.
struct RodItem {
    int32_t ens, fil;
};

// Points per block of the reduction/epilogue kernel, and its threads: the
// block's waves split the source chunks of its points.
constexpr int kReducePoints = 64;
constexpr int kReduceThreads = 256;

// One block of the reduction/epilogue kernel: points [p0, p0 + kReducePoints).
struct PointItem {
    int32_t ens, p0;
};

enum Epilogue : int {
    EPI_WRITE = 0,     // U, W only
    EPI_EULER = 1,     // U, W and a forward Euler step
    EPI_RK_STAGE = 2,  // accumulate stage s, build stage state s + 1
    EPI_RK_FINAL = 3,  // accumulate last stage, finish the step
};

// Runge-Kutta schemes of the stage epilogue.
enum RkScheme : int { RK_SCHEME_RK4 = 0, RK_SCHEME_RK2 = 1 };

// Points the records of an ensemble of n points at rec (a buffer of
// rec_buffer_bytes(n)); FP32C also places the anchored positions and block
// descriptors behind the records, FP64 leaves them null.
inline void set_records(EnsDesc &d, void *rec, int64_t n, bool fp32c) {
    d.rec = rec;
    char *b = static_cast<char *>(rec);
    d.wanch = fp32c ? reinterpret_cast<float4 *>(b + (size_t)n * sizeof(RecF32)) : nullptr;
    d.blk = fp32c ? reinterpret_cast<float *>(b + (size_t)n * (sizeof(RecF32) + sizeof(float4))) : nullptr;
}

// Launch wrappers (mrs_pairs.hip, mrs_kernels.hip).  All return the launch's hipError_t.
hipError_t launch_pack_aos(int prec, const EnsDesc *d_desc, const EnsDesc &h_desc,
                           hipStream_t s);
// elastic < 0: every ensemble uses its own EnsDesc::elastic.  The waveform
// time of the launch is clock + c dt, c the node of RK stage `stage` of
// `scheme` (0 for stage 0); dt = NaN: every ensemble uses its own dt.
hipError_t launch_rod_forces(int prec, int stage_state, int elastic, int scheme, int stage, double dt,
                             const EnsDesc *d_desc, const RodItem *d_items, int n_items, hipStream_t s);
// Lennard-Jones forces of the ensembles with has_lj: the box of every LJ
// source block (box items: (ensemble, first of kBlock / 64 blocks)), then the
// force on every point and the LJ masks (target items: (ensemble, first of
// kLjMaskPoints consecutive points)).
hipError_t launch_lj(int stage_state, const EnsDesc *d_desc, const PointItem *d_box_items, int n_box_items,
                     const PointItem *d_items, int n_items, hipStream_t s);
// queue (two uint32 that are zero before the launch and zero again after
// it) and resident > 0: tiled kernels run the persistent schedule with
// min(n_items, resident) blocks; otherwise one block per item.
hipError_t launch_pairs(int prec, int mode, int tpl, const EnsDesc *d_desc, const PairItem *d_items,
                        int n_items, hipStream_t s, uint32_t *queue = nullptr, int resident = 0);
// Resident blocks per CU of the persistent tiled pair kernel.
int pairs_resident_blocks(int prec, int tpl);
// dt = NaN: every ensemble uses its own EnsDesc::dt.
hipError_t launch_reduce(int epi, int stage, int scheme, double dt, const EnsDesc *d_desc,
                         const PointItem *d_items, int n_items, hipStream_t s);
hipError_t launch_rotsqrt(int64_t count, const double *R, double *S, hipStream_t s);
// out[0] = shader-clock ticks, out[1] = reference-clock ticks of a spin of `cycles` ticks.
hipError_t launch_clock_probe(int64_t cycles, uint64_t *out, hipStream_t s);
// Parareal correction (SoA states of N points): X = Xf + Xg - Xo, D = reorth(Df + Dg - Do).
hipError_t launch_parareal_correct(int N, const double *Xf, const double *Df, const double *Xg, const double *Dg,
                                  const double *Xo, const double *Do, double *X, double *D, hipStream_t s);

// Pair-kernel modes.
// PAIR_QUAD (FP32C): tiles of 64 targets whose four waves split the sources.
enum PairMode : int { PAIR_TILE = 0, PAIR_SPLIT = 1, PAIR_QUAD = 2 };
// Schedules of the tiled pair kernels: one block per item, or a resident
// grid whose blocks claim items from a queue.
enum PairSched : int { SCHED_GRID = 0, SCHED_PERSISTENT = 1 };
// Work-queue counters per plan: one pair of uint32 per pair-kernel launch
// of a stage (split, tile1, tile2), padded.
constexpr int kQueueWords = 16;

}  // namespace mrs
