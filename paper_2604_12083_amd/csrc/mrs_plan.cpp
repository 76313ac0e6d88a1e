// Work lists of the pair kernels: how an ensemble's all-pairs sum (Sec.
// II.C, Eq. superposition) is cut into blocks of (target tile, source chunk)
// and in which order the blocks are dispatched.  Host code only; the order
// and the cut change no result beyond the rounding of the split-K sum, which
// is fixed for a given configuration.
#include <algorithm>
#include <climits>
#include <vector>

#include "mrs_runtime.h"

namespace mrs {

// Default pair-kernel configuration for an ensemble of N points.  Small
// ensembles (split_mode) use the wave-split kernel; larger ones the
// LDS-tiled kernel with 1 (FP32C) or 2 (FP64; 1 for mid-size grids, below)
// targets per lane and
// enough source chunks that the grid holds ~64 blocks per compute unit
// (short blocks keep the tail of the grid short; measured on MI355X at
// 12,800 and 256,000 points).  A chunk has at least 128 sources (64 in small
// grids) and at least N/64, so the split-K partials stay a small fraction of
// the pair work.
//
// Tail split (automatic FP32C tiled configurations of grids of at least four
// blocks per compute unit): the last ~8% of the sources of every target tile
// go into chunks of a quarter chunk (at least 64 sources) whose blocks are
// dispatched last.  A SIMD issues the oldest of its waves first, so the waves
// that start last run alone at the end of the grid; short ones keep that end
// short (measured on MI355X: pair kernel -3.4% at 12,800 points, -0.6% at
// 256,000; the FP64 kernel, two targets per lane, gets slower).
constexpr int kTailPercent = 8, kTailDiv = 4;

// Blocks of the tiled kernel at `tpl` targets per lane and 128-source chunks.
static int64_t blocks_at(int64_t N, int tpl) {
    const int64_t tiles = (N + (int64_t)kBlock * tpl - 1) / ((int64_t)kBlock * tpl);
    return tiles * ((N + 2 * kKahanBlock - 1) / (2 * kKahanBlock));
}

// Mid-size and small grids (measured on MI355X, interleaved A/B against the
// previous rule).  The FP64 kernel takes one target per lane when two would
// give fewer than three blocks per compute unit: twice the waves hide the
// FP64 latency of the near-pair and contact work (3,200 to 6,400 points:
// -7% to -17% alone, -1% to -2% in batches of 16; neutral at 7,680).  When
// 128-source chunks give at most one block per compute unit, chunks shrink
// to 64 sources (2,048 points FP32C: -26% alone, neutral batched; 1,275
// points, 25 swimmers: FP64 23 -> 15 us, and FP32C 48 -> 31 us before that
// size moved to the wave-split kernel).
static bool fp64_one_target(int64_t N, int n_cu) { return blocks_at(N, 2) < (int64_t)3 * n_cu; }
static bool small_grid(int64_t N, int tpl, int n_cu) { return blocks_at(N, tpl) <= (int64_t)n_cu; }

// Ensembles up to 1,024 points use the wave-split kernel (one target per
// wave, lanes split the sources), in both precisions.  Alone it is faster
// than the tiled kernel up to ~1,500 points (MI355X, pair + reduction
// kernels, FP32C: 1,024 points 18.8 vs 25.8 us, 1,280 points 20.4 vs 26.1),
// but in batches of 16 ensembles it loses from ~1,000 points on (1,024
// points 67 vs 44 us, 1,280 points 90 vs 58; 512 points even), so the limit
// stays where the batched cost is still moderate.
static bool split_mode(int64_t N, int) { return N <= 1024; }

// Automatic tiled configurations with at least this many blocks per CU run
// the persistent schedule (blocks claim items from a queue).  In grids this
// deep it was faster than the hardware grid on MI355X (interleaved A/B of
// the pair kernel: 256,000 points -1.3% FP32C and -1.5% FP64, 1,000
// swimmers (51,000 points, 58 blocks per CU) -1.4% FP32C; the tuner's
// one-shot evaluations: 102,400 points -1.3% and -1.1%); in shallow grids
// it is much slower (12,800 points, 12 blocks per CU: +20%).  The FP64
// kernel at two targets per lane keeps four blocks per CU resident instead
// of five, and from about six rounds of them (24 blocks per CU) the
// persistent schedule won there too (51,200 points: -1.9% in the tuner;
// 1,000 swimmers, 24 blocks per CU: -1.3% in interleaved A/B).
constexpr int kPersistentBlocksPerCu = 48, kPersistentBlocksPerCuF64T2 = 24;

PairCfg choose_cfg_for(const PairCfg *tuned, int64_t N, int prec, int n_cu) {
    PairCfg c;
    bool small = false;
    if (tuned) {
        c = *tuned;
        if (c.mode == PAIR_QUAD && prec != MRS_FP32C) c.mode = PAIR_TILE;  // the four-wave split is FP32C only
        if (c.mode == PAIR_QUAD) c.tpl = 1;
    } else {
        c.mode = split_mode(N, prec) ? PAIR_SPLIT : PAIR_TILE;
        c.tpl = (prec == MRS_FP32C) ? 1 : 2;
        c.K = 0;
        if (c.mode == PAIR_TILE && prec == MRS_FP64 && fp64_one_target(N, n_cu)) c.tpl = 1;
    }
    // automatic chunking (also of a stored configuration with chunks = 0):
    // 64-source chunks in small grids, as without a stored configuration
    if (c.mode == PAIR_TILE && c.K <= 0) small = small_grid(N, c.tpl, n_cu);
    if (c.mode == PAIR_SPLIT) {
        c.K = 1;
        c.chunk = (int)N;
        return c;
    }
    const int64_t tile = c.mode == PAIR_QUAD ? 64 : (int64_t)kBlock * c.tpl;
    const int64_t tiles = (N + tile - 1) / tile;
    int64_t chunk;
    const bool automatic = c.K <= 0;
    if (automatic) {
        const int64_t want_blocks = (int64_t)n_cu * 64;
        const int64_t K = (want_blocks + tiles - 1) / tiles;
        chunk = std::max<int64_t>({(N + K - 1) / K, (int64_t)(small ? 1 : 2) * kKahanBlock, N / 64});
    } else {
        chunk = (N + c.K - 1) / c.K;
    }
    chunk = ((chunk + kKahanBlock - 1) / kKahanBlock) * kKahanBlock;
    c.chunk = (int)std::max<int64_t>(chunk, kKahanBlock);
    c.K = (int)std::max<int64_t>(1, (N + c.chunk - 1) / c.chunk);
    c.k_big = c.K;
    c.tail_start = c.tail_chunk = 0;
    const int64_t deep = prec == MRS_FP64 && c.tpl == 2 ? kPersistentBlocksPerCuF64T2 : kPersistentBlocksPerCu;
    if (!tuned && c.mode == PAIR_TILE && tiles * c.K >= deep * n_cu) c.sched = SCHED_PERSISTENT;
    if (automatic && prec == MRS_FP32C && tiles * c.K >= (int64_t)4 * n_cu) {
        const int64_t tc = std::max<int64_t>(kKahanBlock, (c.chunk / kTailDiv + kKahanBlock - 1) / kKahanBlock * kKahanBlock);
        const int64_t tail = (N * kTailPercent / 100 + tc - 1) / tc * tc;
        const int64_t B = (N - tail) / kKahanBlock * kKahanBlock;
        if (B > c.chunk) {
            c.tail_start = (int)B;
            c.tail_chunk = (int)tc;
            c.k_big = (int)((B + c.chunk - 1) / c.chunk);
            c.K = c.k_big + (int)((N - B + tc - 1) / tc);
        }
    }
    return c;
}

void add_items(Plan &P, int e, int64_t N, int n_fil, const PairCfg &c) {
    if (c.mode != PAIR_SPLIT && c.sched == SCHED_PERSISTENT) P.sched = SCHED_PERSISTENT;
    if (c.mode == PAIR_SPLIT) {
        for (int64_t t0 = 0; t0 < N; t0 += kSplitTargetsPerBlock)
            P.split.push_back({e, (int)t0, (int)std::min<int64_t>(kSplitTargetsPerBlock, N - t0), 0, (int)N, 0});
    } else {
        const bool quad = c.mode == PAIR_QUAD;
        const int64_t tile = quad ? 64 : (int64_t)kBlock * c.tpl;
        auto &dst = quad ? P.quad : (c.tpl == 2 ? P.tile2 : P.tile1);
        auto &tail = quad ? P.tailq : (c.tpl == 2 ? P.tail2 : P.tail1);
        // chunk-major: consecutive blocks share a source chunk, so every XCD
        // (blocks go to the 8 XCDs in turn) reads each chunk once into its L2
        const int64_t B = c.tail_start > 0 ? c.tail_start : N;  // end of the regular chunks
        for (int k = 0; k < c.k_big && (int64_t)k * c.chunk < B; k++) {
            const int64_t s0 = (int64_t)k * c.chunk;
            for (int64_t t0 = 0; t0 < N; t0 += tile)
                dst.push_back({e, (int)t0, (int)std::min<int64_t>(tile, N - t0), (int)s0,
                               (int)std::min<int64_t>(c.chunk, B - s0), k});
        }
        int k = c.k_big;
        for (int64_t s0 = B; s0 < N; s0 += c.tail_chunk, k++)
            for (int64_t t0 = 0; t0 < N; t0 += tile)
                tail.push_back({e, (int)t0, (int)std::min<int64_t>(tile, N - t0), (int)s0,
                                (int)std::min<int64_t>(c.tail_chunk, N - s0), k});
    }
    for (int f = 0; f < n_fil; f++) P.rods.push_back({e, f});
    // FP32C tiled kernels read the source-block descriptors, which the rod
    // launch writes: one item per kBlock / 64 blocks
    if (P.prec == MRS_FP32C && c.mode != PAIR_SPLIT && n_fil > 0) {
        const int64_t groups = (N + kBlock - 1) / kBlock;
        for (int64_t g = 0; g < groups; g++) P.rods.push_back({e, (int)(-1 - g)});
    }
    for (int64_t p0 = 0; p0 < N; p0 += kReducePoints) P.pts.push_back({e, (int)p0});
    P.pairs_per_eval += N * N;
}

// Blocks whose source range overlaps their own targets in index order hold
// the near pairs along each filament (masked path plus the FP64 rescan) and
// run longest; dispatching them first keeps them off the tail of a launch.
// The order of blocks does not change any result: each writes its own slots.
void near_blocks_first(std::vector<PairItem> &v) {
    std::stable_partition(v.begin(), v.end(), [](const PairItem &it) {
        return it.src0 < it.tgt0 + it.ntgt + kKahanBlock && it.tgt0 < it.src0 + it.nsrc + kKahanBlock;
    });
}

void order_items(Plan &P) {
    near_blocks_first(P.tile1);
    near_blocks_first(P.tile2);
    near_blocks_first(P.quad);
    P.tile1.insert(P.tile1.end(), P.tail1.begin(), P.tail1.end());
    P.tile2.insert(P.tile2.end(), P.tail2.begin(), P.tail2.end());
    P.quad.insert(P.quad.end(), P.tailq.begin(), P.tailq.end());
    P.tail1.clear();
    P.tail2.clear();
    P.tailq.clear();
}

}  // namespace mrs

using namespace mrs;

extern "C" mrs_status mrs_plan_items(int64_t n, mrs_precision prec, int32_t n_cu, int32_t *mode,
                                     int32_t *targets_per_lane, int32_t *chunks, int32_t *tail_start,
                                     int32_t *items, int64_t max_items, int64_t *n_items) {
    if (!n_items || n < 1 || n > INT32_MAX / 8 || n_cu < 1 || (prec != MRS_FP64 && prec != MRS_FP32C) ||
        max_items < 0)
        return MRS_EINVAL;
    const PairCfg c = choose_cfg_for(nullptr, n, (int)prec, n_cu);
    Plan P;
    P.prec = (int)prec;
    add_items(P, 0, n, 0, c);
    order_items(P);
    const std::vector<PairItem> &v =
        c.mode == PAIR_SPLIT ? P.split : (c.mode == PAIR_QUAD ? P.quad : (c.tpl == 2 ? P.tile2 : P.tile1));
    *n_items = (int64_t)v.size();
    if (mode) *mode = c.mode;
    if (targets_per_lane) *targets_per_lane = c.tpl;
    if (chunks) *chunks = c.K;
    if (tail_start) *tail_start = c.tail_start > 0 ? c.tail_start : (int32_t)n;
    if (!items) return MRS_OK;
    if (max_items < (int64_t)v.size()) return MRS_EINVAL;
    for (size_t i = 0; i < v.size(); i++) {
        int32_t *o = items + 5 * i;
        o[0] = v[i].tgt0;
        o[1] = v[i].ntgt;
        o[2] = v[i].src0;
        o[3] = v[i].nsrc;
        o[4] = v[i].chunk;
    }
    return MRS_OK;
}
