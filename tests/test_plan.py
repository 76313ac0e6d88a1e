"""Host logic of the pair-kernel decomposition, checked on the CPU.

`mrs_plan_items` returns the work list that the automatic configuration
builds for one ensemble (no device is touched).  Every (target, source) pair
of the all-pairs sum (Sec. II.C, Eq. superposition, j = i included) must be
covered exactly once, every block must own its partial-sum slot, and the
dispatch order must be the one the runtime promises: blocks with near pairs
along a filament first, regular chunks chunk-major, short tail chunks last.
"""
import numpy as np
import pytest

import paper_2604_12083_amd as mrs

SIZES = [1, 37, 1024, 1025, 3200, 7680, 12800, 51000, 256000, 262144]


def _cover_check(n, items):
    """Targets: the tiles partition [0, n); per tile, the source ranges of its
    blocks partition [0, n) and their slots are distinct."""
    tiles = {}
    for t0, nt, s0, ns, k in items:
        assert nt >= 1 and ns >= 1 and 0 <= t0 and t0 + nt <= n and 0 <= s0 and s0 + ns <= n
        tiles.setdefault((t0, nt), []).append((s0, ns, k))
    starts = sorted(tiles)
    pos = 0
    for t0, nt in starts:
        assert t0 == pos
        pos += nt
    assert pos == n
    for key, blocks in tiles.items():
        blocks.sort()
        pos = 0
        for s0, ns, _ in blocks:
            assert s0 == pos, (key, s0, pos)
            pos += ns
        assert pos == n
        slots = [k for _, _, k in blocks]
        assert len(set(slots)) == len(slots)
    return tiles


@pytest.mark.parametrize("prec", [mrs.MRS_FP32C, mrs.MRS_FP64])
@pytest.mark.parametrize("n", SIZES)
def test_every_pair_covered_once_with_own_slot(n, prec):
    cfg, items = mrs.mrs_plan_items(n, prec)
    tiles = _cover_check(n, items)
    K = cfg["chunks"]
    assert items[:, 4].min() >= 0 and items[:, 4].max() < K
    split_max = 1024
    if cfg["mode"] == 1:  # wave-split kernel for small ensembles: one chunk
        assert n <= split_max and K == 1
        return
    assert n > split_max
    # every tile has the same K chunks, with slots 0..K-1
    for blocks in tiles.values():
        assert sorted(k for _, _, k in blocks) == list(range(K))
    # chunk boundaries are multiples of 64 sources (anchor blocks, contact masks)
    assert np.all(items[:, 2] % 64 == 0)
    tile = 256 * cfg["targets_per_lane"]
    assert np.all(items[:, 0] % tile == 0) and np.all(items[:, 1] <= tile)


def _is_near(t0, nt, s0, ns):
    return s0 < t0 + nt + 64 and t0 < s0 + ns + 64


@pytest.mark.parametrize("n", [12800, 51000, 256000])
def test_dispatch_order_near_first_chunk_major_tail_last(n):
    cfg, items = mrs.mrs_plan_items(n, mrs.MRS_FP32C)
    K = cfg["chunks"]
    # the tail split: the last ~8% of the sources in short chunks, dispatched last
    tail_src = cfg["tail_start"]
    assert 0.06 * n <= n - tail_src <= 0.12 * n and tail_src % 64 == 0
    tail = items[:, 2] >= tail_src
    assert np.all(items[~tail, 2] + items[~tail, 3] <= tail_src)
    first_tail = np.argmax(tail)
    assert tail.any() and np.all(tail[first_tail:]) and not np.any(tail[:first_tail])
    assert items[tail, 3].max() <= max(64, items[~tail, 3].max() // 4 + 63)
    reg = items[~tail]
    near = np.array([_is_near(*r[:4]) for r in reg])
    first_far = np.argmax(~near)
    assert np.all(near[:first_far]) and not np.any(near[first_far:])
    # chunk-major inside each class: source chunk never decreases
    for part in (reg[near], reg[~near], items[tail]):
        assert np.all(np.diff(part[:, 2]) >= 0)
    assert K == len(np.unique(items[:, 4]))


def test_decomposition_sizes_on_mi355x():
    """The automatic configurations quoted in the design notes for 256 CUs."""
    cfg, items = mrs.mrs_plan_items(12800, mrs.MRS_FP32C)
    assert cfg == {"mode": 0, "targets_per_lane": 1, "chunks": 46 + 16, "tail_start": 11776}
    assert len(items) == 50 * 62
    cfg, items = mrs.mrs_plan_items(12800, mrs.MRS_FP64)
    assert cfg == {"mode": 0, "targets_per_lane": 2, "chunks": 50, "tail_start": 12800} and len(items) == 25 * 50
    cfg, items = mrs.mrs_plan_items(256000, mrs.MRS_FP32C)
    assert cfg["chunks"] == 16 + 6 and sorted(set(items[:, 3].tolist()))[-1] == 15104
    cfg, _ = mrs.mrs_plan_items(256000, mrs.MRS_FP64)
    assert cfg["chunks"] == 33
    cfg, items = mrs.mrs_plan_items(3200, mrs.MRS_FP32C)  # too small a grid for the tail split
    assert cfg["chunks"] == 25 and cfg["tail_start"] == 3200 and items[:, 3].min() == 128
    # mid-size FP64 grids: one target per lane below three blocks per CU at two
    cfg, _ = mrs.mrs_plan_items(6400, mrs.MRS_FP64)
    assert cfg == {"mode": 0, "targets_per_lane": 1, "chunks": 50, "tail_start": 6400}
    cfg, _ = mrs.mrs_plan_items(7680, mrs.MRS_FP64)
    assert cfg["targets_per_lane"] == 2 and cfg["chunks"] == 60
    # at most one block per CU with 128-source chunks: 64-source chunks
    for prec in (mrs.MRS_FP32C, mrs.MRS_FP64):
        cfg, items = mrs.mrs_plan_items(2048, prec)
        assert cfg["targets_per_lane"] == 1 and cfg["chunks"] == 32 and items[:, 3].max() == 64
    for prec in (mrs.MRS_FP32C, mrs.MRS_FP64):
        cfg, _ = mrs.mrs_plan_items(1275, prec)  # 25 swimmers of 51 points
        assert cfg["targets_per_lane"] == 1 and cfg["chunks"] == 20
        # the wave-split kernel up to 1,024 points
        assert mrs.mrs_plan_items(1024, prec)[0]["mode"] == 1 and mrs.mrs_plan_items(1025, prec)[0]["mode"] == 0
    cfg, _ = mrs.mrs_plan_items(1000, mrs.MRS_FP32C)
    assert cfg["mode"] == 1


def test_size_rules_follow_the_cu_count():
    """The one-target and 64-source-chunk rules are stated in blocks per
    compute unit, so a device with fewer CUs switches at smaller sizes."""
    for n_cu, n, prec, tpl, K in [(80, 1275, mrs.MRS_FP32C, 1, 20), (80, 2048, mrs.MRS_FP32C, 1, 16),
                                  (256, 2048, mrs.MRS_FP32C, 1, 32), (80, 3200, mrs.MRS_FP64, 1, 25),
                                  (80, 6400, mrs.MRS_FP64, 2, 50), (256, 6400, mrs.MRS_FP64, 1, 50)]:
        cfg, items = mrs.mrs_plan_items(n, prec, n_cu)
        assert (cfg["targets_per_lane"], cfg["chunks"]) == (tpl, K), (n_cu, n, prec, cfg)
        _cover_check(n, items)


def test_plan_items_invalid_arguments():
    for args in [(0, mrs.MRS_FP32C, 256), (10, 7, 256), (10, mrs.MRS_FP64, 0), (2**31, mrs.MRS_FP64, 256)]:
        with pytest.raises(mrs.MrsError) as ei:
            mrs.mrs_plan_items(*args)
        assert ei.value.status == mrs.MRS_EINVAL
