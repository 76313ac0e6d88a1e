"""GPU parity of the one-shot MRS evaluation against the FP64 oracle.

Error metric: the paper's relative error form (Eq. true_err),
max_i |a_i - b_i|_2 / |b_i|_2, separately for U and Omega.  Tolerances:
1e-12 for MRS_FP64 and 1e-5 for MRS_FP32C.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import eval_dev, rod_of, say

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def mrs():
    import paper_2604_12083_amd as m

    return m


@pytest.fixture(scope="module")
def ctx(mrs):
    c = mrs.mrs_context_create(0)
    yield c
    mrs.mrs_context_destroy(c)


def _cloud(N, seed, box=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, box, (N, 3)), rng.normal(size=(N, 3)), rng.normal(size=(N, 3))


def _check(mrs, ctx, X, f, n, eps, mu, prec, tag, oracle_UW=None):
    say(f"eval {tag} N={len(X)} prec={prec}")
    U, W = eval_dev(mrs, ctx, X, f, n, eps, mu, prec)
    Uo, Wo = oracle_UW if oracle_UW is not None else oracle.mrs_eval(X, f, n, eps, mu)
    eu, ew = oracle.rel_err(U, Uo), oracle.rel_err(W, Wo)
    say(f"  rel err U {eu:.3e} W {ew:.3e}")
    assert eu <= TOL[prec] and ew <= TOL[prec], (tag, prec, eu, ew)
    return eu, ew


@pytest.mark.parametrize("prec", [0, 1])
def test_rod64_eval(mrs, ctx, prec):
    e = synth.rod64()
    _check(mrs, ctx, e.X, e.f, e.n, e.eps, e.mu, prec, "rod64")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("N", [1, 2, 3, 17, 64, 255, 1000, 1024, 1025, 2049, 3000])
def test_sizes_and_ragged_tails(mrs, ctx, prec, N):
    X, f, n = _cloud(N, N, box=0.5)
    _check(mrs, ctx, X, f, n, 0.02, 1.3, prec, f"cloud{N}")


@pytest.mark.parametrize("prec", [0, 1])
def test_ens12800_full(mrs, ctx, prec):
    e = synth.ens12800()
    _check(mrs, ctx, e.X, e.f, e.n, e.eps, e.mu, prec, "ens12800")


@pytest.mark.parametrize("prec", [0, 1])
def test_translation_far_from_origin(mrs, ctx, prec):
    """Large coordinates exercise the hi/lo position split of the FP32C path."""
    e = synth.filaments(8, 64, 2.0, 123)
    Xs = e.X + np.array([1000.25, -750.5, 333.0])
    _check(mrs, ctx, Xs, e.f, e.n, e.eps, e.mu, prec, "shifted")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("eps_units", [1e5, 1e6])
def test_far_from_origin_in_units_of_eps(mrs, ctx, prec, eps_units):
    """An ensemble 1e5 and 1e6 eps from the origin (beyond 2^16 in units of
    eps, where the hi parts of the FP32C positions carry rounding of more than
    a hundredth of eps): the widened boxes keep the near/far and anchoring
    tests valid; 3,000 points so that the tiled kernel and its far paths run."""
    e = synth.filaments(30, 100, 3.0, 124)
    d = eps_units * e.eps * np.array([0.6, -0.64, 0.48])
    _check(mrs, ctx, e.X + d, e.f, e.n, e.eps, e.mu, prec, f"offset {eps_units:g} eps")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("eps", [1e-4, 10.0])
def test_eps_extremes(mrs, ctx, prec, eps):
    X, f, n = _cloud(500, 9, box=1.0)
    _check(mrs, ctx, X, f, n, eps, 1.0, prec, f"eps{eps}")


@pytest.mark.parametrize("prec", [0, 1])
def test_coincident_points(mrs, ctx, prec):
    """Degenerate geometry: pairs at r = 0 between distinct points (every
    kernel function is finite there, Sec. II.C), a block where every pair
    coincides, and duplicates scattered through a cloud."""
    X, f, n = _cloud(300, 12, box=0.6)
    Xd = np.concatenate([X, X[::3]])
    rng = np.random.default_rng(13)
    fd = np.concatenate([f, rng.normal(size=(100, 3))])
    nd = np.concatenate([n, rng.normal(size=(100, 3))])
    _check(mrs, ctx, Xd, fd, nd, 0.02, 1.0, prec, "duplicates")
    Xs = np.tile(np.array([[0.3, -0.2, 0.9]]), (64, 1))
    _check(mrs, ctx, Xs, f[:64], n[:64], 0.05, 1.0, prec, "all-coincident")


@pytest.mark.parametrize("prec", [0, 1])
def test_linearity_and_zero_loads(mrs, ctx, prec):
    """U, Omega are linear in the loads (Eq. superposition): zero loads give
    exactly zero; scaling both loads by 4 scales the results by exactly 4
    (a power of two commutes with every rounding, FP32C records included);
    forces alone plus torques alone give the result of both, per point within
    10x the tolerance times the size of the two parts."""
    X, f, n = _cloud(700, 3)
    z = np.zeros_like(f)
    U, W = eval_dev(mrs, ctx, X, z, z, 0.05, 1.0, prec)
    assert np.all(U == 0) and np.all(W == 0)
    U1, W1 = eval_dev(mrs, ctx, X, f, n, 0.05, 1.0, prec)
    U4, W4 = eval_dev(mrs, ctx, X, 4.0 * f, 4.0 * n, 0.05, 1.0, prec)
    assert np.array_equal(U4, 4.0 * U1) and np.array_equal(W4, 4.0 * W1)
    Uf, Wf = eval_dev(mrs, ctx, X, f, z, 0.05, 1.0, prec)
    Un, Wn = eval_dev(mrs, ctx, X, z, n, 0.05, 1.0, prec)
    for tot, a, b in ((U1, Uf, Un), (W1, Wf, Wn)):
        d = np.linalg.norm(tot - a - b, axis=1)
        scale = np.linalg.norm(a, axis=1) + np.linalg.norm(b, axis=1)
        say(f"superposition prec={prec}: max |d| / (|a| + |b|) = {np.max(d / scale):.3e}")
        assert np.all(d <= 10 * TOL[prec] * scale)


def test_host_entry_matches_device(mrs, ctx):
    X, f, n = _cloud(333, 4)
    U, W = mrs.mrs_eval_host(ctx, X, f, n, 0.03, 0.7, mrs.MRS_FP64)
    Ud, Wd = eval_dev(mrs, ctx, X, f, n, 0.03, 0.7, mrs.MRS_FP64)
    np.testing.assert_array_equal(U, Ud)
    np.testing.assert_array_equal(W, Wd)
    Uo, Wo = oracle.mrs_eval(X, f, n, 0.03, 0.7)
    assert oracle.rel_err(U, Uo) <= 1e-12


def test_invalid_arguments(mrs, ctx):
    X, f, n = _cloud(10, 5)
    with pytest.raises(mrs.MrsError) as ei:
        mrs.mrs_eval_host(ctx, X, f, n, -1.0, 1.0, mrs.MRS_FP64)
    assert ei.value.status == mrs.MRS_EINVAL
    with pytest.raises(mrs.MrsError):
        mrs.mrs_eval_host(ctx, X, f, n, 0.1, 0.0, mrs.MRS_FP64)
    with pytest.raises(mrs.MrsError):
        mrs.mrs_eval_host(ctx, X, f, n, 0.1, 1.0, 7)
    Xb = X.copy()
    Xb[3, 1] = np.nan
    with pytest.raises(mrs.MrsError):
        mrs.mrs_eval_host(ctx, Xb, f, n, 0.1, 1.0, mrs.MRS_FP64)
    # empty input is a no-op
    U, W = mrs.mrs_eval_host(ctx, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), 0.1, 1.0, mrs.MRS_FP64)
    assert U.shape == (0, 3)


@pytest.mark.parametrize("prec", [1, 0])
def test_overflowing_result_is_reported(mrs, ctx, prec):
    """Finite inputs whose velocities overflow (forces near the largest
    double) give MRS_ENUMERIC, not a silent inf; the context stays usable."""
    X, f, n = _cloud(10, 6)
    with pytest.raises(mrs.MrsError) as ei:
        mrs.mrs_eval_host(ctx, X, 1e307 * np.sign(f), n, 1e-3, 1.0, prec)
    assert ei.value.status == mrs.MRS_ENUMERIC
    U, W = mrs.mrs_eval_host(ctx, X, f, n, 0.03, 0.7, prec)
    Uo, Wo = oracle.mrs_eval(X, f, n, 0.03, 0.7)
    assert oracle.rel_err(U, Uo) <= TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
def test_ens256000_full_size_sampled(mrs, ctx, prec):
    """256,000 points, all targets evaluated on the GPU, 2,048 seeded targets
    checked one by one against the oracle."""
    e = synth.ens256000()
    sub = synth.ens256000_subset(e.N)
    say(f"ens256000 N={e.N} prec={prec}")
    U, W = eval_dev(mrs, ctx, e.X, e.f, e.n, e.eps, e.mu, prec)
    Uo, Wo = oracle.mrs_field(e.X[sub], e.X, e.f, e.n, e.eps, e.mu)
    eu, ew = oracle.rel_err(U[sub], Uo), oracle.rel_err(W[sub], Wo)
    say(f"  rel err (2048 sampled targets) U {eu:.3e} W {ew:.3e}")
    assert eu <= TOL[prec] and ew <= TOL[prec]
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(W))


@pytest.mark.parametrize("prec", [1, 0])
def test_autotune_and_every_config_parity(mrs, prec):
    """Every pair-kernel decomposition the tuner can pick gives the same
    result within tolerance; the tuned one is kept for the size class."""
    c = mrs.mrs_context_create(0)
    try:
        e = synth.filaments(20, 128, 4.0, 77)
        Uo, Wo = oracle.mrs_eval(e.X, e.f, e.n, e.eps, e.mu)
        for cfg in [(1, 1, 0), (0, 1, 1), (0, 1, 7), (0, 2, 3), (0, 2, 0), (0, 1, 40)]:
            mrs.mrs_tune_set(c, e.N, prec, *cfg)
            U, W = eval_dev(mrs, c, e.X, e.f, e.n, e.eps, e.mu, prec)
            eu, ew = oracle.rel_err(U, Uo), oracle.rel_err(W, Wo)
            say(f"cfg {cfg} prec={prec}: U {eu:.3e} W {ew:.3e}")
            assert eu <= TOL[prec] and ew <= TOL[prec], cfg
        best, ms = mrs.mrs_autotune(c, e.N, prec, 3)
        say(f"autotune N={e.N} prec={prec}: {best} {ms:.4f} ms")
        assert mrs.mrs_tune_get(c, e.N, prec)["mode"] == best["mode"]
        _check(mrs, c, e.X, e.f, e.n, e.eps, e.mu, prec, "tuned")
    finally:
        mrs.mrs_context_destroy(c)


def test_fp32c_tail_split_config(mrs):
    """Automatic FP32C configurations of grids of at least four blocks per
    compute unit split the last ~8% of every target tile's sources into
    quarter chunks (here 64 sources) dispatched last; FP64, small grids and
    explicit chunk counts keep equal chunks."""
    c = mrs.mrs_context_create(0)
    try:
        assert mrs.mrs_tune_get(c, 12800, 1)["chunks"] == 46 + 16
        assert mrs.mrs_tune_get(c, 12800, 0)["chunks"] == 50
        assert mrs.mrs_tune_get(c, 3200, 1)["chunks"] == 25
        mrs.mrs_tune_set(c, 12800, 1, 0, 1, 50)
        assert mrs.mrs_tune_get(c, 12800, 1)["chunks"] == 50
    finally:
        mrs.mrs_context_destroy(c)


def test_automatic_schedule_by_grid_depth(mrs):
    """Automatic tiled configurations of grids of at least 48 blocks per CU
    (24 for FP64 at two targets per lane) run the persistent schedule,
    shallower ones the hardware grid; a stored configuration keeps its own
    schedule."""
    c = mrs.mrs_context_create(0)
    try:
        sched = lambda n, p: mrs.mrs_tune_get(c, n, p)["schedule"]
        assert sched(12800, 1) == 0 and sched(12800, 0) == 0
        assert sched(25600, 1) == 0 and sched(25600, 0) == 0
        assert sched(51000, 1) == 1 and sched(51000, 0) == 1
        assert sched(256000, 1) == 1 and sched(256000, 0) == 1
        mrs.mrs_tune_set(c, 256000, 1, 0, 1, 0, 0)
        assert sched(256000, 1) == 0
    finally:
        mrs.mrs_context_destroy(c)


@pytest.mark.parametrize("tpl", [1, 2])
def test_fp32c_near_pairs_across_filaments(mrs, tpl):
    """Filaments crossing through one small region: near pairs (r < 4 eps)
    between points far apart in index order must still be taken in FP64."""
    c = mrs.mrs_context_create(0)
    try:
        rng = np.random.default_rng(31)
        F, M = 24, 128
        ds = 1.0 / M
        eps = 1.5 * ds
        X = []
        for _ in range(F):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            s = (np.arange(M) - M / 2) * ds
            X.append(np.array([5.0, 5.0, 5.0]) + rng.normal(scale=0.5 * eps, size=3) + s[:, None] * d[None, :])
        X = np.concatenate(X)
        f, n = rng.normal(size=X.shape), rng.normal(size=X.shape)
        mrs.mrs_tune_set(c, len(X), 1, 0, tpl, 0)
        _check(mrs, c, X, f, n, eps, 1.0, 1, f"crossing-tpl{tpl}")
    finally:
        mrs.mrs_context_destroy(c)


@pytest.mark.parametrize("tpl", [1, 2])
def test_fp32c_every_block_path_far_from_origin(mrs, tpl):
    """Straight filaments at separations from under 4 eps to a few hundred
    eps, 8,000 eps from the origin.  Pairs of a wave's targets and a 64-source
    block take all three paths of the tiled FP32C kernel (masked with the FP64
    near-pair rescan, far with the exact hi/lo separation, far relative to the
    block's anchor); every target must match the oracle, near the origin and
    shifted."""
    c = mrs.mrs_context_create(0)
    try:
        rng = np.random.default_rng(41)
        F, M = 40, 64
        ds = 1.0 / M
        eps = 1.5 * ds
        X = []
        for _ in range(F):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            X.append(rng.uniform(0.0, 200.0 * eps, 3) + (np.arange(M) * ds)[:, None] * d[None, :])
        X = np.concatenate(X)
        f, n = rng.normal(size=X.shape), rng.normal(size=X.shape)
        mrs.mrs_tune_set(c, len(X), 1, 0, tpl, 0)
        _check(mrs, c, X, f, n, eps, 1.0, 1, f"paths-tpl{tpl}")
        Xs = X + np.array([8000.0, -6000.0, 7000.0]) * eps
        _check(mrs, c, Xs, f, n, eps, 1.0, 1, f"paths-shifted-tpl{tpl}")
    finally:
        mrs.mrs_context_destroy(c)


@pytest.mark.parametrize("mode,tpl", [(0, 1), (0, 2), (2, 1)])
def test_fp32c_tiled_block_descriptors_small_and_ragged(mrs, mode, tpl):
    """The tiled FP32C kernels (one or two targets per lane, and the
    four-wave split) read a descriptor per aligned 64-point block (box,
    centre, anchored positions) written beside the records: by the pack
    kernel of a one-shot evaluation and by the rod launch of a resident
    ensemble.  Forced onto sizes below one block, one block and ragged last
    blocks, both routes match the oracle."""
    c = mrs.mrs_context_create(0)
    try:
        for N in (1, 2, 3, 5, 63, 64, 65, 300):
            X, f, n = _cloud(N, 900 + N, box=0.3)
            mrs.mrs_tune_set(c, N, 1, mode, tpl, 0)
            _check(mrs, c, X, f, n, 0.02, 1.0, 1, f"tiled-mode{mode}-tpl{tpl}")
        for nfil, M in ((1, 3), (1, 64), (5, 13), (4, 75), (3, 129)):
            e = synth.filaments(nfil, M, 2.0, 50 + nfil * M)
            mrs.mrs_tune_set(c, e.N, 1, mode, tpl, 0)
            h = mrs.mrs_ensemble_create(c, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod_of(mrs, e.rod()))
            try:
                mrs.mrs_ensemble_eval(c, h, mrs.MRS_FP32C, False)
                _, _, U, W = mrs.mrs_ensemble_get(c, h)
            finally:
                mrs.mrs_ensemble_destroy(h)
            Uo, Wo = oracle.mrs_eval(e.X, e.f, e.n, e.eps, e.mu)
            eu, ew = oracle.rel_err(U, Uo), oracle.rel_err(W, Wo)
            say(f"ensemble {nfil}x{M} mode={mode} tpl={tpl}: U {eu:.3e} W {ew:.3e}")
            assert eu <= TOL[1] and ew <= TOL[1], (nfil, M)
    finally:
        mrs.mrs_context_destroy(c)


@pytest.mark.parametrize("cfg", [None, (0, 2, 0), (2, 1, 0)])
def test_fp32c_descriptors_follow_the_state(mrs, cfg):
    """The block descriptors (boxes, centres, anchored positions) are
    rewritten with the records at every evaluation of a resident ensemble:
    after its state moves to another geometry and then far from the origin,
    each evaluation matches the oracle of the new state (a stale centre
    would shift every anchored separation by the distance moved)."""
    c = mrs.mrs_context_create(0)
    try:
        e = synth.filaments(20, 128, 4.0, 201)  # 2,560 points: tiled kernels
        e2 = synth.filaments(20, 128, 4.0, 202)
        if cfg is not None:
            mrs.mrs_tune_set(c, e.N, 1, *cfg)
        h = mrs.mrs_ensemble_create(c, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod_of(mrs, e.rod()))
        try:
            for tag, X, D in (("initial", e.X, e.D), ("moved", e2.X, e2.D),
                              ("shifted", e2.X + np.array([40.0, -25.0, 60.0]), e2.D), ("back", e.X, e.D)):
                mrs.mrs_ensemble_set_state(c, h, X, D)
                mrs.mrs_ensemble_eval(c, h, mrs.MRS_FP32C, False)
                _, _, U, W = mrs.mrs_ensemble_get(c, h)
                Uo, Wo = oracle.mrs_eval(X, e.f, e.n, e.eps, e.mu)
                eu, ew = oracle.rel_err(U, Uo), oracle.rel_err(W, Wo)
                say(f"{tag} cfg={cfg}: U {eu:.3e} W {ew:.3e}")
                assert eu <= TOL[1] and ew <= TOL[1], (tag, cfg)
        finally:
            mrs.mrs_ensemble_destroy(h)
    finally:
        mrs.mrs_context_destroy(c)
