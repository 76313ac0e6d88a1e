"""Pair-kernel schedules and decompositions beyond the default: the persistent
schedule (a resident grid whose blocks claim work items from a counter that
resets itself at the end of every launch) and the four-wave source split
(tiles of 64 targets whose four waves share the targets and split the
sources).  Every configuration matches the FP64 oracle (Eq. true_err form:
1e-12 FP64, 1e-5 FP32C); a schedule changes no result at all (each work item
writes its own partial sums), also over graph replays with eager work
between them."""
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


# (mode, targets per lane, chunks, schedule); mode 2 (four-wave split) is
# FP32C only and falls back to the tiled kernel in FP64
CFGS = [(0, 1, 0, 0), (0, 1, 0, 1), (0, 2, 3, 1), (0, 1, 40, 1), (2, 1, 0, 0), (2, 1, 7, 0), (2, 1, 0, 1),
        (2, 1, 1, 1)]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("N", [2560, 3001])
def test_configs_match_oracle_and_schedules_match_each_other(mrs, prec, N):
    c = mrs.mrs_context_create(0)
    try:
        if N == 2560:
            e = synth.filaments(20, 128, 4.0, 77)
            X, f, n, eps = e.X, e.f, e.n, e.eps
        else:
            rng = np.random.default_rng(N)
            X, f, n, eps = rng.uniform(0, 0.6, (N, 3)), rng.normal(size=(N, 3)), rng.normal(size=(N, 3)), 0.01
        Uo, Wo = oracle.mrs_eval(X, f, n, eps, 1.0)
        got = {}
        for cfg in CFGS:
            mrs.mrs_tune_set(c, N, prec, *cfg)
            U, W = eval_dev(mrs, c, X, f, n, eps, 1.0, prec)
            eu, ew = oracle.rel_err(U, Uo), oracle.rel_err(W, Wo)
            say(f"N={N} cfg {cfg} prec={prec}: U {eu:.3e} W {ew:.3e} chunks {mrs.mrs_tune_get(c, N, prec)['chunks']}")
            assert eu <= TOL[prec] and ew <= TOL[prec], cfg
            got[cfg] = (U, W)
        # same decomposition, other schedule: identical sums
        for a, b in (((0, 1, 0, 0), (0, 1, 0, 1)), ((2, 1, 0, 0), (2, 1, 0, 1))):
            assert np.array_equal(got[a][0], got[b][0]) and np.array_equal(got[a][1], got[b][1]), (a, b)
    finally:
        mrs.mrs_context_destroy(c)


@pytest.mark.parametrize("mode", [0, 2])
def test_persistent_batch_graph_replays_equal_eager(mrs, mode):
    """Three ensembles stepped together on the persistent schedule: HIP-graph
    replays (the work-queue counters must be back at zero after every
    launch) give bitwise the eager sequence, with eager work between the
    replays, and match the same steps on the grid schedule."""
    c = mrs.mrs_context_create(0)
    try:
        es = [synth.filaments(24, 100, 6.0, 300 + k) for k in range(3)]
        N = es[0].N
        mrs.mrs_tune_set(c, N, mrs.MRS_FP32C, mode, 1, 0, 1)
        mk = lambda: [mrs.mrs_ensemble_create(c, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod_of(mrs, e.rod()))
                      for e in es]
        g, q = mk(), mk()
        try:
            for rep in range(3):
                mrs.mrs_batch_step(c, g, mrs.MRS_RK4, 1e-5, 4, mrs.MRS_FP32C, True, use_graph=True)
                mrs.mrs_batch_step(c, q, mrs.MRS_RK4, 1e-5, 4, mrs.MRS_FP32C, True, use_graph=False)
                mrs.mrs_ensemble_eval(c, q[0], mrs.MRS_FP32C, True)  # eager work between replays
                for a, b in zip(g, q):
                    Xa, Da, _, _ = mrs.mrs_ensemble_get(c, a)
                    Xb, Db, _, _ = mrs.mrs_ensemble_get(c, b)
                    assert np.array_equal(Xa, Xb) and np.array_equal(Da, Db), rep
                say(f"mode {mode} replay {rep}: graph == eager")
            mrs.mrs_tune_set(c, N, mrs.MRS_FP32C, mode, 1, 0, 0)
            grid = mk()
            try:
                mrs.mrs_batch_step(c, grid, mrs.MRS_RK4, 1e-5, 12, mrs.MRS_FP32C, True, use_graph=True)
                for a, b in zip(g, grid):
                    assert np.array_equal(mrs.mrs_ensemble_get(c, a)[0], mrs.mrs_ensemble_get(c, b)[0])
            finally:
                for h in grid:
                    mrs.mrs_ensemble_destroy(h)
        finally:
            for h in g + q:
                mrs.mrs_ensemble_destroy(h)
    finally:
        mrs.mrs_context_destroy(c)
