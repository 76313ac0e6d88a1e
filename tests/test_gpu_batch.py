"""Batched launches: many ensembles (or the fine-propagator time slices of one
Parareal iteration) advanced by one launch sequence, optionally replayed
from a HIP graph.  Each ensemble's result must be identical alone and in the
batch, and graph replays identical to eager launches."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rod_of, say, step_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mrs():
    import paper_2604_12083_amd as m

    return m


@pytest.fixture(scope="module")
def ctx(mrs):
    c = mrs.mrs_context_create(0)
    yield c
    mrs.mrs_context_destroy(c)


def _create(mrs, ctx, e):
    return mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod_of(mrs, e.rod()))


@pytest.mark.parametrize("prec", [1, 0])
def test_batch_equals_alone_mixed_sizes(mrs, ctx, prec):
    ens_in = [synth.filaments(F, M, 10.0, 40 + i) for i, (F, M) in
              enumerate([(4, 64), (32, 100), (9, 200), (1, 37), (60, 128)])]
    alone, batch = [], []
    try:
        for e in ens_in:
            a = _create(mrs, ctx, e)
            mrs.mrs_ensemble_step(ctx, a, mrs.MRS_RK4, 1e-5, 3, prec, True)
            alone.append(a)
        batch = [_create(mrs, ctx, e) for e in ens_in]
        mrs.mrs_batch_step(ctx, batch, mrs.MRS_RK4, 1e-5, 3, prec, True, use_graph=False)
        for i, (a, b) in enumerate(zip(alone, batch)):
            Xa, Da, Ua, Wa = mrs.mrs_ensemble_get(ctx, a)
            Xb, Db, Ub, Wb = mrs.mrs_ensemble_get(ctx, b)
            np.testing.assert_array_equal(Xa, Xb)
            np.testing.assert_array_equal(Da, Db)
            np.testing.assert_array_equal(Ua, Ub)
        say(f"batch == alone for {len(ens_in)} ensembles (prec={prec})")
    finally:
        for h in alone + batch:
            mrs.mrs_ensemble_destroy(h)


@pytest.mark.parametrize("prec", [1, 0])
def test_graph_replays_equal_eager(mrs, ctx, prec):
    base, slices = synth.slices(n_slices=4)
    g = [_create(mrs, ctx, e) for e in slices]
    h = [_create(mrs, ctx, e) for e in slices]
    try:
        for rep in range(3):
            mrs.mrs_batch_step(ctx, g, mrs.MRS_RK4, 1e-5, 2, prec, True, use_graph=True)
            mrs.mrs_batch_step(ctx, h, mrs.MRS_RK4, 1e-5, 2, prec, True, use_graph=False)
            # eager work and synchronisation between replays
            mrs.mrs_ensemble_eval(ctx, h[0], prec, True)
            for a, b in zip(g, h):
                Xa, Da, _, _ = mrs.mrs_ensemble_get(ctx, a)
                Xb, Db, _, _ = mrs.mrs_ensemble_get(ctx, b)
                np.testing.assert_array_equal(Xa, Xb)
                np.testing.assert_array_equal(Da, Db)
        say(f"graph replays == eager (prec={prec})")
    finally:
        for x in g + h:
            mrs.mrs_ensemble_destroy(x)


def test_batched_slices_parity_one_step(mrs, ctx):
    """The 16 slices of 32 filaments x 100 points: one batched RK4 step of
    every slice (all 16) against the oracle's step from the same state."""
    base, slices = synth.slices(n_slices=16)
    hs = [_create(mrs, ctx, e) for e in slices]
    try:
        mrs.mrs_batch_step(ctx, hs, mrs.MRS_RK4, 1e-5, 1, mrs.MRS_FP32C, True, use_graph=True)
        worst = 0.0
        for i in range(len(slices)):
            e = slices[i]
            X1, D1, _, _ = mrs.mrs_ensemble_get(ctx, hs[i])
            Xo, Do, _, _ = oracle.step(e.offsets, e.X, e.D, e.rod(), e.f, e.n, e.eps, e.mu, oracle.RK4, 1e-5, 1)
            ex = step_err(X1, Xo, e.X)
            worst = max(worst, ex)
            assert ex <= 1e-5
        say(f"slices batched RK4 step: worst dX rel err {worst:.3e}")
    finally:
        for x in hs:
            mrs.mrs_ensemble_destroy(x)
