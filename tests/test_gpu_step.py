"""GPU parity of resident-ensemble evaluation and time steps against the FP64
oracle (Sec. III.B.3, Eqs. newx, newD; RK4 fine propagator of Sec. III.A).

Trajectories of two FP64 codes separate by far more than 1e-12 over 100
steps (the dynamics amplify rounding), so the tolerance is enforced on each
step from an identical state ("teacher forcing"): every step, the oracle is
given the GPU's current state and both advance one step.  Per step, the
displacement X1 - X0 is compared with the paper's relative error form (after
removing the rounding of the stored positions themselves, see step_err) and
the frames by their largest per-point difference.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rod_of, say, step_err

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


def _create(mrs, ctx, e, rod=None):
    rod = rod or e.rod()
    return mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod_of(mrs, rod))


def _frame_err(Da, Db):
    return float(np.max(np.linalg.norm((Da - Db).reshape(-1, 3, 3), axis=2)))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("elastic", [True, False])
def test_ensemble_eval(mrs, ctx, prec, elastic):
    e = synth.ens12800()
    ens = _create(mrs, ctx, e)
    try:
        mrs.mrs_ensemble_eval(ctx, ens, prec, elastic)
        _, _, U, W = mrs.mrs_ensemble_get(ctx, ens)
        Uo, Wo = oracle.velocities(e.offsets, e.X, e.D, e.rod(), e.f, e.n, e.eps, e.mu, elastic)
        eu, ew = oracle.rel_err(U, Uo), oracle.rel_err(W, Wo)
        say(f"ensemble eval prec={prec} elastic={elastic}: U {eu:.3e} W {ew:.3e}")
        assert eu <= TOL[prec] and ew <= TOL[prec]
    finally:
        mrs.mrs_ensemble_destroy(ens)


@pytest.mark.parametrize("prec", [0, 1])
def test_rod64_euler_teacher_forced(mrs, ctx, prec):
    """One filament of 64 points, 100 forward-Euler steps at dt = 1e-4."""
    e = synth.rod64()
    rod = e.rod()
    dt = 1e-4
    ens = _create(mrs, ctx, e)
    worst = [0.0, 0.0, 0.0]
    try:
        X, D, _, _ = mrs.mrs_ensemble_get(ctx, ens)
        for step in range(100):
            Xo, Do, Uo, Wo = oracle.step(e.offsets, X, D, rod, e.f, e.n, e.eps, e.mu, oracle.EULER, dt, 1)
            mrs.mrs_ensemble_step(ctx, ens, mrs.MRS_EULER, dt, 1, prec, True)
            X1, D1, U, W = mrs.mrs_ensemble_get(ctx, ens)
            ex = step_err(X1, Xo, X)
            ed = _frame_err(D1, Do)
            eu = max(oracle.rel_err(U, Uo), oracle.rel_err(W, Wo))
            worst = [max(worst[0], ex), max(worst[1], ed), max(worst[2], eu)]
            assert ex <= TOL[prec] and ed <= TOL[prec] and eu <= TOL[prec], (step, ex, ed, eu)
            X, D = X1, D1
        say(f"rod64 euler prec={prec}: worst step dX {worst[0]:.3e} D {worst[1]:.3e} U/W {worst[2]:.3e}")
        # frames stay orthonormal
        Dm = D.reshape(-1, 3, 3)
        assert np.abs(np.einsum("kij,klj->kil", Dm, Dm) - np.eye(3)).max() < 1e-14
    finally:
        mrs.mrs_ensemble_destroy(ens)


@pytest.mark.parametrize("integ", ["RK4", "RK2"])
@pytest.mark.parametrize("prec", [0, 1])
def test_rk_teacher_forced(mrs, ctx, prec, integ):
    """Slice base geometry (32 filaments x 100 points), RK4 / RK2 at dt = 1e-5."""
    base, slices = synth.slices(n_slices=1)
    e = slices[0]
    rod = e.rod()
    dt = 1e-5
    ens = _create(mrs, ctx, e)
    try:
        X, D, _, _ = mrs.mrs_ensemble_get(ctx, ens)
        for step in range(3):
            Xo, Do, _, _ = oracle.step(e.offsets, X, D, rod, e.f, e.n, e.eps, e.mu, getattr(oracle, integ), dt, 1)
            mrs.mrs_ensemble_step(ctx, ens, getattr(mrs, "MRS_" + integ), dt, 1, prec, True)
            X1, D1, _, _ = mrs.mrs_ensemble_get(ctx, ens)
            ex, ed = step_err(X1, Xo, X), _frame_err(D1, Do)
            say(f"{integ} prec={prec} step {step}: dX {ex:.3e} D {ed:.3e}")
            assert ex <= TOL[prec] and ed <= TOL[prec]
            X, D = X1, D1
    finally:
        mrs.mrs_ensemble_destroy(ens)


def test_free_running_rod64_fp64(mrs, ctx):
    """100 free-running Euler steps: reported against the oracle's own
    spread under a 1-ulp perturbation of the input."""
    e = synth.rod64()
    ens = _create(mrs, ctx, e)
    try:
        mrs.mrs_ensemble_step(ctx, ens, mrs.MRS_EULER, 1e-4, 100, mrs.MRS_FP64, True)
        X, D, _, _ = mrs.mrs_ensemble_get(ctx, ens)
    finally:
        mrs.mrs_ensemble_destroy(ens)
    Xo, Do, _, _ = oracle.step(e.offsets, e.X, e.D, e.rod(), e.f, e.n, e.eps, e.mu, oracle.EULER, 1e-4, 100)
    Xp, _, _, _ = oracle.step(e.offsets, np.nextafter(e.X, np.inf), e.D, e.rod(), e.f, e.n, e.eps, e.mu,
                              oracle.EULER, 1e-4, 100)
    gpu = oracle.rel_err(X - e.X, Xo - e.X)
    spread = oracle.rel_err(Xp - e.X, Xo - e.X)
    say(f"free-running 100 Euler steps: GPU vs oracle {gpu:.3e}, oracle 1-ulp spread {spread:.3e}")
    assert gpu <= max(1e3 * spread, 1e-9)


def test_invalid_step_arguments(mrs, ctx):
    e = synth.rod64()
    ens = _create(mrs, ctx, e)
    try:
        with pytest.raises(mrs.MrsError):
            mrs.mrs_ensemble_step(ctx, ens, 3, 1e-4, 1)
        with pytest.raises(mrs.MrsError):
            mrs.mrs_ensemble_step(ctx, ens, mrs.MRS_EULER, float("nan"), 1)
        with pytest.raises(mrs.MrsError):
            mrs.mrs_ensemble_step(ctx, ens, mrs.MRS_EULER, 1e-4, -1)
        mrs.mrs_ensemble_step(ctx, ens, mrs.MRS_EULER, 1e-4, 0)  # no-op
        X, _, _, _ = mrs.mrs_ensemble_get(ctx, ens)
        np.testing.assert_array_equal(X, e.X)
    finally:
        mrs.mrs_ensemble_destroy(ens)
    with pytest.raises(mrs.MrsError):
        mrs.mrs_ensemble_create(ctx, np.array([0, 5, 3], dtype=np.int32), e.X, e.D, None, None, e.eps, e.mu,
                                rod_of(mrs, e.rod()))


def _shuffle_filaments(e, seed):
    """The same ensemble with its filaments listed in another order: the
    offsets, point arrays and the point index map new -> old."""
    F = len(e.offsets) - 1
    order = np.random.default_rng(seed).permutation(F)
    idx = np.concatenate([np.arange(e.offsets[f], e.offsets[f + 1]) for f in order])
    sizes = np.diff(e.offsets)[order]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    return off, idx


@pytest.mark.parametrize("prec", [0, 1])
def test_caller_filament_order_does_not_matter(mrs, ctx, prec):
    """Filaments are stored in a spatial order of the library's choosing and
    every result comes back in the caller's order: the same filaments given
    in another order give the same U, Omega and the same state after steps,
    bit for bit (the stored order, hence every sum, is the same)."""
    e = synth.filaments(37, 51, 6.0, 41)  # filaments shorter than a 64-point block
    off, idx = _shuffle_filaments(e, 5)
    a = _create(mrs, ctx, e)
    b = mrs.mrs_ensemble_create(ctx, off, e.X[idx], e.D[idx], e.f[idx], e.n[idx], e.eps, e.mu,
                                rod_of(mrs, e.rod()))
    try:
        for h in (a, b):
            mrs.mrs_ensemble_eval(ctx, h, prec, True)
        _, _, Ua, Wa = mrs.mrs_ensemble_get(ctx, a)
        _, _, Ub, Wb = mrs.mrs_ensemble_get(ctx, b)
        np.testing.assert_array_equal(Ub, Ua[idx])
        np.testing.assert_array_equal(Wb, Wa[idx])
        Uo, Wo = oracle.velocities(e.offsets, e.X, e.D, e.rod(), e.f, e.n, e.eps, e.mu, True)
        assert oracle.rel_err(Ua, Uo) <= TOL[prec] and oracle.rel_err(Wa, Wo) <= TOL[prec]
        for h in (a, b):
            mrs.mrs_ensemble_step(ctx, h, mrs.MRS_RK2, 1e-5, 3, prec, True)
        Xa, Da, _, _ = mrs.mrs_ensemble_get(ctx, a)
        Xb, Db, _, _ = mrs.mrs_ensemble_get(ctx, b)
        np.testing.assert_array_equal(Xb, Xa[idx])
        np.testing.assert_array_equal(Db, Da[idx])
        # state written in the caller's order reads back unchanged
        mrs.mrs_ensemble_set_state(ctx, b, e.X[idx], e.D[idx])
        Xr, Dr, _, _ = mrs.mrs_ensemble_get(ctx, b)
        np.testing.assert_array_equal(Xr, e.X[idx])
        np.testing.assert_array_equal(Dr, e.D[idx])
    finally:
        mrs.mrs_ensemble_destroy(a)
        mrs.mrs_ensemble_destroy(b)
