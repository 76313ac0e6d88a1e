"""Parareal on one device against the oracle's Parareal and the serial fine
solution (Sec. II.D)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rod_of, say

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


def _ens(mrs, ctx, e):
    return mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod_of(mrs, e.rod()))


def test_parareal_full_iterations_equal_serial_fine(mrs, ctx):
    e = synth.filaments(4, 50, 2.0, 21)
    ns, steps, dt = 5, 8, 1e-5
    a, b = _ens(mrs, ctx, e), _ens(mrs, ctx, e)
    try:
        it, hist = mrs.mrs_parareal(ctx, a, ns, mrs.MRS_RK4, dt, steps, 1, ns, 0.0, mrs.MRS_FP64, True)
        mrs.mrs_ensemble_step(ctx, b, mrs.MRS_RK4, dt, ns * steps, mrs.MRS_FP64, True)
        Xa, Da, _, _ = mrs.mrs_ensemble_get(ctx, a)
        Xb, Db, _, _ = mrs.mrs_ensemble_get(ctx, b)
        say(f"parareal {it} iterations, increments {hist}")
        assert it == ns
        np.testing.assert_array_equal(Xa, Xb)
        np.testing.assert_array_equal(Da, Db)
    finally:
        mrs.mrs_ensemble_destroy(a)
        mrs.mrs_ensemble_destroy(b)


@pytest.mark.parametrize("integ", ["RK2", "RK4"])
def test_parareal_matches_oracle(mrs, ctx, integ):
    e = synth.filaments(2, 16, 1.0, 9)
    ns, steps, dt, iters = 4, 10, 2e-4, 3
    h = _ens(mrs, ctx, e)
    try:
        it, hist = mrs.mrs_parareal(ctx, h, ns, getattr(mrs, "MRS_" + integ), dt, steps, 1, iters, 0.0,
                                    mrs.MRS_FP64, True)
        X, D, _, _ = mrs.mrs_ensemble_get(ctx, h)
    finally:
        mrs.mrs_ensemble_destroy(h)
    U, ohist = oracle.parareal(e.offsets, e.X, e.D, e.rod(), e.f, e.n, e.eps, e.mu, ns, getattr(oracle, integ), dt,
                               steps, 1, iters)
    say(f"{integ}: gpu increments {hist} oracle {ohist}")
    assert it == iters
    np.testing.assert_allclose(hist, ohist, rtol=1e-8)
    disp = np.linalg.norm(U[ns][0] - e.X, axis=1)
    assert np.max(np.linalg.norm(X - U[ns][0], axis=1) / disp) <= 1e-9
    assert np.abs(D - U[ns][1]).max() <= 1e-9


def test_parareal_converges_and_stops_at_tolerance(mrs, ctx):
    """Slice base geometry (32 filaments x 100 points) with the external
    torques scaled by 1e-2 (smooth enough for a coarse Euler propagator):
    the increments fall by orders of
    magnitude per iteration and the iteration stops at the tolerance."""
    base, slices = synth.slices(n_slices=1)
    e = slices[0]
    h = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, 1e-2 * e.n, e.eps, e.mu, rod_of(mrs, e.rod()))
    try:
        it, hist = mrs.mrs_parareal(ctx, h, 8, mrs.MRS_RK4, 1e-5, 20, 2, 8, 1e-11, mrs.MRS_FP64, True)
        say(f"32 x 100 slice base (torques x 1e-2), 8 slices: {it} iterations, increments {hist}")
        assert it < 8 and hist[-1] <= 1e-11
        assert np.all(np.diff(np.log10(hist)) < -1.0)
    finally:
        mrs.mrs_ensemble_destroy(h)
    h = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, 1e-2 * e.n, e.eps, e.mu, rod_of(mrs, e.rod()))
    try:
        it, hist = mrs.mrs_parareal(ctx, h, 8, mrs.MRS_RK4, 1e-5, 20, 2, 8, 1e-6, mrs.MRS_FP32C, True)
        say(f"FP32C: {it} iterations, increments {hist}")
        assert hist[-1] <= 1e-6
    finally:
        mrs.mrs_ensemble_destroy(h)


def test_parareal_invalid_arguments(mrs, ctx):
    e = synth.filaments(2, 16, 1.0, 9)
    h = _ens(mrs, ctx, e)
    try:
        with pytest.raises(mrs.MrsError):
            mrs.mrs_parareal(ctx, h, 2, mrs.MRS_RK4, 1e-5, 4, 1, 3)  # max_iter > n_slices
        with pytest.raises(mrs.MrsError):
            mrs.mrs_parareal(ctx, h, 2, mrs.MRS_RK4, 1e-5, 0, 1, 2)
    finally:
        mrs.mrs_ensemble_destroy(h)


def _run_both(mrs, ctx, make, args, group):
    """The regular and the pipelined schedule on fresh copies of one ensemble."""
    a, b = make(), make()
    try:
        it_r, h_r = mrs.mrs_parareal(ctx, a, *args)
        it_p, h_p = mrs.mrs_parareal_pipelined(ctx, b, *args, group=group)
        Xa, Da, _, _ = mrs.mrs_ensemble_get(ctx, a)
        Xb, Db, _, _ = mrs.mrs_ensemble_get(ctx, b)
        ta, tb = mrs.mrs_ensemble_get_time(ctx, a), mrs.mrs_ensemble_get_time(ctx, b)
    finally:
        mrs.mrs_ensemble_destroy(a)
        mrs.mrs_ensemble_destroy(b)
    return (it_r, h_r, Xa, Da, ta), (it_p, h_p, Xb, Db, tb)


def _assert_same(r, p):
    assert r[0] == p[0]
    np.testing.assert_array_equal(r[1], p[1])
    np.testing.assert_array_equal(r[2], p[2])
    np.testing.assert_array_equal(r[3], p[3])
    assert r[4] == p[4]


@pytest.mark.parametrize("prec", ["FP64", "FP32C"])
@pytest.mark.parametrize("group", [1, 2, 0, 5])
def test_pipelined_equals_regular_all_iterations(mrs, ctx, prec, group):
    """Sec. II.D: the pipelined schedule computes the regular iterates bit for
    bit, for every group size (1, 2, the default, all slices)."""
    e = synth.filaments(4, 50, 2.0, 21)
    ns = 5
    args = (ns, mrs.MRS_RK4, 1e-5, 8, 1, ns, 0.0, getattr(mrs, "MRS_" + prec), True)
    r, p = _run_both(mrs, ctx, lambda: _ens(mrs, ctx, e), args, group)
    say(f"{prec} group {group}: {p[0]} iterations, increments {p[1]}")
    assert p[0] == ns
    _assert_same(r, p)


@pytest.mark.parametrize("group", [1, 3])
def test_pipelined_stops_where_regular_stops(mrs, ctx, group):
    """With a tolerance the pipelined schedule stops at the same iteration
    with the same increments and state (the fine groups of the next
    iteration start only once the increment exceeds the tolerance)."""
    base, slices = synth.slices(n_slices=1)
    e = slices[0]
    make = lambda: mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, 1e-2 * e.n, e.eps, e.mu,
                                           rod_of(mrs, e.rod()))
    args = (8, mrs.MRS_RK4, 1e-5, 20, 2, 8, 1e-11, mrs.MRS_FP64, True)
    r, p = _run_both(mrs, ctx, make, args, group)
    say(f"group {group}: {p[0]} iterations, increments {p[1]}")
    assert p[0] < 8 and p[1][-1] <= 1e-11
    _assert_same(r, p)


def test_pipelined_invalid_group(mrs, ctx):
    e = synth.filaments(2, 16, 1.0, 9)
    h = _ens(mrs, ctx, e)
    try:
        with pytest.raises(mrs.MrsError):
            mrs.mrs_parareal_pipelined(ctx, h, 3, mrs.MRS_RK4, 1e-5, 4, 1, 3, group=4)
        with pytest.raises(mrs.MrsError):
            mrs.mrs_parareal_pipelined(ctx, h, 3, mrs.MRS_RK4, 1e-5, 4, 1, 3, group=-1)
        with pytest.raises(mrs.MrsError):
            mrs.mrs_parareal_pipelined(ctx, h, 2, mrs.MRS_RK4, 1e-5, 4, 1, 3)  # max_iter > n_slices
    finally:
        mrs.mrs_ensemble_destroy(h)


def test_workers_kept_between_calls(mrs, ctx):
    """Repeated calls on one ensemble reuse its Parareal workers (and their
    plans and graphs): from the same start state they give the same bits,
    with more slices than before too; after the loads change the workers
    are rebuilt and the result is that of a fresh ensemble with the new
    loads; destroying the ensemble releases its workers."""
    e = synth.filaments(4, 50, 2.0, 31)
    rng = np.random.default_rng(32)
    f2 = rng.normal(size=e.X.shape)
    ns, steps, dt = 4, 6, 1e-5
    h = _ens(mrs, ctx, e)
    try:
        runs = []
        for k, nsl in enumerate((ns, ns, ns + 2, ns)):
            mrs.mrs_ensemble_set_state(ctx, h, e.X, e.D)
            mrs.mrs_ensemble_set_time(ctx, h, 0.0)
            it, hist = mrs.mrs_parareal(ctx, h, nsl, mrs.MRS_RK4, dt, steps, 1, 2, 0.0, mrs.MRS_FP32C, True)
            X, D, _, _ = mrs.mrs_ensemble_get(ctx, h)
            runs.append((nsl, X, D, hist))
            say(f"call {k}: {nsl} slices, increments {hist}")
        for a, b in ((0, 1), (0, 3)):
            assert np.array_equal(runs[a][1], runs[b][1]) and np.array_equal(runs[a][2], runs[b][2])
            assert np.array_equal(runs[a][3], runs[b][3])
        # new loads: same result as a fresh ensemble created with them
        mrs.mrs_ensemble_set_external(ctx, h, f2, e.n)
        mrs.mrs_ensemble_set_state(ctx, h, e.X, e.D)
        mrs.mrs_ensemble_set_time(ctx, h, 0.0)
        mrs.mrs_parareal(ctx, h, ns, mrs.MRS_RK4, dt, steps, 1, 2, 0.0, mrs.MRS_FP32C, True)
        Xh, Dh, _, _ = mrs.mrs_ensemble_get(ctx, h)
        g = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, f2, e.n, e.eps, e.mu, rod_of(mrs, e.rod()))
        try:
            mrs.mrs_parareal(ctx, g, ns, mrs.MRS_RK4, dt, steps, 1, 2, 0.0, mrs.MRS_FP32C, True)
            Xg, Dg, _, _ = mrs.mrs_ensemble_get(ctx, g)
        finally:
            mrs.mrs_ensemble_destroy(g)
        assert np.array_equal(Xh, Xg) and np.array_equal(Dh, Dg)
        assert not np.array_equal(Xh, runs[0][1])
    finally:
        mrs.mrs_ensemble_destroy(h)
