"""The boundary's contract beyond plain parity: external loads replaced after
creation (the loads f, n of Eq. superposition), non-finite results reported
as MRS_ENUMERIC by every call that checks them, and one-shot evaluations
queued on different streams without a host synchronisation between them.

Parity bar as everywhere: the paper's relative error (Eq. true_err),
1e-12 for MRS_FP64 and 1e-5 for MRS_FP32C, against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import dev, rod_of, say

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


def _velocities(e, f, n, include_elastic):
    return oracle.velocities(e.offsets, e.X, e.D, e.rod(), f, n, e.eps, e.mu, include_elastic=include_elastic)


@pytest.mark.parametrize("prec", [0, 1])
def test_set_external_then_eval(mrs, ctx, prec):
    """An ensemble created without loads takes them later; replacing them
    (and zeroing either) gives the oracle's velocities for the new loads,
    with and without the elastic forces."""
    e = synth.filaments(12, 100, 4.0, 71)
    rng = np.random.default_rng(72)
    f2, n2 = rng.normal(size=e.X.shape), rng.normal(size=e.X.shape)
    h = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, None, None, e.eps, e.mu, rod_of(mrs, e.rod()))
    try:
        cases = [("loads after creation", e.f, e.n, False), ("same, with rod forces", e.f, e.n, True),
                 ("replaced", f2, n2, True), ("torques zeroed", f2, None, False), ("forces zeroed", None, n2, True)]
        for tag, f, n, el in cases:
            say(f"set_external {tag} prec={prec}")
            mrs.mrs_ensemble_set_external(ctx, h, f, n)
            mrs.mrs_ensemble_eval(ctx, h, prec, el)
            _, _, U, W = mrs.mrs_ensemble_get(ctx, h)
            z = np.zeros_like(e.X)
            Uo, Wo = _velocities(e, z if f is None else f, z if n is None else n, el)
            eu, ew = oracle.rel_err(U, Uo), oracle.rel_err(W, Wo)
            say(f"  rel err U {eu:.3e} W {ew:.3e}")
            assert eu <= TOL[prec] and ew <= TOL[prec], (tag, eu, ew)
        # no loads and no rod forces: exactly zero velocities
        mrs.mrs_ensemble_set_external(ctx, h, None, None)
        mrs.mrs_ensemble_eval(ctx, h, prec, False)
        _, _, U, W = mrs.mrs_ensemble_get(ctx, h)
        assert not U.any() and not W.any()
    finally:
        mrs.mrs_ensemble_destroy(h)


def test_set_external_steps_match_oracle(mrs, ctx):
    """Loads set after creation are held constant through steps (teacher-forced
    against the oracle's step from the same state)."""
    e = synth.rod64()
    h = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, None, None, e.eps, e.mu, rod_of(mrs, e.rod()))
    try:
        mrs.mrs_ensemble_set_external(ctx, h, e.f, e.n)
        X0, D0 = e.X, e.D
        for k in range(3):
            mrs.mrs_ensemble_step(ctx, h, mrs.MRS_EULER, 1e-4, 1, mrs.MRS_FP64, True)
            X1, D1, _, _ = mrs.mrs_ensemble_get(ctx, h)
            Xo, Do, _, _ = oracle.step(e.offsets, X0, D0, e.rod(), e.f, e.n, e.eps, e.mu, oracle.EULER, 1e-4, 1)
            ex, ed = oracle.rel_err(X1, Xo), oracle.rel_err(D1, Do)
            say(f"step {k}: X {ex:.3e} D {ed:.3e}")
            assert ex <= 1e-12 and ed <= 1e-12
            X0, D0 = X1, D1
    finally:
        mrs.mrs_ensemble_destroy(h)


def test_set_external_rejects_non_finite(mrs, ctx):
    e = synth.rod64()
    h = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, None, None, e.eps, e.mu, rod_of(mrs, e.rod()))
    try:
        bad = e.f.copy()
        bad[5, 1] = np.nan
        with pytest.raises(mrs.MrsError) as ex:
            mrs.mrs_ensemble_set_external(ctx, h, bad, None)
        assert ex.value.status == mrs.MRS_EINVAL
    finally:
        mrs.mrs_ensemble_destroy(h)


def _numeric(mrs, fn):
    with pytest.raises(mrs.MrsError) as ex:
        fn()
    assert ex.value.status == mrs.MRS_ENUMERIC, ex.value
    say(f"  MRS_ENUMERIC: {ex.value}")


def test_enumeric_overflowing_records_and_steps(mrs, ctx):
    """Finite inputs whose results overflow: forces of 1e38 exceed single
    precision once scaled by 1/eps (FP32C records), and a step of 1e307 sends
    the positions past the double range.  Every checked call reports it, the
    results are still returned, and the next finite call is MRS_OK again."""
    e = synth.rod64()
    rod = rod_of(mrs, e.rod())
    big = np.full_like(e.f, 1e38)
    h = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, big, e.n, e.eps, e.mu, rod)
    ok = mrs.mrs_ensemble_create(ctx, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod)
    try:
        say("FP32C eval with 1e38 forces")
        _numeric(mrs, lambda: mrs.mrs_ensemble_eval(ctx, h, mrs.MRS_FP32C, False))
        _numeric(mrs, lambda: mrs.mrs_ensemble_get(ctx, h))
        say("FP64 eval of the same loads stays finite")
        mrs.mrs_ensemble_eval(ctx, h, mrs.MRS_FP64, False)
        _, _, U, _ = mrs.mrs_ensemble_get(ctx, h)
        assert np.all(np.isfinite(U))
        say("batched eval with one overflowing ensemble")
        _numeric(mrs, lambda: mrs.mrs_batch_eval(ctx, [ok, h], mrs.MRS_FP32C, False))
        mrs.mrs_batch_eval(ctx, [ok], mrs.MRS_FP32C, False)
        say("step of 1e307")
        _numeric(mrs, lambda: mrs.mrs_ensemble_step(ctx, ok, mrs.MRS_EULER, 1e307, 1, mrs.MRS_FP64, True))
        mrs.mrs_ensemble_set_state(ctx, ok, e.X, e.D)
        mrs.mrs_ensemble_step(ctx, ok, mrs.MRS_EULER, 1e-4, 1, mrs.MRS_FP64, True)
        _numeric(mrs, lambda: mrs.mrs_batch_step(ctx, [ok], mrs.MRS_RK4, 1e307, 1, mrs.MRS_FP64, True, True))
        mrs.mrs_ensemble_set_state(ctx, ok, e.X, e.D)
        say("Parareal with an overflowing coarse step")
        _numeric(mrs, lambda: mrs.mrs_parareal(ctx, ok, 2, mrs.MRS_EULER, 1e307, 1, 1, 1, 0.0, mrs.MRS_FP64, True))
        mrs.mrs_ensemble_set_state(ctx, ok, e.X, e.D)
        it, _ = mrs.mrs_parareal(ctx, ok, 2, mrs.MRS_EULER, 1e-5, 2, 1, 2, 0.0, mrs.MRS_FP64, True)
        assert it == 2
    finally:
        mrs.mrs_ensemble_destroy(h)
        mrs.mrs_ensemble_destroy(ok)


def test_enumeric_served_request(mrs):
    """A served request whose result overflows completes with MRS_ENUMERIC
    (its arrays still returned) while the request beside it is unaffected."""
    ctx = mrs.mrs_context_create(0)
    try:
        e = synth.filaments(3, 64, 2.0, 81)
        rod = rod_of(mrs, e.rod())
        srv = mrs.mrs_server_start(ctx, mrs.MRS_FP32C, 1 << 30, 8)
        try:
            t_bad = mrs.mrs_server_submit(srv, 0, e.offsets, e.X, e.D, np.full_like(e.f, 1e38), e.n, e.eps, e.mu, rod)
            t_ok = mrs.mrs_server_submit(srv, 1, e.offsets, e.X, e.D, e.f, e.n, e.eps, e.mu, rod, dt=1e-5, nsteps=3,
                                         integ=mrs.MRS_RK4)
            st, info, out = mrs.mrs_server_wait(srv, t_bad, e.N, timeout_s=60)
            say(f"overflowing request: status {st}")
            assert st == mrs.MRS_ENUMERIC and out is not None and not np.all(np.isfinite(out[2]))
            st, info, out = mrs.mrs_server_wait(srv, t_ok, e.N, timeout_s=60)
            assert st == mrs.MRS_OK and np.all(np.isfinite(out[0]))
        finally:
            mrs.mrs_server_stop(srv)
    finally:
        mrs.mrs_context_destroy(ctx)


@pytest.mark.parametrize("prec", [0, 1])
def test_eval_device_on_two_streams_without_sync(mrs, prec):
    """Evaluations queued on two streams back to back (no host wait between
    them, growing scratch included) each give their own oracle result."""
    import torch

    ctx = mrs.mrs_context_create(0)
    try:
        probs = []
        for k, N in enumerate((300, 2500, 1200, 4000)):
            rng = np.random.default_rng(90 + k)
            X, f, n = rng.uniform(0, 1, (N, 3)), rng.normal(size=(N, 3)), rng.normal(size=(N, 3))
            probs.append((X, f, n, 0.02 + 0.01 * k))
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        dev_in = [(dev(X), dev(f), dev(n)) for X, f, n, _ in probs]
        outs = [(torch.empty_like(d[0]), torch.empty_like(d[0])) for d in dev_in]
        torch.cuda.synchronize()
        for k, ((X, f, n, eps), (dX, df, dn), (U, W)) in enumerate(zip(probs, dev_in, outs)):
            mrs.mrs_eval_device(ctx, len(X), dX, df, dn, eps, 1.0, prec, U, W, streams[k % 2])
        torch.cuda.synchronize()
        for k, ((X, f, n, eps), (U, W)) in enumerate(zip(probs, outs)):
            Uo, Wo = oracle.mrs_eval(X, f, n, eps, 1.0)
            eu, ew = oracle.rel_err(U.cpu().numpy(), Uo), oracle.rel_err(W.cpu().numpy(), Wo)
            say(f"stream {k % 2} N={len(X)}: U {eu:.3e} W {ew:.3e}")
            assert eu <= TOL[prec] and ew <= TOL[prec], (k, eu, ew)
    finally:
        mrs.mrs_context_destroy(ctx)
