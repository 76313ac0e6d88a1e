"""The allocation-free evaluation (mrs_eval_device_noalloc) against the
allocating one (mrs_eval_device) through the C ABI: two calls in a row, the
second with a smaller input, in both precisions, at the bar of the parity
tests (the paper's relative error form, Eq. true_err: 1e-12 for MRS_FP64,
1e-5 for MRS_FP32C), plus the oracle on the same inputs, a size whose
default partial sums do not fit the scratch, and the size limit."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def mrs():
    import paper_2604_12083_amd as m

    return m


def _cloud(N, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (N, 3)), rng.normal(size=(N, 3)), rng.normal(size=(N, 3)), 0.02


def _both(mrs, ctx, X, f, n, eps, prec):
    import torch

    dX, df, dn = dev(X), dev(f), dev(n)
    U0, W0 = torch.empty_like(dX), torch.empty_like(dX)
    U1, W1 = torch.full_like(dX, np.nan), torch.full_like(dX, np.nan)
    s = torch.cuda.current_stream()
    mrs.mrs_eval_device(ctx, len(X), dX, df, dn, eps, 1.0, prec, U0, W0, s)
    mrs.mrs_eval_device_noalloc(ctx, len(X), dX, df, dn, eps, 1.0, prec, U1, W1, s)
    torch.cuda.synchronize()
    return (U0.cpu().numpy(), W0.cpu().numpy()), (U1.cpu().numpy(), W1.cpu().numpy())


@pytest.mark.parametrize("prec", [1, 0])
def test_noalloc_matches_eval_device_twice(mrs, prec):
    """12,800 points (the benchmark ensemble), then 3,000: same configuration
    as mrs_eval_device, so the same sums; checked against it and the oracle."""
    ctx = mrs.mrs_context_create(0)
    try:
        e = synth.ens12800()
        for tag, (X, f, n, eps) in (("ens12800", (e.X, e.f, e.n, e.eps)), ("cloud3000", _cloud(3000, 5))):
            say(f"noalloc {tag} N={len(X)} prec={prec}")
            (U0, W0), (U1, W1) = _both(mrs, ctx, X, f, n, eps, prec)
            eu, ew = oracle.rel_err(U1, U0), oracle.rel_err(W1, W0)
            say(f"  vs mrs_eval_device: U {eu:.3e} W {ew:.3e}")
            assert eu <= TOL[prec] and ew <= TOL[prec], (tag, eu, ew)
            idx = np.sort(np.random.default_rng(7).choice(len(X), min(len(X), 1024), replace=False))
            Uo, Wo = oracle.mrs_field(X[idx], X, f, n, eps, 1.0)
            eu, ew = oracle.rel_err(U1[idx], Uo), oracle.rel_err(W1[idx], Wo)
            say(f"  vs oracle ({len(idx)} targets): U {eu:.3e} W {ew:.3e}")
            assert eu <= TOL[prec] and ew <= TOL[prec], (tag, eu, ew)
    finally:
        mrs.mrs_context_destroy(ctx)


@pytest.mark.parametrize("prec", [1, 0])
def test_noalloc_fewer_chunks_when_partials_do_not_fit(mrs, prec):
    """100,000 points: the default decomposition's partial sums exceed the
    scratch, so the call uses fewer, longer source chunks; then a small call."""
    ctx = mrs.mrs_context_create(0)
    try:
        big = synth.filaments(400, 250, 20.0, 61)
        for tag, (X, f, n, eps) in (("fil100000", (big.X, big.f, big.n, big.eps)), ("cloud700", _cloud(700, 6))):
            say(f"noalloc {tag} N={len(X)} prec={prec}")
            (U0, W0), (U1, W1) = _both(mrs, ctx, X, f, n, eps, prec)
            eu, ew = oracle.rel_err(U1, U0), oracle.rel_err(W1, W0)
            say(f"  vs mrs_eval_device: U {eu:.3e} W {ew:.3e}")
            assert eu <= TOL[prec] and ew <= TOL[prec], (tag, eu, ew)
            idx = np.sort(np.random.default_rng(8).choice(len(X), min(len(X), 512), replace=False))
            Uo, Wo = oracle.mrs_field(X[idx], X, f, n, eps, 1.0)
            eu, ew = oracle.rel_err(U1[idx], Uo), oracle.rel_err(W1[idx], Wo)
            say(f"  vs oracle ({len(idx)} targets): U {eu:.3e} W {ew:.3e}")
            assert eu <= TOL[prec] and ew <= TOL[prec], (tag, eu, ew)
    finally:
        mrs.mrs_context_destroy(ctx)


def test_noalloc_rejects_sizes_beyond_the_scratch(mrs):
    """Host-side check before any device work: more than 500,000 points."""
    import torch

    ctx = mrs.mrs_context_create(0)
    try:
        t = torch.zeros((4, 3), dtype=torch.float64, device="cuda:0")
        with pytest.raises(mrs.MrsError) as ex:
            mrs.mrs_eval_device_noalloc(ctx, 500_001, t, t, t, 0.1, 1.0, mrs.MRS_FP32C, t, t)
        assert ex.value.status == mrs.MRS_EINVAL and "500000" in str(ex.value), ex.value
        say(f"rejected: {ex.value}")
    finally:
        mrs.mrs_context_destroy(ctx)


@pytest.mark.parametrize("prec", [1, 0])
def test_noalloc_with_tuned_schedules(mrs, prec):
    """Table entries with the persistent schedule and the four-wave split
    (FP32C; FP64 falls back to the tiled kernel): the work-queue counters of
    the allocation-free call live in its scratch and start at zero on every
    call, so two calls in a row give the allocating call's sums."""
    ctx = mrs.mrs_context_create(0)
    try:
        for cfg in ((2, 1, 0, 1), (0, 1, 0, 1), (2, 1, 9, 0)):
            for N, seed in ((3000, 11), (2100, 12)):
                mrs.mrs_tune_set(ctx, N, prec, *cfg)
                X, f, n, eps = _cloud(N, seed)
                (U0, W0), (U1, W1) = _both(mrs, ctx, X, f, n, eps, prec)
                eu, ew = oracle.rel_err(U1, U0), oracle.rel_err(W1, W0)
                say(f"noalloc cfg {cfg} N={N} prec={prec}: vs mrs_eval_device U {eu:.3e} W {ew:.3e}")
                assert eu <= TOL[prec] and ew <= TOL[prec], (cfg, N, eu, ew)
    finally:
        mrs.mrs_context_destroy(ctx)
