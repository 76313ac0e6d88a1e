"""Pins of the oracle's explicit time steps (Sec. III.B.3, Eqs. newx, newD;
the fine propagator of Sec. III.A is an explicit Runge-Kutta method).

  * Convergence orders: with zero moduli the positions follow the autonomous
    ODE dX/dt = U(X) driven by fixed loads, so forward Euler must converge
    at order 1, the midpoint RK2 at order 2 and the classical RK4 at order
    4 (error ratios ~2, ~4 and ~16 when dt halves), measured against a much
    finer RK4 solution.
  * With the elastic coupling on, the angular velocity changes within a step
    and the frames feed back into the forces: RK4 (frames by
    Runge-Kutta-Munthe-Kaas) must still converge at order 4 in both the
    frames and the positions, and RK2 at order 2 (a frame update that skips
    the dexp^-1 terms, or gets their sign wrong, falls to order 2).
  * One Euler step equals its definition composed from the pinned pieces
    (rod forces, MRS sum, Rodrigues update, re-orthonormalisation).
  * Frames stay orthonormal and right-handed over many steps.
"""
import math

import numpy as np
import pytest

import synth


def _small(seed=21, F=2, M=16):
    e = synth.filaments(F, M, 0.6, seed)
    return e


def _run(oracle_mod, e, rod, integ, T, nsteps, elastic=False):
    X, D, _, _ = oracle_mod.step(e.offsets, e.X, e.D, rod, e.f, e.n, e.eps, e.mu, integ,
                                 T / nsteps, nsteps, include_elastic=elastic)
    return X, D


@pytest.mark.slow
def test_convergence_orders(oracle_mod):
    e = _small()
    rod = e.rod(a=(0, 0, 0), b=(0, 0, 0))
    T = 0.01  # short enough that the step sizes below are in the asymptotic regime
    Xref, _ = _run(oracle_mod, e, rod, oracle_mod.RK4, T, 256)
    errs = {}
    for integ, steps in ((oracle_mod.EULER, (32, 64, 128)), (oracle_mod.RK4, (8, 16, 32))):
        errs[integ] = [np.abs(_run(oracle_mod, e, rod, integ, T, s)[0] - Xref).max() for s in steps]
    errs[2] = [np.abs(_run(oracle_mod, e, rod, oracle_mod.RK2, T, s)[0] - Xref).max() for s in (16, 32, 64)]
    r_e = [errs[1][i] / errs[1][i + 1] for i in range(2)]
    r_2 = [errs[2][i] / errs[2][i + 1] for i in range(2)]
    r_4 = [errs[4][i] / errs[4][i + 1] for i in range(2)]
    assert all(1.8 < r < 2.3 for r in r_e), (errs[1], r_e)
    assert all(3.5 < r < 4.6 for r in r_2), (errs[2], r_2)
    assert all(13.0 < r < 19.0 for r in r_4), (errs[4], r_4)


def test_convergence_orders_with_elastic_coupling(oracle_mod):
    e = _small()
    rod = e.rod(a=(1e-3,) * 3, b=(1e-2,) * 3)
    T = 1e-3
    Xref, Dref = _run(oracle_mod, e, rod, oracle_mod.RK4, T, 128, elastic=True)
    for integ, steps, lo, hi in ((oracle_mod.RK4, (4, 8, 16), 14.0, 18.0), (oracle_mod.RK2, (8, 16, 32), 3.6, 4.4)):
        ex, ed = [], []
        for s in steps:
            X, D = _run(oracle_mod, e, rod, integ, T, s, elastic=True)
            ex.append(np.abs(X - Xref).max())
            ed.append(np.abs(D - Dref).max())
        rx = [ex[i] / ex[i + 1] for i in range(2)]
        rd = [ed[i] / ed[i + 1] for i in range(2)]
        assert all(lo < r < hi for r in rx), (integ, ex, rx)
        assert all(lo < r < hi for r in rd), (integ, ed, rd)


def test_rkmk_stage_correction(oracle_mod):
    """The second RK4 stage from a state whose first-stage Omega is w0: the
    stage frame is Rod(dt/2 w0) D, and the step's frame sums take
    k = Omega - theta x Omega / 2 + theta x (theta x Omega) / 12 with
    theta = dt/2 w0.  Checked on one step against the four stages composed
    from the oracle's own velocities and Rodrigues update."""
    e = _small(7)
    rod = e.rod(a=(1e-3,) * 3, b=(1e-2,) * 3)
    dt = 2e-3
    X0, D0 = e.X.copy(), e.D.copy()

    def vel(X, D):
        return oracle_mod.velocities(e.offsets, X, D, rod, e.f, e.n, e.eps, e.mu)

    def rot(W, h, D):
        out = np.empty_like(D)
        for k in range(len(D)):
            for i in range(3):
                out[k, 3 * i:3 * i + 3] = oracle_mod.rodrigues(h * W[k], D[k, 3 * i:3 * i + 3])
        return out

    c, w = (0.0, 0.5, 0.5, 1.0), (1 / 6, 2 / 6, 2 / 6, 1 / 6)
    Ua, Wa = np.zeros_like(X0), np.zeros_like(X0)
    U, k = None, None
    for s in range(4):
        Xs = X0 if s == 0 else X0 + c[s] * dt * U
        Ds = D0 if s == 0 else rot(k, c[s] * dt, D0)
        U, W = vel(Xs, Ds)
        if s > 0:
            th = c[s] * dt * k
            t1 = np.cross(th, W)
            W = W - 0.5 * t1 + np.cross(th, t1) / 12.0
        k = W
        Ua += w[s] * U
        Wa += w[s] * k
    X1 = X0 + dt * Ua
    D1 = oracle_mod.reorthonormalize(rot(Wa, dt, D0))
    Xs, Ds, _, _ = oracle_mod.step(e.offsets, X0, D0, rod, e.f, e.n, e.eps, e.mu, oracle_mod.RK4, dt, 1)
    np.testing.assert_allclose(Xs, X1, rtol=0, atol=1e-14)
    np.testing.assert_allclose(Ds, D1, rtol=0, atol=1e-14)


def test_euler_step_composition(oracle_mod):
    e = synth.rod64()
    rod = e.rod()
    dt = 1e-4
    g, m = oracle_mod.rod_forces(e.offsets, e.X, e.D, rod, e.f, e.n)
    U, W = oracle_mod.mrs_eval(e.X, g, m, e.eps, e.mu)
    X1 = e.X + dt * U
    D1 = np.zeros_like(e.D)
    for k in range(e.N):
        for i in range(3):
            D1[k, 3 * i:3 * i + 3] = oracle_mod.rodrigues(dt * W[k], e.D[k, 3 * i:3 * i + 3])
    D1 = oracle_mod.reorthonormalize(D1)
    Xs, Ds, Us, Ws = oracle_mod.step(e.offsets, e.X, e.D, rod, e.f, e.n, e.eps, e.mu, oracle_mod.EULER, dt, 1)
    np.testing.assert_array_equal(Xs, X1)
    np.testing.assert_array_equal(Ds, D1)
    np.testing.assert_array_equal(Us, U)
    np.testing.assert_array_equal(Ws, W)


def test_rk4_single_stage_quantities(oracle_mod):
    """The first stage of an RK4 step is evaluated at the unmodified state."""
    e = _small(5)
    rod = e.rod()
    _, _, U, W = oracle_mod.step(e.offsets, e.X, e.D, rod, e.f, e.n, e.eps, e.mu, oracle_mod.RK4, 1e-5, 1)
    U0, W0 = oracle_mod.velocities(e.offsets, e.X, e.D, rod, e.f, e.n, e.eps, e.mu)
    np.testing.assert_array_equal(U, U0)
    np.testing.assert_array_equal(W, W0)


def test_frames_stay_orthonormal(oracle_mod):
    e = synth.rod64()
    X, D, _, _ = oracle_mod.step(e.offsets, e.X, e.D, e.rod(), e.f, e.n, e.eps, e.mu, oracle_mod.EULER, 1e-4, 20)
    Dm = D.reshape(-1, 3, 3)
    np.testing.assert_allclose(np.einsum("kij,klj->kil", Dm, Dm), np.broadcast_to(np.eye(3), Dm.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(Dm), 1.0, atol=1e-14)
    assert np.all(np.isfinite(X))
