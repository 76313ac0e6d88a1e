"""Pins of the oracle's swimming workload (Sec. IV): the preferred
strain-twist waveform and the Lennard-Jones repulsion between filaments.

  * Lennard-Jones: the force of one pair against the derivative of the
    potential written out by hand; force = minus the finite-difference
    gradient of the total energy; nothing beyond the cutoff or within a
    filament; zero total force and torque (pair forces along the separation).
  * Waveform: a rod built in the preferred shape of time t (planar, bent
    about its second director with discrete curvature equal to
    -k^2 A sin(k s + f t) at every segment midpoint, no shear or stretch)
    carries no elastic load at time t, and does at other times; zero
    amplitude gives the plain rod.
  * Time stepping: the clock advances by dt per step, steps compose, and
    RK4 keeps order 4 on the time-dependent problem (stage times
    t + c_s dt); Euler and the midpoint RK2 keep orders 1 and 2.
"""
import math

import numpy as np
import pytest

import synth


def _two_points(r):
    X = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    return np.array([0, 1, 2], dtype=np.int32), X


@pytest.mark.parametrize("ratio", [0.8, 0.95, 1.0, 1.05, 1.12, 1.13, 1.5])
def test_lj_pair_force_closed_form(oracle_mod, ratio):
    sig, e = 0.03, 2.5
    r = ratio * sig
    off, X = _two_points(r)
    F = oracle_mod.lj_forces(off, X, (sig, e))
    # -dU/dr of U = 4 e ((sig/r)^12 - (sig/r)^6), written out term by term
    dUdr = 4.0 * e * (-12.0 * sig ** 12 / r ** 13 + 6.0 * sig ** 6 / r ** 7)
    expect = -dUdr if r < 2.0 ** (1.0 / 6.0) * sig else 0.0
    np.testing.assert_allclose(F[1], [expect, 0.0, 0.0], rtol=1e-13, atol=0.0)
    np.testing.assert_allclose(F[0], [-expect, 0.0, 0.0], rtol=1e-13, atol=0.0)


def _tangle(seed=5):
    """Three short filaments passing close to one another."""
    rng = np.random.default_rng(seed)
    M, ds = 10, 0.01
    X = []
    for _ in range(3):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = rng.normal(scale=0.01, size=3)
        X.append(c + (np.arange(M) - M / 2)[:, None] * ds * d[None, :])
    return np.array([0, M, 2 * M, 3 * M], dtype=np.int32), np.concatenate(X)


def test_lj_force_is_minus_energy_gradient(oracle_mod):
    off, X = _tangle()
    lj = (0.02, 1.0)
    rc = 2.0 ** (1.0 / 6.0) * lj[0]
    F = oracle_mod.lj_forces(off, X, lj)
    fil = np.repeat(np.arange(3), 10)
    r = np.linalg.norm(X[:, None, :] - X[None, :, :], axis=-1)
    other = fil[:, None] != fil[None, :]
    assert np.sum(other & (r < rc)) >= 6, "geometry must put some pairs inside the cutoff"
    assert np.min(np.abs(r[other] - rc)) > 1e-5, "no pair may sit at the truncation"
    h = 1e-8
    G = np.zeros_like(X)
    for i in range(X.shape[0]):
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, c] += h
            Xm[i, c] -= h
            G[i, c] = (oracle_mod.lj_energy(off, Xp, lj) - oracle_mod.lj_energy(off, Xm, lj)) / (2 * h)
    scale = np.abs(F).max()
    assert scale > 0
    np.testing.assert_allclose(F, -G, atol=1e-6 * scale, rtol=0)


def test_lj_cutoff_exclusion_and_balance(oracle_mod):
    off, X = _tangle(7)
    lj = (0.02, 1.0)
    F = oracle_mod.lj_forces(off, X, lj)
    # total force and torque vanish: pair forces are equal, opposite, central
    scale = np.abs(F).max() * X.shape[0]
    assert np.abs(F.sum(axis=0)).max() <= 1e-13 * scale
    assert np.abs(np.cross(X, F).sum(axis=0)).max() <= 1e-13 * scale * np.abs(X).max()
    # one filament alone feels nothing, however close its points are
    one = np.array([0, 10], dtype=np.int32)
    assert np.all(oracle_mod.lj_forces(one, X[:10], (1.0, 1.0)) == 0.0)
    # filaments pulled apart beyond the cutoff feel nothing
    Xf = X.copy()
    Xf[10:20] += 10.0
    Xf[20:30] += 20.0
    assert np.all(oracle_mod.lj_forces(off, Xf, lj) == 0.0)


def test_lj_enters_as_point_force_on_the_fluid(oracle_mod):
    e = synth.filaments(3, 12, 0.05, 9)
    rod = e.rod()
    lj = (2.0 * e.eps, 0.5)
    g0, m0 = oracle_mod.rod_forces(e.offsets, e.X, e.D, rod, e.f, e.n)
    g1, m1 = oracle_mod.rod_forces(e.offsets, e.X, e.D, rod, e.f, e.n, lj=lj)
    F = oracle_mod.lj_forces(e.offsets, e.X, lj)
    assert np.abs(F).max() > 0
    np.testing.assert_array_equal(g1, g0 + F)
    np.testing.assert_array_equal(m1, m0)
    U, W = oracle_mod.velocities(e.offsets, e.X, e.D, rod, e.f, e.n, e.eps, e.mu, include_elastic=False, lj=lj)
    Ue, We = oracle_mod.mrs_eval(e.X, e.f + F, e.n, e.eps, e.mu)
    np.testing.assert_array_equal(U, Ue)
    np.testing.assert_array_equal(W, We)


def _preferred_shape(M, ds, wave, t):
    """Planar rod whose discrete strain-twist is (0, -k^2 A sin(k s + f t), 0)
    at every segment midpoint s = (k + 1/2) ds, with no shear or stretch.

    Frames rotate about the fixed second director e_y: D1 = (cos q, 0, -sin q),
    D3 = (sin q, 0, cos q).  For an increment a between nodes, the difference
    of the third directors is 2 sin(a/2) times the first director of the
    half-way frame, so the curvature about D2 is 2 sin(a/2)/ds; the segment
    vector is ds times the half-way third director."""
    A, k, f = wave
    q = np.zeros(M)
    for j in range(M - 1):
        om = -k * k * A * math.sin(k * (j + 0.5) * ds + f * t)
        q[j + 1] = q[j] + 2.0 * math.asin(0.5 * ds * om)
    X = np.zeros((M, 3))
    for j in range(M - 1):
        h = 0.5 * (q[j] + q[j + 1])
        X[j + 1] = X[j] + ds * np.array([math.sin(h), 0.0, math.cos(h)])
    D = np.zeros((M, 9))
    D[:, 0], D[:, 2] = np.cos(q), -np.sin(q)
    D[:, 4] = 1.0
    D[:, 6], D[:, 8] = np.sin(q), np.cos(q)
    return X, D


def test_waveform_preferred_shape_is_load_free(oracle_mod):
    M, ds = 51, 1.0 / 50
    wave = (0.05, 2 * math.pi, 40.0)
    t = 0.013
    X, D = _preferred_shape(M, ds, wave, t)
    off = np.array([0, M], dtype=np.int32)
    rod = synth.RodParams(a=(1.0, 1.0, 1.0), b=(1.0, 1.0, 1.0), ds=ds)
    g, m = oracle_mod.rod_forces(off, X, D, rod, wave=wave, t=t)
    g2, m2 = oracle_mod.rod_forces(off, X, D, rod, wave=wave, t=t + 0.5 * math.pi / wave[2])
    load = max(np.abs(g2).max(), np.abs(m2).max())
    assert load > 1e-3, load
    assert np.abs(g).max() <= 1e-10 * load and np.abs(m).max() <= 1e-10 * load, (np.abs(g).max(), np.abs(m).max())
    # without the waveform the same shape is loaded (it is bent)
    g0, m0 = oracle_mod.rod_forces(off, X, D, rod)
    assert np.abs(m0).max() > 1e-3


def test_waveform_zero_amplitude_is_plain_rod(oracle_mod):
    e = synth.filaments(2, 20, 1.0, 4)
    rod = e.rod(a=(0.3, 0.3, 0.2), b=(1.0, 1.0, 2.0))
    g0, m0 = oracle_mod.rod_forces(e.offsets, e.X, e.D, rod, e.f, e.n)
    g1, m1 = oracle_mod.rod_forces(e.offsets, e.X, e.D, rod, e.f, e.n, wave=(0.0, 3.0, 7.0), t=0.4)
    np.testing.assert_array_equal(g0, g1)
    np.testing.assert_array_equal(m0, m1)


def test_clock_and_step_composition(oracle_mod):
    e = synth.filaments(2, 16, 0.5, 6)
    rod = e.rod(a=(1e-3, 1e-3, 1e-3))
    wave, lj = (0.1, 2 * math.pi, 30.0), (2.0 * e.eps, 1e-3)
    dt, t0 = 1e-4, 0.25
    X3, D3, _, _, t3 = oracle_mod.step_ex(e.offsets, e.X, e.D, rod, e.f, e.n, e.eps, e.mu, oracle_mod.RK4, dt, 3,
                                          wave=wave, t=t0, lj=lj)
    assert t3 == ((t0 + dt) + dt) + dt
    X, D, t = e.X, e.D, t0
    for _ in range(3):
        X, D, _, _, t = oracle_mod.step_ex(e.offsets, X, D, rod, e.f, e.n, e.eps, e.mu, oracle_mod.RK4, dt, 1,
                                           wave=wave, t=t, lj=lj)
    np.testing.assert_array_equal(X, X3)
    np.testing.assert_array_equal(D, D3)
    assert t == t3


@pytest.mark.slow
def test_orders_on_the_time_dependent_problem(oracle_mod):
    """The waveform drives the rod through its time argument; with stage
    times t + c_s dt the three integrators keep their orders."""
    M = 16
    e = synth.filaments(1, M, 1.0, 3)
    rod = e.rod(a=(0.02, 0.02, 0.02), b=(0.0, 0.0, 0.0))
    wave = (0.2, 2 * math.pi, 300.0)
    zero = np.zeros_like(e.f)
    T = 0.004

    def run(integ, n):
        X, _, _, _ = oracle_mod.step(e.offsets, e.X, e.D, rod, zero, zero, e.eps, e.mu, integ, T / n, n,
                                     wave=wave, t=0.0)
        return X

    Xref = run(oracle_mod.RK4, 512)
    moved = np.abs(Xref - e.X).max()
    assert moved > 1e-4, moved
    ratios = {}
    for integ, steps in ((oracle_mod.EULER, (64, 128, 256)), (oracle_mod.RK2, (32, 64, 128)),
                         (oracle_mod.RK4, (8, 16, 32))):
        err = [np.abs(run(integ, s) - Xref).max() for s in steps]
        ratios[integ] = [err[i] / err[i + 1] for i in range(2)]
    assert all(1.8 < r < 2.3 for r in ratios[oracle_mod.EULER]), ratios
    assert all(3.5 < r < 4.6 for r in ratios[oracle_mod.RK2]), ratios
    assert all(13.0 < r < 19.0 for r in ratios[oracle_mod.RK4]), ratios
