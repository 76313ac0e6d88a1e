"""Pins of the oracle's Parareal iteration (Sec. II.D, Eqs. initial,
intermediate, serial_correct).

  * Exactness: after k iterations the first k slice boundaries equal the
    serial fine solution exactly (the algorithm's defining property: slice k
    is then the fine propagation of an exact state).
  * With the coarse propagator identical to the fine one (both forward
    Euler with the same steps), iteration 0 already is the fine solution and
    the first increment is exactly zero.
  * The increments decrease over the iterations of a well-resolved run,
    and with smooth forcing (no external torques) four iterations bring
    the error against the serial fine solution to ~1e-12, the behaviour the
    paper reports for its runs (Sec. IV.B, Fig. 5).
"""
import numpy as np

import synth


def _serial(oracle_mod, e, rod, ns, integ, dt, steps):
    X, D = e.X, e.D
    out = [(X, D)]
    for _ in range(ns):
        X, D, _, _ = oracle_mod.step(e.offsets, X, D, rod, e.f, e.n, e.eps, e.mu, integ, dt, steps)
        out.append((X, D))
    return out


def test_parareal_exact_after_k_iterations(oracle_mod):
    e = synth.filaments(2, 16, 1.0, 9)
    rod = e.rod()
    ns, steps, dt = 4, 10, 2e-4
    ref = _serial(oracle_mod, e, rod, ns, oracle_mod.RK2, dt, steps)
    for k in range(1, ns + 1):
        U, hist = oracle_mod.parareal(e.offsets, e.X, e.D, rod, e.f, e.n, e.eps, e.mu, ns, oracle_mod.RK2, dt,
                                      steps, 1, k)
        for n in range(1, k + 1):
            np.testing.assert_array_equal(U[n][0], ref[n][0])
            np.testing.assert_array_equal(U[n][1], ref[n][1])
    assert all(np.diff(hist) < 0), hist


def test_parareal_coarse_equal_fine(oracle_mod):
    e = synth.filaments(1, 20, 1.0, 3)
    rod = e.rod()
    U, hist = oracle_mod.parareal(e.offsets, e.X, e.D, rod, e.f, e.n, e.eps, e.mu, 3, oracle_mod.EULER, 1e-4, 5, 5, 1)
    assert hist[0] == 0.0


def test_parareal_four_iterations_reach_1e12(oracle_mod):
    e = synth.filaments(4, 50, 2.0, 21)
    rod = e.rod()
    ns, steps, dt = 8, 20, 1e-5
    zero = np.zeros_like(e.n)
    X, D = e.X, e.D
    for _ in range(ns):
        X, D, _, _ = oracle_mod.step(e.offsets, X, D, rod, e.f, zero, e.eps, e.mu, oracle_mod.RK4, dt, steps)
    U, hist = oracle_mod.parareal(e.offsets, e.X, e.D, rod, e.f, zero, e.eps, e.mu, ns, oracle_mod.RK4, dt, steps, 2, 4)
    eta = oracle_mod.rel_err(U[ns][0], X)
    assert eta < 1e-11, (eta, hist)
    assert all(np.diff(np.log10(hist)) < -1.0), hist
