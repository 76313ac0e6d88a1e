"""Pins of the oracle's discrete Kirchhoff rod forces (Sec. II.B, Alg. 1).

Closed forms for three uniform states whose strains are known exactly:
  * uniform stretch of a straight rod: F = b3 delta D3 on every segment;
  * uniform twist by alpha per segment: N3 = a3 2 sin(alpha/2)/ds, which
    also pins the half-angle mid frame (the full-angle frame would give
    sin(alpha)/ds);
  * uniform bend about D2 (circular arc): N2 = a2 2 sin(alpha/2)/ds with F = 0.
Invariants: total force and total torque about the origin vanish (free
ends), rigid rotations rotate g and m, translations leave them unchanged,
a stress-free state gives zero, and relaxation through the MRS dissipates
the elastic energy (fixes the sign of the force handed to the fluid).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth


def _straight(M, ds, stretch=0.0):
    X = np.zeros((M, 3))
    X[:, 2] = np.arange(M) * ds * (1 + stretch)
    D = np.tile(np.eye(3).reshape(9), (M, 1))
    return X, D


def _rod(a=(0.3, 0.4, 0.5), b=(1.5, 1.7, 2.0), om=(0.0, 0.0, 0.0), ds=0.05):
    return synth.RodParams(a, b, om, ds)


def test_uniform_stretch(oracle_mod):
    M, ds, delta = 12, 0.05, 0.03
    rod = _rod(ds=ds)
    X, D = _straight(M, ds, delta)
    g, m = oracle_mod.rod_forces([0, M], X, D, rod)
    want = np.zeros((M, 3))
    want[0, 2] = rod.b[2] * delta
    want[-1, 2] = -rod.b[2] * delta
    np.testing.assert_allclose(g, want, atol=1e-13)
    np.testing.assert_allclose(m, 0.0, atol=1e-13)


@pytest.mark.parametrize("alpha", [0.01, 0.3, 1.2])
def test_uniform_twist(oracle_mod, alpha):
    M, ds = 10, 0.1
    rod = _rod(ds=ds)
    X, _ = _straight(M, ds)
    D = np.zeros((M, 9))
    for k in range(M):
        c, s = math.cos(k * alpha), math.sin(k * alpha)
        D[k] = [c, s, 0, -s, c, 0, 0, 0, 1]
    g, m = oracle_mod.rod_forces([0, M], X, D, rod)
    N3 = rod.a[2] * 2 * math.sin(alpha / 2) / ds
    want = np.zeros((M, 3))
    want[0, 2] = N3
    want[-1, 2] = -N3
    np.testing.assert_allclose(g, 0.0, atol=1e-12)
    np.testing.assert_allclose(m, want, atol=1e-12 * max(1, N3))
    # the intrinsic twist that matches the state removes the torque
    rod2 = _rod(om=(0.0, 0.0, 2 * math.sin(alpha / 2) / ds), ds=ds)
    g2, m2 = oracle_mod.rod_forces([0, M], X, D, rod2)
    np.testing.assert_allclose(m2, 0.0, atol=1e-12)


@pytest.mark.parametrize("alpha", [0.02, 0.4])
def test_uniform_bend(oracle_mod, alpha):
    M, ds = 9, 0.1
    rod = _rod(ds=ds)
    D = np.zeros((M, 9))
    X = np.zeros((M, 3))
    for k in range(M):
        Q = Rotation.from_rotvec([0, k * alpha, 0]).as_matrix()
        D[k] = (Q @ np.eye(3)).T.reshape(9)  # rows = directors Q e_i
        if k > 0:
            Qh = Rotation.from_rotvec([0, (k - 0.5) * alpha, 0]).as_matrix()
            X[k] = X[k - 1] + ds * Qh[:, 2]
    g, m = oracle_mod.rod_forces([0, M], X, D, rod)
    N2 = rod.a[1] * 2 * math.sin(alpha / 2) / ds
    want = np.zeros((M, 3))
    want[0, 1] = N2
    want[-1, 1] = -N2
    np.testing.assert_allclose(g, 0.0, atol=1e-12)
    np.testing.assert_allclose(m, want, atol=1e-12 * max(1, N2))


def _perturbed(seed, F=3, M=20):
    e = synth.filaments(F, M, 1.0, seed, draw_loads=False)
    rng = np.random.default_rng(seed + 100)
    e.X = e.X + rng.normal(scale=2e-3, size=e.X.shape)
    rot = Rotation.from_rotvec(rng.normal(scale=0.05, size=(e.N, 3))).as_matrix()
    Dm = e.D.reshape(e.N, 3, 3)
    e.D = np.einsum("pab,pib->pia", rot, Dm).reshape(e.N, 9)
    return e


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_force_and_torque_balance(oracle_mod, seed):
    e = _perturbed(seed)
    rod = _rod(ds=e.ds)
    g, m = oracle_mod.rod_forces(e.offsets, e.X, e.D, rod)
    for f0, f1 in zip(e.offsets[:-1], e.offsets[1:]):
        gs, ms, Xs = g[f0:f1], m[f0:f1], e.X[f0:f1]
        scale = np.abs(gs).sum() * (1 + np.abs(Xs).max()) + np.abs(ms).sum()
        assert np.abs(gs.sum(0)).max() <= 1e-13 * scale
        assert np.abs((ms + np.cross(Xs, gs)).sum(0)).max() <= 1e-13 * scale


def test_frame_indifference_and_translation(oracle_mod):
    e = _perturbed(7)
    rod = _rod(ds=e.ds)
    g, m = oracle_mod.rod_forces(e.offsets, e.X, e.D, rod)
    Q = Rotation.random(random_state=11).as_matrix()
    DQ = np.einsum("ab,pib->pia", Q, e.D.reshape(e.N, 3, 3)).reshape(e.N, 9)
    gq, mq = oracle_mod.rod_forces(e.offsets, e.X @ Q.T + 5.0, DQ, rod)
    np.testing.assert_allclose(gq, g @ Q.T, atol=1e-12 * np.abs(g).max())
    np.testing.assert_allclose(mq, m @ Q.T, atol=1e-12 * np.abs(m).max())


def test_stress_free_and_external_loads(oracle_mod):
    M, ds = 8, 0.125
    X, D = _straight(M, ds)
    rod = _rod(ds=ds)
    rng = np.random.default_rng(0)
    fe, ne = rng.normal(size=(M, 3)), rng.normal(size=(M, 3))
    g, m = oracle_mod.rod_forces([0, M], X, D, rod, fe, ne)
    np.testing.assert_allclose(g, fe, atol=1e-14)
    np.testing.assert_allclose(m, ne, atol=1e-14)


def test_single_point_filament(oracle_mod):
    X = np.zeros((1, 3))
    D = np.eye(3).reshape(1, 9)
    g, m = oracle_mod.rod_forces([0, 1], X, D, _rod())
    assert np.all(g == 0) and np.all(m == 0)


def test_relaxation_dissipates_energy(oracle_mod):
    e = _perturbed(5, F=2, M=24)
    rod = synth.RodParams((1e-3, 1e-3, 1e-3), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), e.ds)
    X, D = e.X, e.D
    z = np.zeros_like(X)
    E = [oracle_mod.rod_energy(e.offsets, X, D, rod)]
    for _ in range(15):
        X, D, _, _ = oracle_mod.step(e.offsets, X, D, rod, z, z, e.eps, 1.0, oracle_mod.EULER, 2e-4, 1)
        E.append(oracle_mod.rod_energy(e.offsets, X, D, rod))
    E = np.array(E)
    assert np.all(np.diff(E) < 0), E
    assert E[-1] < 0.97 * E[0]
