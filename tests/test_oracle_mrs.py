"""Pins of the oracle's MRS superposition sum (Sec. II.C, Eq. superposition).

Each test checks the oracle against something it does not compute itself:
  * the regularised Stokes equations, by finite differences of its own field:
    incompressibility, the rotlet momentum balance with the torque body force,
    the Stokeslet momentum balance with the pressure derived symbolically,
    omega = curl(u)/2 for both force and torque sources;
  * reciprocity (symmetry of the mobility), linearity, translation, rotation
    and permutation invariance;
  * a brute-force 6N x 6N mobility matrix built from the symbolic H1..H5.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from tests import symbolic


def _field(oracle_mod, x, X0, f, n, eps, mu=1.0):
    U, W = oracle_mod.mrs_field(np.atleast_2d(x), X0[None], f[None], n[None], eps, mu)
    return U, W


def _fd_points(x, h):
    pts = [x]
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        pts += [x + e, x - e]
    return np.array(pts)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_field_divergence_free_and_vorticity(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    eps, mu, h = 0.4, 1.7, 1e-4
    X0 = rng.normal(size=3)
    f = rng.normal(size=3)
    n = rng.normal(size=3)
    for dist in (0.1, 0.5, 2.0):
        d = rng.normal(size=3)
        x = X0 + dist * d / np.linalg.norm(d)
        U, W = _field(oracle_mod, _fd_points(x, h), X0, f, n, eps, mu)
        grad = np.zeros((3, 3))  # grad[c, k] = d u_k / d x_c
        for c in range(3):
            grad[c] = (U[1 + 2 * c] - U[2 + 2 * c]) / (2 * h)
        scale = np.abs(grad).max()
        assert abs(np.trace(grad)) <= 1e-6 * scale
        curl = np.array([grad[1, 2] - grad[2, 1], grad[2, 0] - grad[0, 2], grad[0, 1] - grad[1, 0]])
        np.testing.assert_allclose(W[0], 0.5 * curl, atol=1e-6 * scale)


def _laplacian(F, h):
    return sum(F[1 + 2 * c] - 2 * F[0] + F[2 + 2 * c] for c in range(3)) / h**2


@pytest.mark.parametrize("seed", [0, 1])
def test_rotlet_momentum_balance(oracle_mod, seed):
    # mu Lap u + curl(n phi)/2 = 0 with zero pressure, curl(n phi) = grad(phi) x n.
    rng = np.random.default_rng(seed)
    eps, mu, h = 0.5, 1.3, 1e-3
    X0 = rng.normal(size=3)
    n = rng.normal(size=3)
    for dist in (0.2, 0.7, 1.5):
        d = rng.normal(size=3)
        x = X0 + dist * d / np.linalg.norm(d)
        U, _ = _field(oracle_mod, _fd_points(x, h), X0, np.zeros(3), n, eps, mu)
        rv = x - X0
        r = np.linalg.norm(rv)
        phi = oracle_mod.blob(r, eps)
        dphi = -7.0 * r * phi / (r * r + eps * eps)  # derivative of the blob formula
        body = 0.5 * np.cross(dphi * rv / r, n)
        lap = mu * _laplacian(U, h)
        res = lap + body
        assert np.linalg.norm(res) <= 1e-5 * (np.linalg.norm(lap) + np.linalg.norm(body))


@pytest.mark.slow
@pytest.mark.parametrize("seed", [0, 1])
def test_stokeslet_momentum_balance(oracle_mod, seed):
    # mu Lap u - grad p + f phi = 0 with p = (f . r) G'(r)/r, G from Delta G = phi.
    Gp = symbolic.numeric()["Gp"]
    rng = np.random.default_rng(seed)
    eps, mu, h = 0.5, 0.8, 1e-3
    X0 = rng.normal(size=3)
    f = rng.normal(size=3)
    for dist in (0.2, 0.7, 1.5):
        d = rng.normal(size=3)
        x = X0 + dist * d / np.linalg.norm(d)
        pts = _fd_points(x, h)
        U, _ = _field(oracle_mod, pts, X0, f, np.zeros(3), eps, mu)

        def p(y):
            rv = y - X0
            r = np.linalg.norm(rv)
            return np.dot(f, rv) * Gp(r, eps) / r

        gradp = np.array([(p(pts[1 + 2 * c]) - p(pts[2 + 2 * c])) / (2 * h) for c in range(3)])
        phi = oracle_mod.blob(np.linalg.norm(x - X0), eps)
        lap = mu * _laplacian(U, h)
        res = lap - gradp + f * phi
        scale = np.linalg.norm(lap) + np.linalg.norm(gradp) + np.linalg.norm(f * phi)
        assert np.linalg.norm(res) <= 1e-5 * scale


def _random_cloud(rng, N, spread=1.0):
    return rng.normal(size=(N, 3)) * spread, rng.normal(size=(N, 3)), rng.normal(size=(N, 3))


def test_reciprocity(oracle_mod):
    rng = np.random.default_rng(5)
    X, f, n = _random_cloud(rng, 40, 0.3)
    f2, n2 = rng.normal(size=(40, 3)), rng.normal(size=(40, 3))
    eps = 0.05
    U, W = oracle_mod.mrs_eval(X, f, n, eps)
    U2, W2 = oracle_mod.mrs_eval(X, f2, n2, eps)
    lhs = np.sum(U * f2) + np.sum(W * n2)
    rhs = np.sum(U2 * f) + np.sum(W2 * n)
    scale = np.sum(np.abs(U * f2)) + np.sum(np.abs(W * n2))
    assert abs(lhs - rhs) <= 1e-13 * scale


def test_linearity(oracle_mod):
    rng = np.random.default_rng(6)
    X, f, n = _random_cloud(rng, 30)
    f2, n2 = rng.normal(size=(30, 3)), rng.normal(size=(30, 3))
    a, b, eps = 0.7, -1.9, 0.1
    U1, W1 = oracle_mod.mrs_eval(X, f, n, eps)
    U2, W2 = oracle_mod.mrs_eval(X, f2, n2, eps)
    U, W = oracle_mod.mrs_eval(X, a * f + b * f2, a * n + b * n2, eps)
    np.testing.assert_allclose(U, a * U1 + b * U2, rtol=1e-12, atol=1e-12 * np.abs(U).max())
    np.testing.assert_allclose(W, a * W1 + b * W2, rtol=1e-12, atol=1e-12 * np.abs(W).max())


def test_translation_rotation_permutation(oracle_mod):
    rng = np.random.default_rng(7)
    X, f, n = _random_cloud(rng, 50, 0.5)
    eps = 0.08
    U, W = oracle_mod.mrs_eval(X, f, n, eps)
    Ut, Wt = oracle_mod.mrs_eval(X + np.array([3.0, -1.25, 0.5]), f, n, eps)
    assert oracle_mod.rel_err(Ut, U) < 1e-13 and oracle_mod.rel_err(Wt, W) < 1e-13
    Q = Rotation.random(random_state=3).as_matrix()
    Ur, Wr = oracle_mod.mrs_eval(X @ Q.T, f @ Q.T, n @ Q.T, eps)
    assert oracle_mod.rel_err(Ur, U @ Q.T) < 1e-13 and oracle_mod.rel_err(Wr, W @ Q.T) < 1e-13
    perm = rng.permutation(50)
    Up, Wp = oracle_mod.mrs_eval(X[perm], f[perm], n[perm], eps)
    assert oracle_mod.rel_err(Up, U[perm]) < 1e-13 and oracle_mod.rel_err(Wp, W[perm]) < 1e-13


def _skew(v):
    return np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])


@pytest.mark.slow
@pytest.mark.parametrize("N", [1, 2, 3, 5, 8])
def test_bruteforce_mobility_matrix(oracle_mod, N):
    """Explicit 6N x 6N mobility built from the symbolic kernels; r_ij = x_i - x_j."""
    import sympy as sp

    d = symbolic.derive()
    Hn = symbolic.numeric()["H"]
    rng = np.random.default_rng(100 + N)
    eps, mu = 0.15, 0.9
    X, f, n = _random_cloud(rng, N, 0.2)
    H0 = [float(sp.limit(h, symbolic.r, 0).subs(symbolic.eps, eps)) for h in (d["H"][0], d["H"][3])]
    Mob = np.zeros((6 * N, 6 * N))
    for i in range(N):
        for j in range(N):
            rv = X[i] - X[j]
            r = np.linalg.norm(rv)
            if i == j:
                H1, H2, H3, H4, H5 = H0[0], 0.0, 0.0, H0[1], 0.0
            else:
                H1, H2, H3, H4, H5 = (h(r, eps) for h in Hn)
            rr = np.outer(rv, rv)
            Mob[6 * i:6 * i + 3, 6 * j:6 * j + 3] = H1 * np.eye(3) + H2 * rr
            Mob[6 * i:6 * i + 3, 6 * j + 3:6 * j + 6] = -H3 * _skew(rv)  # n x r
            Mob[6 * i + 3:6 * i + 6, 6 * j:6 * j + 3] = -H3 * _skew(rv)  # f x r
            Mob[6 * i + 3:6 * i + 6, 6 * j + 3:6 * j + 6] = H4 * np.eye(3) + H5 * rr
    y = Mob @ np.concatenate([f, n], axis=1).reshape(-1) / mu
    y = y.reshape(N, 6)
    U, W = oracle_mod.mrs_eval(X, f, n, eps, mu)
    assert oracle_mod.rel_err(U, y[:, :3]) < 1e-12
    assert oracle_mod.rel_err(W, y[:, 3:]) < 1e-12
    np.testing.assert_allclose(Mob, Mob.T, atol=1e-12 * np.abs(Mob).max())


def test_config_shapes_and_frames():
    e = synth.rod64()
    assert e.N == 64 and e.eps == pytest.approx(1.5 / 64)
    e2 = synth.ens12800()
    assert e2.N == 12800 and e2.n_fil == 100
    for ens in (e, e2):
        D = ens.D.reshape(-1, 3, 3)
        np.testing.assert_allclose(np.einsum("kij,klj->kil", D, D), np.broadcast_to(np.eye(3), D.shape), atol=1e-14)
        np.testing.assert_allclose(np.linalg.det(D), 1.0, atol=1e-14)
    again = synth.ens12800()
    assert np.array_equal(again.X, e2.X) and np.array_equal(again.f, e2.f)
    sub = synth.ens256000_subset()
    assert len(sub) == 2048 and len(np.unique(sub)) == 2048
