"""Pins of the oracle's blob and kernel functions H1..H5 (Sec. II.C).

The paper prints the blob but not H1..H5 (it names them in Eqs.
velocity_field / angular_velocity_field and defers H1, H2 to the cited
Olson et al. model).  The oracle's closed forms are pinned here against
  * a symbolic derivation from the blob (tests/symbolic.py),
  * the normalisation of the blob (it integrates to one),
  * the point limits r = 0 (self-interaction) computed symbolically,
  * the singular Stokeslet / rotlet / potential-dipole limits for r >> eps,
    which are textbook forms independent of the regularisation.
"""
import math

import numpy as np
import pytest
import sympy as sp
from scipy import integrate

from tests import symbolic


@pytest.fixture(scope="module")
def sym():
    return symbolic.numeric()


def test_blob_integrates_to_one(oracle_mod):
    for eps in (0.01, 0.3, 2.0):
        val, err = integrate.quad(lambda x: 4 * math.pi * x * x * oracle_mod.blob(x, eps), 0, np.inf,
                                  limit=200)
        assert abs(val - 1.0) < 1e-8


def test_blob_matches_paper_formula_values(oracle_mod):
    # phi(0) = 15/(8 pi eps^3); phi decays like 15 eps^4/(8 pi r^7).
    eps = 0.2
    assert oracle_mod.blob(0.0, eps) == pytest.approx(15 / (8 * math.pi * eps**3), rel=1e-14)
    r = 1e3
    assert oracle_mod.blob(r, eps) == pytest.approx(15 * eps**4 / (8 * math.pi * r**7), rel=1e-6)


@pytest.mark.slow
def test_hfuncs_match_symbolic_derivation(oracle_mod, sym):
    rng = np.random.default_rng(11)
    for _ in range(200):
        eps = 10 ** rng.uniform(-3, 1)
        r = eps * 10 ** rng.uniform(-3, 3)
        want = np.array([h(r, eps) for h in sym["H"]])
        got = oracle_mod.hfuncs(r, eps)
        scale = np.array([1 / eps, 1 / eps**3, 1 / eps**2, 1 / eps**3, 1 / eps**5])
        # compare relative to each function's natural scale (H4 changes sign)
        assert np.all(np.abs(got - want) <= 1e-12 * np.maximum(np.abs(want), 1e-6 * scale)), (r, eps)


@pytest.mark.slow
def test_hfuncs_self_limit_symbolic(oracle_mod):
    d = symbolic.derive()
    lim = [sp.limit(h, symbolic.r, 0) for h in d["H"]]
    for eps in (0.05, 1.0, 3.0):
        got = oracle_mod.hfuncs(0.0, eps)
        want = [float(l.subs(symbolic.eps, eps)) for l in lim]
        # H2 and H5 multiply (f.r) r and (n.r) r, so only their finiteness matters at r=0
        assert got[0] == pytest.approx(want[0], rel=1e-14)
        assert got[2] == pytest.approx(want[2], rel=1e-14)
        assert got[3] == pytest.approx(want[3], rel=1e-14)
        assert np.all(np.isfinite(got))


def test_single_point_closed_form(oracle_mod):
    # One source at the target: U = f/(4 pi mu eps), Omega = 5 n/(16 pi mu eps^3).
    eps, mu = 0.07, 2.5
    X = np.array([[1.0, -2.0, 3.0]])
    f = np.array([[0.3, -1.1, 0.7]])
    n = np.array([[-0.4, 0.2, 0.9]])
    U, W = oracle_mod.mrs_eval(X, f, n, eps, mu)
    np.testing.assert_allclose(U, f / (4 * math.pi * mu * eps), rtol=1e-14)
    np.testing.assert_allclose(W, 5 * n / (16 * math.pi * mu * eps**3), rtol=1e-14)


def _singular(x, X0, f, n, mu):
    """Textbook singular Stokeslet + rotlet velocity and its vorticity/2."""
    rv = x - X0
    r = np.linalg.norm(rv)
    u = (f / r + np.dot(f, rv) * rv / r**3) / (8 * math.pi * mu) + np.cross(n, rv) / (8 * math.pi * mu * r**3)
    w = np.cross(f, rv) / (8 * math.pi * mu * r**3) + (-n / r**3 + 3 * np.dot(n, rv) * rv / r**5) / (16 * math.pi * mu)
    return u, w


def test_far_field_singular_limits(oracle_mod):
    rng = np.random.default_rng(3)
    mu = 1.3
    for _ in range(20):
        X0 = rng.normal(size=3)
        f = rng.normal(size=3)
        n = rng.normal(size=3)
        x = X0 + rng.normal(size=3) * 3
        r = np.linalg.norm(x - X0)
        for ratio in (1e-2, 1e-3):
            eps = ratio * r
            U, W = oracle_mod.mrs_field(x[None], X0[None], f[None], n[None], eps, mu)
            u, w = _singular(x, X0, f, n, mu)
            # deviation is O(eps^2/r^2)
            assert np.linalg.norm(U[0] - u) <= 20 * ratio**2 * np.linalg.norm(u)
            assert np.linalg.norm(W[0] - w) <= 20 * ratio**2 * np.linalg.norm(w)
