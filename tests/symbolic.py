"""Symbolic re-derivation of the MRS kernel functions from the blob.

Independent of the oracle: starts from the blob phi_eps of Sec. II.C and
the regularised-Stokeslet construction, never from the closed forms the
oracle types in.

  Delta G = phi  (radial: (r^2 G')' = r^2 phi, G -> 0 at infinity)
  Delta B = G    (radial: (r^2 B')' = r^2 G, B' regular at 0)
  force f:   mu u = (f . grad) grad B - f G
             => H1 = B'/r - G,  H2 = (B'' - B'/r) / r^2
  torque n:  body force curl(n phi)/2 gives mu u = n x grad(G)/2
             => H3 = G'/(2 r)
  omega = curl(u)/2 of the torque field:
             mu omega = (n phi - (n . grad) grad G)/4
             => H4 = (phi - G'/r)/4,  H5 = -(G'' - G'/r) / (4 r^2)
"""
from __future__ import annotations

import functools

import sympy as sp

r, eps = sp.symbols("r epsilon", positive=True)


@functools.lru_cache(maxsize=1)
def derive():
    phi = 15 * eps**4 / (8 * sp.pi * (r**2 + eps**2) ** sp.Rational(7, 2))
    Gp = sp.integrate(r**2 * phi, r)
    Gp = sp.simplify((Gp - Gp.subs(r, 0)) / r**2)
    G = sp.integrate(Gp, r)
    G = sp.simplify(G - sp.limit(G, r, sp.oo))
    Bp = sp.integrate(r**2 * G, r)
    Bp = sp.simplify((Bp - sp.limit(Bp, r, 0)) / r**2)
    Bpp = sp.diff(Bp, r)
    Gpp = sp.diff(Gp, r)
    H = [
        sp.simplify(Bp / r - G),
        sp.simplify((Bpp - Bp / r) / r**2),
        sp.simplify(Gp / (2 * r)),
        sp.simplify((phi - Gp / r) / 4),
        sp.simplify(-(Gpp - Gp / r) / (4 * r**2)),
    ]
    return {"phi": phi, "G": G, "Gp": Gp, "Bp": Bp, "H": H}


@functools.lru_cache(maxsize=1)
def numeric():
    """Lambdified H1..H5(r, eps), phi(r, eps) and G'(r, eps) for numpy arrays."""
    d = derive()
    Hs = [sp.lambdify((r, eps), h, "numpy") for h in d["H"]]
    return {
        "H": Hs,
        "phi": sp.lambdify((r, eps), d["phi"], "numpy"),
        "Gp": sp.lambdify((r, eps), d["Gp"], "numpy"),
    }
