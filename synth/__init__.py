"""Seeded synthetic inputs for the MRS filament workloads.

This module only builds inputs: filament centrelines, material frames,
point forces and torques, perturbed time-slice states and request streams.
It holds none of the method's arithmetic (no blob, no kernel functions, no
rod mechanics, no time stepping), so both the FP64 oracle side and the GPU
side can draw identical inputs from it without sharing any of the method.

Geometry.  The paper's experiments use rod-shaped filaments discretised into
M points along a centreline, with an orthonormal material frame per point
whose third director is the unit tangent (Sec. II.A-II.B, Sec. IV.A).  A
filament here is a planar sinusoid of amplitude 0.1 and wavelength 1 about a
straight axis: X(s) = base + s d + 0.1 sin(2 pi s) p, s_k = k ds, ds = 1/M.

Frames.  D3 is the unit tangent of the analytic curve at s_k, D2 is the
plane normal d x p and D1 = D2 x D3, which makes every frame orthonormal and
right-handed.

Layouts.  Positions, forces and torques are row-major (N, 3) float64 arrays.
Frames are (N, 9) with D[k, 3*i + c] = component c of director D^{i+1} at
point k.  Filaments are concatenated and described by CSR offsets
(n_fil + 1 int32 entries).

Random draws use numpy's PCG64 generator (default_rng) in the fixed order
documented on each function; N(0, s) denotes a normal with standard
deviation s.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = [
    "Ensemble",
    "RodParams",
    "DEFAULT_ROD",
    "filaments",
    "rod64",
    "ens12800",
    "slices",
    "serving_requests",
    "ens256000",
    "ens256000_subset",
    "poisson_arrivals",
]


@dataclasses.dataclass
class RodParams:
    """Elastic moduli of the Kirchhoff rod and its intrinsic strain-twist.

    a = (bending, bending, twist) moduli, b = (shear, shear, stretch) moduli,
    omega0 = intrinsic strain-twist vector, ds = arclength spacing.
    """

    a: tuple = (1e-4, 1e-4, 1e-4)
    b: tuple = (1.0, 1.0, 1.0)
    omega0: tuple = (0.0, 0.0, 0.0)
    ds: float = 1.0 / 64.0


DEFAULT_ROD = RodParams()


@dataclasses.dataclass
class Ensemble:
    """One ensemble of filaments: state plus the per-point external loads."""

    offsets: np.ndarray  # (n_fil + 1,) int32 CSR offsets
    X: np.ndarray  # (N, 3) float64 positions
    D: np.ndarray  # (N, 9) float64 frames
    f: np.ndarray  # (N, 3) float64 point forces on the fluid
    n: np.ndarray  # (N, 3) float64 point torques on the fluid
    eps: float
    mu: float
    ds: float

    @property
    def N(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_fil(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def rod(self, a=DEFAULT_ROD.a, b=DEFAULT_ROD.b, omega0=DEFAULT_ROD.omega0) -> RodParams:
        return RodParams(tuple(a), tuple(b), tuple(omega0), self.ds)

    def copy(self) -> "Ensemble":
        return Ensemble(self.offsets.copy(), self.X.copy(), self.D.copy(),
                        self.f.copy(), self.n.copy(), self.eps, self.mu, self.ds)


def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _sinusoid(base, d, p, M, ds, amp=0.1, wavelength=1.0):
    """Centreline points and frames of one sinusoidal filament."""
    s = np.arange(M, dtype=np.float64) * ds
    k = 2.0 * math.pi / wavelength
    X = base[None, :] + s[:, None] * d[None, :] + (amp * np.sin(k * s))[:, None] * p[None, :]
    tangent = _unit(d[None, :] + (amp * k * np.cos(k * s))[:, None] * p[None, :])
    normal = np.broadcast_to(np.cross(d, p), (M, 3))
    D1 = np.cross(normal, tangent)
    D = np.concatenate([D1, normal, tangent], axis=1)
    return X, np.ascontiguousarray(D)


def filaments(F: int, M: int, box: float, seed, draw_loads: bool = True):
    """Seeded ensemble of F sinusoidal filaments of M points in [0, box]^3.

    Draw order from one default_rng(seed): bases (F x 3 uniform in the box),
    directions (F x 3 N(0,1), normalised), plane phases (F uniform on
    [0, 2 pi)), then forces f (N x 3 N(0,1)) and torques n (N x 3 N(0,1)).
    The sinusoid plane vector is p = cos(psi) p0 + sin(psi) (d x p0) with
    p0 = unit(d x a), a = e_x unless |d_x| > 0.9, then a = e_y.
    eps = 1.5 ds, mu = 1.
    """
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    ds = 1.0 / M
    bases = rng.uniform(0.0, box, size=(F, 3))
    dirs = _unit(rng.normal(size=(F, 3)))
    psi = rng.uniform(0.0, 2.0 * math.pi, size=F)
    N = F * M
    if draw_loads:
        f = rng.normal(size=(N, 3))
        n = rng.normal(size=(N, 3))
    else:
        f = np.zeros((N, 3))
        n = np.zeros((N, 3))
    Xs, Ds = [], []
    for i in range(F):
        d = dirs[i]
        a = np.array([0.0, 1.0, 0.0]) if abs(d[0]) > 0.9 else np.array([1.0, 0.0, 0.0])
        p0 = _unit(np.cross(d, a))
        p = math.cos(psi[i]) * p0 + math.sin(psi[i]) * np.cross(d, p0)
        X, D = _sinusoid(bases[i], d, p, M, ds)
        Xs.append(X)
        Ds.append(D)
    offsets = (np.arange(F + 1, dtype=np.int64) * M).astype(np.int32)
    return Ensemble(offsets, np.concatenate(Xs), np.concatenate(Ds), f, n,
                    eps=1.5 * ds, mu=1.0, ds=ds)


def rod64() -> Ensemble:
    """One filament of 64 points, X_k = (s_k, 0.1 sin 2 pi s_k, 0), s_k = k/64.

    Frames with plane normal e_z; eps = 1.5/64; mu = 1; f then n drawn
    N(0,1) (64 x 3 each) from default_rng(1).
    """
    M = 64
    ds = 1.0 / M
    X, D = _sinusoid(np.zeros(3), np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]), M, ds)
    rng = np.random.default_rng(1)
    f = rng.normal(size=(M, 3))
    n = rng.normal(size=(M, 3))
    return Ensemble(np.array([0, M], dtype=np.int32), X, D, f, n, eps=1.5 * ds, mu=1.0, ds=ds)


def ens12800() -> Ensemble:
    """100 filaments x 128 points in [0,10]^3 (12,800 points), seed 2."""
    return filaments(100, 128, 10.0, 2)


def ens256000() -> Ensemble:
    """1,000 filaments x 256 points in [0,50]^3 (256,000 points), seed 5."""
    return filaments(1000, 256, 50.0, 5)


def ens256000_subset(N: int = 256_000, k: int = 2048) -> np.ndarray:
    """Seeded check subset of targets for the 256,000-point ensemble."""
    return np.sort(np.random.default_rng(55).choice(N, k, replace=False)).astype(np.int64)


def slices(n_slices: int = 16, F: int = 32, M: int = 100, box: float = 10.0, seed: int = 3,
           sigma: float = 1e-3):
    """Base ensemble (32 filaments x 100 points, seed 3) and n_slices perturbed copies.

    After the base draws, the same rng draws per slice: a position
    perturbation (N x 3 N(0, sigma)) and a rotation vector per point
    (N x 3 N(0, sigma)); the slice frames are the base frames rotated by
    that rotation vector.  The external loads are the base draw's f, n.
    """
    rng = np.random.default_rng(seed)
    base = filaments(F, M, box, rng)
    slices = []
    for _ in range(n_slices):
        e = base.copy()
        e.X = base.X + rng.normal(scale=sigma, size=base.X.shape)
        rot = Rotation.from_rotvec(rng.normal(scale=sigma, size=(base.N, 3))).as_matrix()
        Dm = base.D.reshape(base.N, 3, 3)  # [point, director, component]
        e.D = np.ascontiguousarray(np.einsum("pab,pib->pia", rot, Dm).reshape(base.N, 9))
        slices.append(e)
    return base, slices


@dataclasses.dataclass
class SwimParams:
    """Parameters of the swimming workload (Sec. IV): waveform (A, k, f) of
    the preferred strain-twist (0, -k^2 A sin(k s + f t), 0), Lennard-Jones
    (sigma, energy) with sigma = 3 eps, rod moduli and the fine time step."""

    wave: tuple
    lj: tuple
    rod: RodParams
    dt: float


def swimmers(F: int, M: int = 51, box: float = 3.0, seed=11, height: float = 1.0, spread: float = 0.2,
             min_gap: float = 0.2, max_tries: int = 1000) -> Ensemble:
    """F straight swimmers of length 1 (M points, ds = 1/(M - 1)), lying
    parallel to the plane z = 0.

    Draw order from one default_rng(seed), per swimmer: centre (x, y) uniform
    in [0, box]^2, height uniform in [height - spread/2, height + spread/2],
    in-plane direction angle uniform on [0, 2 pi).  A swimmer with a point
    closer than min_gap to a point of an earlier one is drawn again (at most
    max_tries times).  Frames: D3 along the rod, D2 = e_z, D1 = D2 x D3, so
    the waveform bends the rod in the plane parallel to z = 0.  eps = 4 ds,
    mu = 1, no external loads (the waveform drives the swimmer).
    """
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    ds = 1.0 / (M - 1)
    s = np.arange(M) * ds - 0.5
    reach = 1.0 + min_gap
    cells = {}
    Xs, Ds = [], []
    for i in range(F):
        for _ in range(max_tries):
            cx, cy = rng.uniform(0.0, box, size=2)
            cz = rng.uniform(height - 0.5 * spread, height + 0.5 * spread)
            ang = rng.uniform(0.0, 2.0 * math.pi)
            d = np.array([math.cos(ang), math.sin(ang), 0.0])
            X = np.array([cx, cy, cz]) + s[:, None] * d[None, :]
            key = (int(cx // reach), int(cy // reach))
            near = [j for dx in (-1, 0, 1) for dy in (-1, 0, 1) for j in cells.get((key[0] + dx, key[1] + dy), [])]
            if all(np.min(np.linalg.norm(X[:, None, :] - Xs[j][None, :, :], axis=-1)) >= min_gap for j in near):
                break
        else:
            raise ValueError("swimmers: box too crowded for min_gap")
        cells.setdefault(key, []).append(i)
        d1 = np.cross([0.0, 0.0, 1.0], d)
        D = np.tile(np.concatenate([d1, [0.0, 0.0, 1.0], d]), (M, 1))
        Xs.append(X)
        Ds.append(D)
    N = F * M
    offsets = (np.arange(F + 1, dtype=np.int64) * M).astype(np.int32)
    return Ensemble(offsets, np.concatenate(Xs), np.concatenate(Ds), np.zeros((N, 3)), np.zeros((N, 3)),
                    eps=4.0 * ds, mu=1.0, ds=ds)


def swim_params(e: Ensemble, amplitude: float = 0.05, wavelength: float = 1.0, frequency: float = 20.0 * math.pi,
                lj_energy: float = 1e-4, a=(1e-3, 1e-3, 1e-3), b=(1.0, 1.0, 1.0), dt: float = 1e-6) -> SwimParams:
    """Waveform, Lennard-Jones and moduli of the swimming workload for ensemble e."""
    return SwimParams(wave=(amplitude, 2.0 * math.pi / wavelength, frequency), lj=(3.0 * e.eps, lj_energy),
                      rod=e.rod(a=a, b=b), dt=dt)


@dataclasses.dataclass
class RequestSpec:
    n_fil: int
    M: int
    kind: int  # 0 = one U/Omega evaluation, 1 = a run of RK4 steps
    seed: int


def serving_requests(n_req: int = 256, seed: int = 4):
    """Fixed request sequence of the serving workload.

    Per request, drawn in this order from default_rng(seed): filament count
    round(exp(U[ln 4, ln 1024])), points per filament uniform integer in
    [64, 256], kind 0/1 with probability 1/2, and a per-request seed used by
    `filaments(..., box=10)`.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_req):
        F = int(round(math.exp(rng.uniform(math.log(4), math.log(1024)))))
        M = int(rng.integers(64, 257))
        kind = int(rng.integers(0, 2))
        s = int(rng.integers(0, 2**31 - 1))
        out.append(RequestSpec(F, M, kind, s))
    return out


def poisson_arrivals(n: int, rate: float, seed: int = 44) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
