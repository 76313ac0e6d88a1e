"""FP64 CPU oracle for the MRS filament hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this package to produce expected values.  The product
library never imports, links or calls it, and it shares no code with the HIP
path.  The arithmetic lives in ``mrs_oracle.c`` (plain C, double precision);
each of its functions cites the passage of arxiv 2604.12083 it restates.

Parity status per function (how each is pinned independently of itself is
listed in the tests under ``tests/test_oracle_*.py``):
  mrs_field / mrs_eval      pinned (symbolic re-derivation from the blob,
                            Stokes-equation residuals by finite differences,
                            singular far-field limits, reciprocity,
                            translation/rotation invariance, brute-force
                            mobility matrix on tiny inputs)
  rotsqrt                   pinned (S^2 = R, orthogonality, scipy sqrtm,
                            principal-branch trace, Table II magnitudes)
  rodrigues                 pinned (scipy expm of the skew matrix)
  rod_forces / rod_energy   pinned (closed forms for stretch, twist and bend,
                            force and torque balance, frame indifference,
                            energy dissipation under relaxation)
  step (Euler, RK2, RK4)    pinned (convergence orders 1, 2 and 4, reduction
                            of one RK stage to Euler, energy decay)
  swimming waveform         pinned (a rod built in the preferred shape of
                            time t carries no elastic load, and loads at
                            other times; zero amplitude reduces to Omega_0)
  lj_forces / lj_energy     pinned (closed-form pair force, force = minus the
                            finite-difference gradient of the energy, cutoff,
                            same-filament exclusion, zero total force and
                            torque)
Absolute U/Omega values of the configured workloads are "parity unpinned"
by the paper itself, which prints none.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compile mrs_oracle.c into liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-Wno-unused-parameter",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_blob.restype = ctypes.c_double
            lib.oracle_blob.argtypes = [ctypes.c_double, ctypes.c_double]
            lib.oracle_hfuncs.argtypes = [ctypes.c_double, ctypes.c_double, _d]
            lib.oracle_mrs_field.argtypes = [ctypes.c_int64, _d, ctypes.c_int64, _d, _d, _d,
                                             ctypes.c_double, ctypes.c_double, _d, _d]
            lib.oracle_mrs_eval.argtypes = [ctypes.c_int64, _d, _d, _d, ctypes.c_double,
                                            ctypes.c_double, _d, _d]
            lib.oracle_rotsqrt_batch.argtypes = [ctypes.c_int64, _d, _d]
            lib.oracle_rotsqrt_literal.argtypes = [_d, _d, ctypes.c_double, ctypes.c_double]
            lib.oracle_rodrigues.argtypes = [_d, _d, _d]
            lib.oracle_rod_forces.argtypes = [ctypes.c_int32, _i32, _d, _d, _d, _d, _d,
                                              ctypes.c_double, _d, _d, _d, _d]
            lib.oracle_rod_forces_ex.argtypes = [ctypes.c_int32, _i32, _d, _d, _d, _d, _d, ctypes.c_double,
                                                 _d, _d, _d, ctypes.c_double, _d, _d, _d]
            lib.oracle_lj_forces.argtypes = [ctypes.c_int32, _i32, _d, _d, _d]
            lib.oracle_lj_energy.restype = ctypes.c_double
            lib.oracle_lj_energy.argtypes = [ctypes.c_int32, _i32, _d, _d]
            lib.oracle_velocities_ex.argtypes = [ctypes.c_int32, _i32, _d, _d, _d, _d, _d, ctypes.c_double,
                                                 _d, _d, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                 _d, ctypes.c_double, _d, _d, _d]
            lib.oracle_step_ex.argtypes = [ctypes.c_int32, _i32, _d, _d, _d, _d, _d, ctypes.c_double, _d, _d,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int32, ctypes.c_int, _d, _d, _d, _d, _d]
            lib.oracle_rod_energy.restype = ctypes.c_double
            lib.oracle_rod_energy.argtypes = [ctypes.c_int32, _i32, _d, _d, _d, _d, _d,
                                              ctypes.c_double]
            lib.oracle_reorthonormalize.argtypes = [ctypes.c_int64, _d]
            lib.oracle_velocities.argtypes = [ctypes.c_int32, _i32, _d, _d, _d, _d, _d,
                                              ctypes.c_double, _d, _d, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int, _d, _d]
            lib.oracle_step.argtypes = [ctypes.c_int32, _i32, _d, _d, _d, _d, _d,
                                        ctypes.c_double, _d, _d, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int, _d, _d]
            lib.oracle_num_threads.restype = ctypes.c_int
            lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
            _lib = lib
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _p(a):
    return None if a is None else a.ctypes.data_as(_d)


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def blob(r: float, eps: float) -> float:
    return _load().oracle_blob(float(r), float(eps))


def hfuncs(r: float, eps: float) -> np.ndarray:
    H = np.zeros(5)
    _load().oracle_hfuncs(float(r), float(eps), _p(H))
    return H


def mrs_field(xt, X, f, n, eps, mu=1.0):
    """U, Omega at arbitrary targets xt (nt x 3) from sources X, f, n (ns x 3)."""
    xt, X, f, n = (_f64(v).reshape(-1, 3) for v in (xt, X, f, n))
    U = np.zeros_like(xt)
    W = np.zeros_like(xt)
    _load().oracle_mrs_field(xt.shape[0], _p(xt), X.shape[0], _p(X), _p(f), _p(n),
                             float(eps), float(mu), _p(U), _p(W))
    return U, W


def mrs_eval(X, f, n, eps, mu=1.0):
    """U, Omega at the source points themselves (Eq. superposition)."""
    X, f, n = (_f64(v).reshape(-1, 3) for v in (X, f, n))
    U = np.zeros_like(X)
    W = np.zeros_like(X)
    _load().oracle_mrs_eval(X.shape[0], _p(X), _p(f), _p(n), float(eps), float(mu), _p(U), _p(W))
    return U, W


def rotsqrt(R):
    """Principal square roots of a batch of rotations (..., 3, 3)."""
    R = _f64(R)
    shp = R.shape
    R = R.reshape(-1, 9)
    S = np.zeros_like(R)
    _load().oracle_rotsqrt_batch(R.shape[0], _p(R), _p(S))
    return S.reshape(shp)


def rotsqrt_literal(R, tol0=1e-12, tolpi=1e-8):
    R = _f64(R).reshape(9)
    S = np.zeros(9)
    _load().oracle_rotsqrt_literal(_p(R), _p(S), float(tol0), float(tolpi))
    return S.reshape(3, 3)


def rodrigues(v, D):
    v = _f64(v).reshape(3)
    D = _f64(D).reshape(3)
    out = np.zeros(3)
    _load().oracle_rodrigues(_p(v), _p(D), _p(out))
    return out


def _rod_args(rod):
    a = _f64(rod.a, (3,))
    b = _f64(rod.b, (3,))
    o = _f64(rod.omega0, (3,))
    return a, b, o, float(rod.ds)


def _wave(wave):
    """(A, k, f) of the swimming waveform, or None."""
    return None if wave is None else np.ascontiguousarray(wave, dtype=np.float64).reshape(3)


def _lj(lj):
    """(sigma, energy) of the Lennard-Jones repulsion, or None."""
    return None if lj is None else np.ascontiguousarray(lj, dtype=np.float64).reshape(2)


def rod_forces(offsets, X, D, rod, fext=None, next_=None, wave=None, t=0.0, lj=None):
    """Point force g and torque m on the fluid per node (N x 3 each); with the
    swimming waveform (A, k, f) at time t and the Lennard-Jones repulsion
    (sigma, energy) when given."""
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    X = _f64(X).reshape(-1, 3)
    D = _f64(D).reshape(-1, 9)
    a, b, o, ds = _rod_args(rod)
    fe = None if fext is None else _f64(fext).reshape(-1, 3)
    ne = None if next_ is None else _f64(next_).reshape(-1, 3)
    wv, lp = _wave(wave), _lj(lj)
    g = np.zeros_like(X)
    m = np.zeros_like(X)
    _load().oracle_rod_forces_ex(len(off) - 1, off.ctypes.data_as(_i32), _p(X), _p(D), _p(a), _p(b),
                                 _p(o), ds, _p(fe), _p(ne), _p(wv), float(t), _p(lp), _p(g), _p(m))
    return g, m


def lj_forces(offsets, X, lj):
    """Lennard-Jones force on every point from the points of other filaments."""
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    X = _f64(X).reshape(-1, 3)
    F = np.zeros_like(X)
    _load().oracle_lj_forces(len(off) - 1, off.ctypes.data_as(_i32), _p(X), _p(_lj(lj)), _p(F))
    return F


def lj_energy(offsets, X, lj) -> float:
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    X = _f64(X).reshape(-1, 3)
    return _load().oracle_lj_energy(len(off) - 1, off.ctypes.data_as(_i32), _p(X), _p(_lj(lj)))


def rod_energy(offsets, X, D, rod) -> float:
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    X = _f64(X).reshape(-1, 3)
    D = _f64(D).reshape(-1, 9)
    a, b, o, ds = _rod_args(rod)
    return _load().oracle_rod_energy(len(off) - 1, off.ctypes.data_as(_i32), _p(X), _p(D),
                                     _p(a), _p(b), _p(o), ds)


def reorthonormalize(D):
    D = _f64(D).reshape(-1, 9).copy()
    _load().oracle_reorthonormalize(D.shape[0], _p(D))
    return D


def velocities(offsets, X, D, rod, fext, next_, eps, mu=1.0, include_elastic=True, wave=None, t=0.0, lj=None):
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    X = _f64(X).reshape(-1, 3)
    D = _f64(D).reshape(-1, 9)
    a, b, o, ds = _rod_args(rod)
    fe = _f64(fext).reshape(-1, 3)
    ne = _f64(next_).reshape(-1, 3)
    U = np.zeros_like(X)
    W = np.zeros_like(X)
    _load().oracle_velocities_ex(len(off) - 1, off.ctypes.data_as(_i32), _p(X), _p(D), _p(a), _p(b),
                                 _p(o), ds, _p(fe), _p(ne), float(eps), float(mu),
                                 int(bool(include_elastic)), _p(_wave(wave)), float(t), _p(_lj(lj)),
                                 _p(U), _p(W))
    return U, W


EULER = 1
RK2 = 2
RK4 = 4


def step_ex(offsets, X, D, rod, fext, next_, eps, mu, integrator, dt, nsteps, include_elastic=True,
            wave=None, t=0.0, lj=None):
    """Advance (X, D) by nsteps from time t; returns new X, D, the first-stage
    U, Omega of the last step and the new time (t advanced by dt per step)."""
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    X = _f64(X).reshape(-1, 3).copy()
    D = _f64(D).reshape(-1, 9).copy()
    a, b, o, ds = _rod_args(rod)
    fe = _f64(fext).reshape(-1, 3)
    ne = _f64(next_).reshape(-1, 3)
    U = np.zeros_like(X)
    W = np.zeros_like(X)
    tt = np.array([float(t)])
    _load().oracle_step_ex(len(off) - 1, off.ctypes.data_as(_i32), _p(X), _p(D), _p(a), _p(b),
                           _p(o), ds, _p(fe), _p(ne), float(eps), float(mu), int(integrator),
                           float(dt), int(nsteps), int(bool(include_elastic)), _p(_wave(wave)), _p(tt),
                           _p(_lj(lj)), _p(U), _p(W))
    return X, D, U, W, float(tt[0])


def step(offsets, X, D, rod, fext, next_, eps, mu, integrator, dt, nsteps, include_elastic=True,
         wave=None, t=0.0, lj=None):
    """Advance (X, D) by nsteps; returns new X, D and first-stage U, Omega of the last step."""
    X, D, U, W, _ = step_ex(offsets, X, D, rod, fext, next_, eps, mu, integrator, dt, nsteps, include_elastic,
                            wave, t, lj)
    return X, D, U, W


def rel_err(a, b) -> float:
    """The paper's relative error form (Eq. true_err): max_i |a_i - b_i|_2 / |b_i|_2."""
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    return float(np.max(num / np.where(den == 0, 1.0, den))) if len(num) else 0.0


def parareal(offsets, X0, D0, rod, fext, next_, eps, mu, n_slices, fine_integ, fine_dt, fine_steps,
             coarse_steps, max_iter, tol=0.0, include_elastic=True):
    """Standard Parareal (Sec. II.D, Eqs. initial, intermediate, serial_correct).

    The slice propagators advance one time slice of length
    Delta T = fine_dt * fine_steps: F takes `fine_steps` steps of `fine_integ`,
    G takes `coarse_steps` forward-Euler steps (Sec. III.A: the coarse solver
    is explicit Euler).  The state of a slice boundary is (X, D); the
    correction of Eq. serial_correct is applied to both and the frames are
    re-orthonormalised afterwards.  Iteration k keeps slices n < k, sets
    slice k to its fine value and corrects slices k+1.. serially.  The
    iteration stops when the relative increment (Eq. true_err, second form)
    over all slice-boundary positions drops to `tol` or after `max_iter`.

    Returns (states, history): states[n] = (X, D) at T_n for n = 0..n_slices,
    history = list of relative increments per iteration.
    """
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    dT_coarse = fine_dt * fine_steps / coarse_steps

    def F(X, D):
        Xn, Dn, _, _ = step(off, X, D, rod, fext, next_, eps, mu, fine_integ, fine_dt, fine_steps, include_elastic)
        return Xn, Dn

    def G(X, D):
        Xn, Dn, _, _ = step(off, X, D, rod, fext, next_, eps, mu, EULER, dT_coarse, coarse_steps, include_elastic)
        return Xn, Dn

    # k = 0: serial coarse sweep (Eq. initial)
    U = [(np.array(X0, dtype=np.float64).reshape(-1, 3), np.array(D0, dtype=np.float64).reshape(-1, 9))]
    Gold = [None]
    for n in range(1, n_slices + 1):
        g = G(*U[n - 1])
        Gold.append(g)
        U.append(g)
    history = []
    for k in range(1, max_iter + 1):
        Fv = [None] + [F(*U[n - 1]) for n in range(1, n_slices + 1)]  # Eq. intermediate (in parallel)
        new = list(U[:k])
        new.append(Fv[k])
        Gnew = list(Gold)
        for n in range(k + 1, n_slices + 1):  # Eq. serial_correct
            g = G(*new[n - 1])
            Gnew[n] = g
            X = Fv[n][0] + g[0] - Gold[n][0]
            D = reorthonormalize(Fv[n][1] + g[1] - Gold[n][1])
            new.append((X, D))
        # Eq. true_err, second form: |x^k - x^{k-1}| / |x^k|
        inc = max(rel_err(U[n][0], new[n][0]) if n >= k else 0.0 for n in range(1, n_slices + 1))
        history.append(inc)
        U, Gold = new, Gnew
        if inc <= tol:
            break
    return U, history
