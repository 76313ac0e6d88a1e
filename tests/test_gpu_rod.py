"""GPU parity of the rod stage (rotation square root, rod forces) against the
FP64 oracle (Sec. II.B, Alg. 1, Sec. III.B.1)."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth
from tests.gpu_util import dev, rod_of, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mrs():
    import paper_2604_12083_amd as m

    return m


@pytest.fixture(scope="module")
def ctx(mrs):
    c = mrs.mrs_context_create(0)
    yield c
    mrs.mrs_context_destroy(c)


def _rotsqrt_gpu(mrs, ctx, R):
    import torch

    dR = dev(R.reshape(-1, 9))
    dS = torch.empty_like(dR)
    mrs.mrs_rotsqrt_device(ctx, dR.shape[0], dR, dS, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return dS.cpu().numpy().reshape(-1, 3, 3)


def test_rotsqrt_random_and_edges(mrs, ctx):
    R = list(Rotation.random(2000, random_state=7).as_matrix())
    rng = np.random.default_rng(1)
    for th in (0.0, 1e-12, 1e-7, 1e-3, math.pi / 2, math.pi - 1e-3, math.pi - 1e-8, math.pi - 1e-12):
        for _ in range(8):
            R.append(Rotation.from_rotvec(th * synth._unit(rng.normal(size=3))).as_matrix())
    R = np.array(R)
    say(f"rotsqrt count={len(R)}")
    S = _rotsqrt_gpu(mrs, ctx, R)
    So = oracle.rotsqrt(R)
    ang = np.linalg.norm(Rotation.from_matrix(R).as_rotvec(), axis=1)
    for i in range(len(R)):
        assert np.linalg.norm(S[i] @ S[i] - R[i]) < 4e-15
        assert np.linalg.norm(S[i].T @ S[i] - np.eye(3)) < 4e-15
        if ang[i] < math.pi - 1e-6:  # unique principal root
            assert np.abs(S[i] - So[i]).max() < 1e-13, (i, ang[i])


def test_rotsqrt_table2_protocol(mrs, ctx):
    rng = np.random.default_rng(2604)
    axis = synth._unit(rng.normal(size=3))
    thetas = np.linspace(-0.1, math.pi + 0.1, 100)
    R = np.array([Rotation.from_rotvec(t * axis).as_matrix() for t in thetas])
    S = _rotsqrt_gpu(mrs, ctx, R)
    err = np.array([np.linalg.norm(S[i] @ S[i] - R[i]) for i in range(len(R))])
    say(f"table2 protocol: mean {err.mean():.3e} median {np.median(err):.3e} max {err.max():.3e}")
    assert err.max() <= 1.35e-14 and err.mean() <= 2.76e-15


def _rod_gpu(mrs, ctx, e, rod, fe=None, ne=None):
    import torch

    dX, dD = dev(e.X), dev(e.D)
    g = torch.empty_like(dX)
    m = torch.empty_like(dX)
    mrs.mrs_rod_forces_device(ctx, e.offsets, dX, dD, rod_of(mrs, rod), None if fe is None else dev(fe),
                              None if ne is None else dev(ne), g, m, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return g.cpu().numpy(), m.cpu().numpy()


def _perturb(e, seed, sx=2e-3, sr=0.05):
    rng = np.random.default_rng(seed)
    e = e.copy()
    e.X = e.X + rng.normal(scale=sx, size=e.X.shape)
    rot = Rotation.from_rotvec(rng.normal(scale=sr, size=(e.N, 3))).as_matrix()
    e.D = np.einsum("pab,pib->pia", rot, e.D.reshape(e.N, 3, 3)).reshape(e.N, 9)
    return e


@pytest.mark.parametrize("case", ["rod64", "ens12800", "long300", "tiny", "bigturn"])
def test_rod_forces_parity(mrs, ctx, case):
    if case == "rod64":
        e = _perturb(synth.rod64(), 1)
    elif case == "ens12800":
        e = _perturb(synth.ens12800(), 2)
    elif case == "long300":  # longer than one block chunk of nodes
        e = _perturb(synth.filaments(3, 300, 1.0, 3, draw_loads=True), 3)
    elif case == "tiny":  # filaments of 1 and 2 points
        e = synth.filaments(4, 2, 1.0, 4)
        e.offsets = np.array([0, 1, 3, 5, 8], dtype=np.int32)
    else:  # large frame rotations between neighbours (near-pi segment rotations)
        e = _perturb(synth.filaments(2, 40, 1.0, 5), 5, sr=1.2)
    rod = synth.RodParams((0.3, 0.2, 0.1), (1.0, 1.5, 2.0), (0.1, -0.2, 0.3), e.ds)
    say(f"rod_forces {case} N={e.N}")
    g, m = _rod_gpu(mrs, ctx, e, rod, e.f, e.n)
    go, mo = oracle.rod_forces(e.offsets, e.X, e.D, rod, e.f, e.n)
    # absolute error relative to the largest load (ends are exact zeros of the elastic part)
    sg, sm = np.abs(go).max(), np.abs(mo).max()
    eg, em = np.abs(g - go).max() / sg, np.abs(m - mo).max() / sm
    say(f"  max err g {eg:.3e} m {em:.3e}")
    assert eg <= 1e-12 and em <= 1e-12
    # per point: a point's force is the difference of its two segment forces
    # plus its external force (Eq. discrete_f), so its error is measured
    # against the size of those terms; the segment forces are the running
    # sums of (g - f) along each filament (the last one is zero)
    worst = 0.0
    for a, b in zip(e.offsets[:-1], e.offsets[1:]):
        seg = np.cumsum(go[a:b] - e.f[a:b], axis=0)
        prev = np.vstack([np.zeros((1, 3)), seg[:-1]])
        scale = np.linalg.norm(seg, axis=1) + np.linalg.norm(prev, axis=1) + np.linalg.norm(e.f[a:b], axis=1)
        d = np.linalg.norm(g[a:b] - go[a:b], axis=1)
        worst = max(worst, float(np.max(d / np.where(scale > 0, scale, 1.0))))
        assert np.all(d <= 1e-12 * scale + 1e-300)
    say(f"  per-point g error / size of its terms: {worst:.3e}")
