"""Helpers of the GPU parity tests (device transfers, tolerance checks)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def eval_dev(mrs, ctx, X, f, n, eps, mu, prec):
    import torch

    dX, df, dn = dev(X), dev(f), dev(n)
    U = torch.empty_like(dX)
    W = torch.empty_like(dX)
    s = torch.cuda.current_stream()
    mrs.mrs_eval_device(ctx, dX.shape[0], dX, df, dn, eps, mu, prec, U, W, s)
    torch.cuda.synchronize()
    return U.cpu().numpy(), W.cpu().numpy()


def rod_of(mrs, e_rod):
    return mrs.rod_params(e_rod.a, e_rod.b, e_rod.omega0, e_rod.ds)


def step_err(X1, X1o, X0):
    """Relative error of a step's displacement, max over points:
    |X1 - X1o| / |X1o - X0|, after removing the rounding of the stored
    positions themselves (each side rounds every component once, at most
    2 ulp of |X| together), which no arithmetic can avoid."""
    X1, X1o, X0 = (np.asarray(a, dtype=np.float64).reshape(len(a), -1) for a in (X1, X1o, X0))
    diff = np.linalg.norm(X1 - X1o, axis=1)
    slack = 2.0 * np.finfo(np.float64).eps * np.linalg.norm(X1o, axis=1)
    disp = np.linalg.norm(X1o - X0, axis=1)
    err = np.maximum(diff - slack, 0.0) / np.where(disp == 0, 1.0, disp)
    return float(err.max()) if len(err) else 0.0
