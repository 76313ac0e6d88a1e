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
