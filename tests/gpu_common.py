"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare with the oracle on the same seeded inputs."""

import math

import numpy as np

from oracle import fastfcm as ff


def oracle_params(w, Sigma_D=None):
    return ff.Params(L=w["L"], M=w["grid"], a=w["a"], Sigma=w["Sigma"], M_G=w["M_G"],
                     R_c=w["R_c"], eta=w.get("eta", 1.0), Sigma_D=Sigma_D)


def make_plan(w, precision, **kw):
    from paper_2310_12651_amd import Plan
    return Plan(w["N"], w["L"], w["a"], w["Sigma"], w["grid"], w["R_c"], eta=w.get("eta", 1.0),
                support=w["M_G"], precision=precision, **kw)


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_to_oracle_grid(g):
    """GPU field (3, z, y, x) -> oracle axis order (3, x, y, z)."""
    return np.ascontiguousarray(np.transpose(g, (0, 3, 2, 1)))


def oracle_to_gpu_grid(f):
    return np.ascontiguousarray(np.transpose(f, (0, 3, 2, 1)))


def normwise(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def eps_mean(V, U):
    """The paper's error measure (Sec. 5.1): mean over particles of |V-U|/|U|."""
    return float(np.mean(np.linalg.norm(V - U, axis=1) / np.linalg.norm(U, axis=1)))
