"""Shared helpers of the GPU parity tests (inputs from the seeded generators,
references from the CPU oracle)."""
import numpy as np

from paper_1011_0911_amd import synth as S


def relerr(a, b):
    """max |a - b| / max |b| (element-wise, stricter than the norm ratio)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def make_ctx(Q, L, eps, kappa, csw, seed, bc=-1, **cfg):
    import torch

    U = S.random_su3_links(L, eps, seed)
    c = Q.Context(L, Q.default_config(**cfg), bc=bc)
    c.set_gauge(torch.from_numpy(U))
    c.set_params(kappa, csw)
    return c, U


def to_np(t):
    return t.detach().cpu().numpy()
