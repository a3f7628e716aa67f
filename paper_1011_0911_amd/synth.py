"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module draws random numbers and nothing else of the method: it holds no
Dirac-operator, solver or network arithmetic.  Both sides receive the arrays it
returns as plain inputs, so a parity test never depends on how either side
would have generated them.

Layouts (canonical, complex128):
  * site index  lex = ((x0*L1 + x1)*L2 + x2)*L3 + x3   (x0 = time, slowest)
  * gauge field U[lex, mu, a, b]        shape (V, 4, 3, 3)
  * spinor      psi[lex, s, c]          shape (V, 4, 3)
  * even field  psi_e[lex >> 1, s, c]   shape (V/2, 4, 3), even sites only

Link recipe (the paper runs on dynamical beta=5.3 ensembles that are not
available; these random SU(3) fields stand in for them): for every link draw a
3x3 complex matrix with independent N(0,1) real and imaginary parts, take its
Hermitian part, remove the trace, and exponentiate U = exp(i*eps*H) through a
Hermitian eigen-decomposition.  Links are drawn in canonical order (site, then
direction) from one numpy Generator seeded with `seed`.
"""
from __future__ import annotations

import numpy as np


def volume(L):
    L = tuple(int(v) for v in L)
    if len(L) != 4:
        raise ValueError("lattice must have 4 extents (L0 = time, L1, L2, L3)")
    v = 1
    for x in L:
        v *= x
    return v


def random_su3_links(L, eps: float, seed: int) -> np.ndarray:
    """U_mu(x) = exp(i*eps*H), H traceless Hermitian with Gaussian entries."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((V, 4, 3, 3, 2))
    a = g[..., 0] + 1j * g[..., 1]
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    U = np.einsum("...ij,...j,...kj->...ik", v, ph, np.conj(v), optimize=True)
    return np.ascontiguousarray(U.astype(np.complex128))


def unit_links(L) -> np.ndarray:
    V = volume(L)
    U = np.zeros((V, 4, 3, 3), np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def gaussian_field(nsites: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Gaussian spinor field(s): Re and Im of every component ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    shape = (nsites, 4, 3, 2) if nrhs is None else (nrhs, nsites, 4, 3, 2)
    g = rng.standard_normal(shape)
    return np.ascontiguousarray(g[..., 0] + 1j * g[..., 1])


def gaussian_field_device(nsites: int, seed: int, nrhs: int, device="cuda"):
    """Gaussian spinor fields generated on the device (torch, complex128, shape
    (nrhs, nsites, 4, 3)): Re and Im ~ N(0,1) from a generator seeded with
    `seed`.  For bulk inputs whose values no CPU check needs (training sources)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    g = torch.randn((nrhs, nsites, 4, 3, 2), dtype=torch.float64, device=device, generator=gen)
    return torch.view_as_complex(g).contiguous()


def random_gauge_transform(L, seed: int) -> np.ndarray:
    """One random SU(3) matrix per site (for covariance checks), shape (V,3,3)."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((V, 3, 3, 2))
    a = g[..., 0] + 1j * g[..., 1]
    q, r = np.linalg.qr(a)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    q[..., :, 0] /= det[..., None]
    return np.ascontiguousarray(q)


def random_weights(n: int, seed: int, scale: float) -> np.ndarray:
    """Complex Gaussian values (network weights for tests), std `scale` per part."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 2)) * scale
    return np.ascontiguousarray(g[:, 0] + 1j * g[:, 1])


def even_sites(L) -> np.ndarray:
    """Canonical lex indices of the even sites, in the order of index lex >> 1."""
    V = volume(L)
    lex = np.arange(V)
    x3 = lex % L[3]
    x2 = (lex // L[3]) % L[2]
    x1 = (lex // (L[3] * L[2])) % L[1]
    x0 = lex // (L[3] * L[2] * L[1])
    par = (x0 + x1 + x2 + x3) & 1
    return lex[par == 0]


def odd_sites(L) -> np.ndarray:
    V = volume(L)
    lex = np.arange(V)
    x3 = lex % L[3]
    x2 = (lex // L[3]) % L[2]
    x1 = (lex // (L[3] * L[2])) % L[1]
    x0 = lex // (L[3] * L[2] * L[1])
    par = (x0 + x1 + x2 + x3) & 1
    return lex[par == 1]


# Seeds of the workloads (gauge field i: 1000+i; sources: 2000+100*i+r;
# training sources 3000+; test sources 4000+; deflation start fields 5000+).
def gauge_seed(cfg: int) -> int:
    return 1000 + cfg


def source_seed(cfg: int, r: int = 0) -> int:
    return 2000 + 100 * cfg + r


def dfl_seed(cfg: int) -> int:
    return 5000 + cfg
