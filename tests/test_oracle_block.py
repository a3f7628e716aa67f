"""Pins of the oracle's Dirichlet block solves (the BiCGstab block inversions of
the DD-HMC forces, Sect. 3): on lattices with at least two blocks per
direction, D_Lambda is the restriction of D to the block's sites (a hop that
leaves the block is exactly an entry outside the block's rows and columns), so
each block solution is compared with a dense LU solve of that restriction built
from the oracle's D; plus the block structure (a block's solution does not see
the source elsewhere), the reported residual, sampled blocks, and zero sources."""
import numpy as np
import pytest

import oracle as O
from paper_1011_0911_amd import synth as S

KAPPA, CSW = 0.1357, 1.9


def block_sites(L, bs, blk):
    nb = [L[i] // bs[i] for i in range(4)]
    c = np.unravel_index(blk, nb)
    x = np.indices(bs).reshape(4, -1).T + np.array(c) * np.array(bs)
    return np.ravel_multi_index(x.T, L)  # lexicographic order within the block


def dense_block(L, U, A, sites):
    V = int(np.prod(L))
    n = sites.size * 12
    cols = []
    for s in sites:
        for k in range(12):
            e = np.zeros((V, 12), np.complex128)
            e[s, k] = 1.0
            cols.append(O.apply_D(L, U, A, e.reshape(V, 4, 3)).reshape(V, 12)[sites].reshape(-1))
    return np.stack(cols, 1).reshape(n, n)


@pytest.mark.parametrize("L,bs", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 4, 4, 4), (4, 2, 2, 2))])
def test_block_solve_matches_dense_restriction(L, bs):
    U = S.random_su3_links(L, 0.6, 31)
    A, Ai = O.clover(L, U, KAPPA, CSW)
    V = int(np.prod(L))
    eta = S.gaussian_field(V, 32)
    psi, it, res = O.block_solve(L, U, A, Ai, bs, eta, tol=1e-12)
    nblk = int(np.prod([L[i] // bs[i] for i in range(4)]))
    assert it.size == nblk and np.all(it > 0) and np.all(res <= 1e-12)
    for blk in (0, nblk // 2 + 1, nblk - 1):
        sites = block_sites(L, bs, blk)
        D = dense_block(L, U, A, sites)
        ref = np.linalg.solve(D, eta.reshape(V, 12)[sites].reshape(-1))
        got = psi.reshape(V, 12)[sites].reshape(-1)
        # |r_e| <= 1e-12 |b| on the reduced system; the full-block error is within
        # a modest condition factor of that
        assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max(), blk
        # and the block residual itself
        assert np.linalg.norm(D @ got - eta.reshape(V, 12)[sites].reshape(-1)) < 1e-10 * np.linalg.norm(ref)


def test_block_solve_structure():
    L, bs = (8, 4, 4, 4), (4, 2, 2, 2)
    U = S.random_su3_links(L, 0.6, 33)
    A, Ai = O.clover(L, U, KAPPA, CSW)
    V = int(np.prod(L))
    eta = S.gaussian_field(V, 34)
    psi, it, _ = O.block_solve(L, U, A, Ai, bs, eta, tol=1e-10)
    # the source outside block 5 does not reach it
    sites = block_sites(L, bs, 5)
    eta2 = S.gaussian_field(V, 35)
    eta2.reshape(V, 12)[sites] = eta.reshape(V, 12)[sites]
    psi2, _, _ = O.block_solve(L, U, A, Ai, bs, eta2, tol=1e-10)
    assert np.array_equal(psi2.reshape(V, 12)[sites], psi.reshape(V, 12)[sites])
    # solving a list of blocks gives the same values on them, zero elsewhere
    psi3, it3, _ = O.block_solve(L, U, A, Ai, bs, eta, tol=1e-10, blocks=[5, 2])
    for b, k in ((5, 0), (2, 1)):
        s = block_sites(L, bs, b)
        assert np.array_equal(psi3.reshape(V, 12)[s], psi.reshape(V, 12)[s]) and it3[k] == it[b]
    others = np.setdiff1d(np.arange(V), np.concatenate([block_sites(L, bs, 5), block_sites(L, bs, 2)]))
    assert np.abs(psi3.reshape(V, 12)[others]).max() == 0.0
    # zero source: zero solution without iterations
    psi0, it0, res0 = O.block_solve(L, U, A, Ai, bs, np.zeros_like(eta), tol=1e-10)
    assert np.abs(psi0).max() == 0.0 and np.all(it0 == 0) and np.all(res0 == 0)
