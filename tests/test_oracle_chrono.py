"""Pins of the oracle's chronological inversion guess (Sect. 3: the solutions of
earlier inversions predict the next one): it is the least-squares combination
of the stored solutions, so it is exact when the source lies in the span of
their images, its residual is orthogonal to every image D psi_i, and no single
stored solution, however scaled, has a smaller residual.  And the deflation
refresh: a build started from an orthonormal basis with no inverse-iteration
rounds returns that basis."""
import numpy as np

import oracle as O
from paper_1011_0911_amd import synth as S

L = (4, 4, 4, 4)
V = 256


def setup():
    U = S.random_su3_links(L, 0.5, 31)
    A, Ai = O.clover(L, U, 0.1355, 1.9)
    prev = S.gaussian_field(V, 32, nrhs=4)
    return U, A, Ai, prev


def test_guess_exact_in_span():
    U, A, _, prev = setup()
    c = np.array([0.7 - 0.2j, -1.1j, 0.3, 2.0 + 0.5j])
    x = np.tensordot(c, prev, 1)
    eta = O.apply_D(L, U, A, x)
    g = O.chrono_guess(L, U, A, prev, eta)
    assert np.linalg.norm(g - x) < 1e-12 * np.linalg.norm(x)


def test_guess_residual_orthogonal_and_optimal():
    U, A, _, prev = setup()
    eta = S.gaussian_field(V, 33)
    g = O.chrono_guess(L, U, A, prev, eta)
    r = eta - O.apply_D(L, U, A, g)
    for p in prev:
        Dp = O.apply_D(L, U, A, p)
        assert abs(np.vdot(Dp, r)) < 1e-10 * np.linalg.norm(Dp) * np.linalg.norm(r)
        # the best multiple of one stored solution alone does no better
        a = np.vdot(Dp, eta) / np.vdot(Dp, Dp)
        assert np.linalg.norm(eta - a * Dp) >= np.linalg.norm(r) * (1 - 1e-12)


def test_refresh_without_rounds_keeps_an_orthonormal_basis():
    U, A, Ai, _ = setup()
    bs = (2, 2, 2, 2)
    d = O.Deflation(L, bs, 4)
    d.build(U, A, Ai, bs, 2, 4, 2, S.gaussian_field(V, 34, nrhs=4))
    W = d.basis()
    d2 = O.Deflation(L, bs, 4)
    d2.build(U, A, Ai, bs, 2, 4, 0, W)
    assert np.abs(d2.basis() - W).max() < 1e-13
    assert np.abs(d2.little() - d.little()).max() < 1e-12 * np.abs(d.little()).max()
