"""Pins of the oracle's link derivatives of S_eff (Eq. 4; the molecular-dynamics
forces of Sect. 2) against central finite differences of the action itself,
exp(eps T^a) acting on one link at a time or on all links at once, on the 2^4
and 4.4.2.2 lattices, term by term; plus gauge covariance and the cases where a
term has no link dependence (c_sw = 0 for the log-det term, dm = 0 for the
phi2 term)."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
from paper_1011_0911_amd import synth as S

KAPPA, CSW, DM = 0.13, 1.9, 0.2


def gell_mann():
    lam = np.zeros((8, 3, 3), np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return 0.5j * lam  # T^a = i lambda^a / 2


T = gell_mann()


def setup(L, seed):
    U = S.random_su3_links(L, 0.5, seed)
    V = int(np.prod(L))
    phi = S.gaussian_field(V // 2, seed + 1, nrhs=2)
    return U, phi


def term(L, U, phi, part, dm=DM, csw=CSW):
    _, t = O.s_eff(L, U, KAPPA, csw, dm, phi[0], phi[1])
    return {1: t[0], 2: t[1], 4: t[2]}[part]


def moved(U, omega, eps):
    """exp(eps omega(x, mu)) U_mu(x) for every link (omega: (V, 4, 3, 3))."""
    out = U.copy()
    for x in range(U.shape[0]):
        for mu in range(4):
            if np.any(omega[x, mu]):
                out[x, mu] = expm(eps * omega[x, mu]) @ U[x, mu]
    return out


def fd(L, U, phi, part, omega, h=1e-3, **kw):
    """4-point central difference (error O(h^4)) of the term along omega."""
    s = [term(L, moved(U, omega, e * h), phi, part, **kw) for e in (2, 1, -1, -2)]
    return (-s[0] + 8 * s[1] - 8 * s[2] + s[3]) / (12 * h)


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 2, 2)])
@pytest.mark.parametrize("part", [1, 2, 4])
def test_force_matches_finite_differences(L, part):
    U, phi = setup(L, 40 + len(L) + sum(L))
    f = O.force(L, U, KAPPA, CSW, DM, phi[0], phi[1], parts=part)
    V = int(np.prod(L))
    scale = np.abs(f).max()
    assert scale > 1e-3
    rng = np.random.default_rng(part + V)
    # single components at random links (and one time-boundary link, where the
    # fermion sign enters the hop but not the clover leaves)
    picks = [(int(rng.integers(V)), int(rng.integers(4)), int(rng.integers(8))) for _ in range(5)]
    picks.append((V - 1, 0, int(rng.integers(8))))
    for x, mu, a in picks:
        om = np.zeros((V, 4, 3, 3), np.complex128)
        om[x, mu] = T[a]
        d = fd(L, U, phi, part, om)
        assert abs(d - f[x, mu, a]) < 1e-7 * scale, (x, mu, a, d, f[x, mu, a])
    # every link at once along a random direction: the directional derivative
    c = rng.standard_normal((V, 4, 8))
    om = np.einsum("xma,aij->xmij", c, T)
    d = fd(L, U, phi, part, om)
    ref = float((c * f).sum())
    assert abs(d - ref) < 1e-7 * np.abs(c * f).sum(), (d, ref)


def test_total_force_is_sum_of_terms():
    L = (4, 4, 2, 2)
    U, phi = setup(L, 61)
    parts = [O.force(L, U, KAPPA, CSW, DM, phi[0], phi[1], parts=p) for p in (1, 2, 4)]
    tot = O.force(L, U, KAPPA, CSW, DM, phi[0], phi[1], parts=7)
    assert np.abs(tot - sum(parts)).max() < 1e-12 * np.abs(tot).max()


def test_force_vanishing_terms():
    L = (4, 4, 2, 2)
    U, phi = setup(L, 62)
    # c_sw = 0: the log-det term does not depend on the links
    f0 = O.force(L, U, KAPPA, 0.0, DM, phi[0], phi[1], parts=1)
    assert np.abs(f0).max() == 0.0
    # dm = 0: the phi2 term is |phi2|^2
    assert np.abs(O.force(L, U, KAPPA, CSW, 0.0, phi[0], phi[1], parts=4)).max() == 0.0
    # phi1 term at c_sw = 0 still moves with the hops: finite differences agree
    f = O.force(L, U, KAPPA, 0.0, DM, phi[0], phi[1], parts=2)
    om = np.zeros((64, 4, 3, 3), np.complex128)
    om[5, 2] = T[3]
    d = fd(L, U, phi, 2, om, csw=0.0)
    assert abs(d - f[5, 2, 3]) < 1e-7 * np.abs(f).max()


def test_force_gauge_covariance():
    # U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag, phi(x) -> g(x) phi(x): S_eff is unchanged
    # and the force matrices F = sum_a f^a T^a transform as F -> g(x) F g(x)^dag
    L = (4, 4, 2, 2)
    U, phi = setup(L, 63)
    V = int(np.prod(L))
    g = S.random_su3_links(L, 1.0, 64)[:, 0]
    Ug = np.empty_like(U)
    x = np.indices(L).reshape(4, -1).T
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % L[mu]
        ly = np.ravel_multi_index(y.T, L)
        Ug[:, mu] = g @ U[:, mu] @ g[ly].conj().transpose(0, 2, 1)
    ev, _ = O._sites(L)
    phig = np.einsum("xab,rxsb->rxsa", g[ev], phi)
    f = O.force(L, U, KAPPA, CSW, DM, phi[0], phi[1])
    fg = O.force(L, Ug, KAPPA, CSW, DM, phig[0], phig[1])
    F = np.einsum("xma,aij->xmij", f, T)
    Fg = np.einsum("xma,aij->xmij", fg, T)
    ref = g[:, None] @ F @ g[:, None].conj().transpose(0, 1, 3, 2)
    assert np.abs(Fg - ref).max() < 1e-10 * np.abs(F).max()
