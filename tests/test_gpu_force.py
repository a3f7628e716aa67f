"""GPU link derivatives of S_eff (Eq. 4; the molecular-dynamics forces of Sect. 2)
against the oracle's, element by element, term by term, with the plain and the
deflated solver; invalid calls; gauge covariance at the 32^3x64 size; and, at
16^4, the directional derivative of the GPU's own S_eff.

Tolerances: the log-det term involves no solve (1e-12 of the largest component);
the pseudofermion terms are bilinear in solutions that meet relative residual
1e-10 with a condition number of order 10 on these fields, so their components
agree to ~1e-9 of the largest; 1e-7 is asserted."""
import numpy as np
import pytest

from paper_1011_0911_amd import synth as S
from tests.gpu_util import make_ctx, to_np

pytestmark = pytest.mark.gpu
KAPPA, CSW, DM = 0.1357, 1.9, 0.2


@pytest.fixture(scope="module")
def Q():
    from paper_1011_0911_amd import qdd

    qdd.lib()
    return qdd


def gell_mann_T():
    lam = np.zeros((8, 3, 3), np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return 0.5j * lam


@pytest.mark.parametrize("terms", [1, 2, 4, 7])
def test_force_parity_plain(Q, orc, terms):
    # 4^4 (the oracle solves densely) with the unpreconditioned solver
    L = (4, 4, 4, 4)
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.6, KAPPA, CSW, 801, max_nrhs=2, force=1)
    phi = S.gaussian_field(V // 2, 802, nrhs=2)
    f, info = ctx.force(DM, phi[0], phi[1], terms)
    ref = orc.force(L, U, KAPPA, CSW, DM, phi[0], phi[1], parts=terms)
    f = to_np(f)
    e = np.abs(f - ref).max() / np.abs(ref).max()
    print(f"terms {terms}: max |f| {np.abs(ref).max():.3e} err {e:.2e}; solves {[i['iters'] for i in info]}")
    assert e < (1e-12 if terms == 1 else 1e-7)
    if terms & 6:
        assert all(i["converged"] and i["true_res"] <= 1e-10 for i in info)


def test_force_parity_deflated(Q, orc):
    # 8^4 with the SAP-preconditioned, deflated solver (FP32 SAP); the oracle solves by GMRES
    L = (8, 8, 8, 8)
    V = int(np.prod(L))
    BS = (4, 4, 4, 4)
    ctx, U = make_ctx(Q, L, 0.6, KAPPA, CSW, 803, max_nrhs=2, force=1, sap_bs=BS, sap_prec=1, dfl_Ns=8,
                      dfl_bs=BS, dfl_nit=3, precond=Q.PRECOND_DFL)
    ctx.dfl_build(S.gaussian_field(V, 804, nrhs=8))
    phi = S.gaussian_field(V // 2, 805, nrhs=2)
    f, info = ctx.force(DM, phi[0], phi[1], 7)
    ref = orc.force(L, U, KAPPA, CSW, DM, phi[0], phi[1], parts=7)
    e = np.abs(to_np(f) - ref).max() / np.abs(ref).max()
    print(f"deflated 8^4: err {e:.2e}; solves {[i['iters'] for i in info]}")
    assert e < 1e-7


def test_force_terms_add_and_invalid_calls(Q):
    L = (4, 4, 4, 8)
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.6, KAPPA, CSW, 806, max_nrhs=2, force=1)
    phi = S.gaussian_field(V // 2, 807, nrhs=2)
    parts = [to_np(ctx.force(DM, phi[0], phi[1], t)[0]) for t in (1, 2, 4)]
    tot = to_np(ctx.force(DM, phi[0], phi[1], 7)[0])
    assert np.abs(tot - sum(parts)).max() < 1e-9 * np.abs(tot).max()
    # dm = 0: the phi2 term does not depend on the links
    assert np.abs(to_np(ctx.force(0.0, phi[0], phi[1], 4)[0])).max() == 0.0
    for bad in ((-0.1, 7), (DM, 0), (DM, 8)):
        with pytest.raises(Q.QddError):
            ctx.force(bad[0], phi[0], phi[1], bad[1])
    plain, _ = make_ctx(Q, L, 0.6, KAPPA, CSW, 806, max_nrhs=2)  # created without config.force
    with pytest.raises(Q.QddError):
        plain.force(DM, phi[0], phi[1], 1)
    one, _ = make_ctx(Q, L, 0.6, KAPPA, CSW, 806, max_nrhs=1, force=1)
    with pytest.raises(Q.QddError):  # the pseudofermion terms solve two right-hand sides at once
        one.force(DM, phi[0], phi[1], 2)
    assert np.array_equal(to_np(one.force(DM, phi[0], phi[1], 1)[0]), parts[0])


def _gauge_transform(L, U, g):
    x = np.indices(L).reshape(4, -1).T
    Ug = np.empty_like(U)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % L[mu]
        Ug[:, mu] = g @ U[:, mu] @ g[np.ravel_multi_index(y.T, L)].conj().transpose(0, 2, 1)
    return Ug


def test_force_gauge_covariance_full_size(Q):
    # 32^3 x 64 with the FP16-storage SAP solver: under U_mu(x) -> g(x) U_mu(x)
    # g(x+mu)^dag, phi -> g phi the force matrices F = sum_a f^a T^a transform as
    # F(x, mu) -> g(x) F g(x)^dag
    import torch

    L = (64, 32, 32, 32)
    V = int(np.prod(L))
    cfg = dict(max_nrhs=2, force=1, sap_bs=(4, 4, 4, 4), sap_prec=2, precond=Q.PRECOND_SAP, nkv=8)
    U = S.random_su3_links(L, 0.6, 1003)
    g = S.random_su3_links(L, 1.0, 808)[:, 0]
    Ug = _gauge_transform(L, U, g)
    phi = S.gaussian_field(V // 2, 809, nrhs=2)
    ev = np.nonzero((np.indices(L).sum(0).reshape(-1) & 1) == 0)[0]
    phig = np.einsum("xab,rxsb->rxsa", g[ev], phi)
    out = []
    for UU, ph in ((U, phi), (Ug, phig)):
        ctx = Q.Context(L, Q.default_config(**cfg))
        ctx.set_gauge(torch.from_numpy(UU))
        ctx.set_params(KAPPA, CSW)
        f, info = ctx.force(DM, ph[0], ph[1], 7)
        print("solves", [i["iters"] for i in info], flush=True)
        assert all(i["converged"] for i in info)
        out.append(to_np(f))
        del ctx
        torch.cuda.empty_cache()
    T = gell_mann_T()
    F = np.einsum("xma,aij->xmij", out[0], T)
    Fg = np.einsum("xma,aij->xmij", out[1], T)
    ref = g[:, None] @ F @ g[:, None].conj().transpose(0, 1, 3, 2)
    e = np.abs(Fg - ref).max() / np.abs(F).max()
    print(f"gauge covariance at 32^3x64: {e:.2e}")
    assert e < 1e-7


def test_force_is_derivative_of_gpu_action(Q):
    # 16^4: the directional derivative of the GPU's S_eff (qdd_action) along a
    # random direction of all links, by a 4-point central difference, equals
    # sum c^a f^a of the GPU force
    import torch

    L = (16, 16, 16, 16)
    V = int(np.prod(L))
    U = S.random_su3_links(L, 0.6, 811)
    phi = S.gaussian_field(V // 2, 812, nrhs=2)
    ctx = Q.Context(L, Q.default_config(max_nrhs=2, force=1, sap_bs=(4, 4, 4, 4), sap_prec=1,
                                        precond=Q.PRECOND_SAP, tol=1e-12))
    ctx.set_gauge(torch.from_numpy(U))
    ctx.set_params(KAPPA, CSW)
    f = to_np(ctx.force(DM, phi[0], phi[1], 7)[0])
    rng = np.random.default_rng(813)
    c = rng.standard_normal((V, 4, 8))
    om = torch.from_numpy(np.einsum("xma,aij->xmij", c, gell_mann_T()))
    Ut = torch.from_numpy(U)

    def s_at(h):
        ctx.set_gauge(torch.linalg.matrix_exp(h * om) @ Ut)
        ctx.set_params(KAPPA, CSW)
        return ctx.action(DM, phi[0], phi[1])[0]

    h = 1e-3
    s = [s_at(e * h) for e in (2, 1, -1, -2)]
    d = (-s[0] + 8 * s[1] - 8 * s[2] + s[3]) / (12 * h)
    ref = float((c * f).sum())
    print(f"directional derivative: finite difference {d:.8e}, force {ref:.8e}, rel {abs(d - ref) / abs(ref):.2e}")
    assert abs(d - ref) < 1e-6 * np.abs(c * f).sum()
