"""GPU parity of local deflation against the oracle: subspace build (SAP inverse
iteration + block Gram-Schmidt), the little Dirac operator, the little-operator
GCR, the two-level preconditioner and the deflated SAP-GCR solve.

Both sides run the same deterministic FP64 algorithm on the same start fields;
the basis and little operator agree to rounding (tolerance 1e-10 relative, the
Gram-Schmidt of nearly parallel SAP iterates amplifies rounding differences by
the conditioning of the start set)."""
import numpy as np
import pytest

from paper_1011_0911_amd import synth as S
from tests.gpu_util import make_ctx, relerr, to_np

pytestmark = pytest.mark.gpu
L = (8, 8, 8, 8)
BS = (4, 4, 4, 4)
NS = 6


@pytest.fixture(scope="module")
def Q():
    from paper_1011_0911_amd import qdd

    qdd.lib()
    return qdd


@pytest.fixture(scope="module")
def built(Q, orc):
    V = 4096
    ctx, U = make_ctx(Q, L, 0.5, 0.1355, 1.9, 47, sap_bs=BS, ncy=2, nmr=4, sap_prec=0, dfl_Ns=NS, dfl_bs=BS,
                      dfl_nit=2, dfl_coarse_tol=1e-12, precond=Q.PRECOND_DFL, max_nrhs=2)
    A, Ai = orc.clover(L, U, 0.1355, 1.9)
    init = S.gaussian_field(V, 48, nrhs=NS)
    ctx.dfl_build(init)
    d = orc.Deflation(L, BS, NS)
    d.build(U, A, Ai, BS, 2, 4, 2, init)
    return ctx, U, A, Ai, d


def test_dfl_basis_and_little_operator_parity(Q, built):
    ctx, U, A, Ai, d = built
    basis, little = ctx.dfl_export()
    basis, little = to_np(basis), to_np(little)
    eb = relerr(basis, d.basis())
    el = relerr(little, d.little())
    print(f"basis err {eb:.2e} little err {el:.2e}")
    assert eb < 1e-10 and el < 1e-10
    # block orthonormality of the GPU basis itself
    nb = np.array(L) // np.array(BS)
    x = np.array(np.unravel_index(np.arange(4096), L)).T
    bid = np.ravel_multi_index((x // np.array(BS)).T, nb)
    for b in (0, 7, 15):
        Wb = basis[:, bid == b].reshape(NS, -1)
        assert np.abs(Wb.conj() @ Wb.T - np.eye(NS)).max() < 1e-13


def test_coarse_solve_parity(Q, built):
    ctx, U, A, Ai, d = built
    f = S.gaussian_field(d.nblk * NS // 12, 49).reshape(d.nblk, NS)
    c_o, _ = d.coarse_solve(f, 1e-13)
    c_g, it = ctx.dfl_coarse_solve(f[None], 1e-13)
    e = relerr(to_np(c_g)[0], c_o)
    print("coarse iters", it, "err", e)
    assert e < 1e-10


def test_two_level_preconditioner_parity(Q, built):
    ctx, U, A, Ai, d = built
    r = S.gaussian_field(4096, 50, nrhs=2)
    out = to_np(ctx.dfl_precond(r))
    for k in range(2):
        ref = d.precond(U, A, Ai, BS, 2, 4, 1e-12, r[k])
        e = relerr(out[k], ref)
        print("precond err", e)
        assert e < 1e-9


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_deflated_solve(Q, orc, prec):
    V = 4096
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 51, sap_bs=BS, sap_prec=prec, dfl_Ns=8, dfl_bs=BS, dfl_nit=3,
                      precond=Q.PRECOND_DFL, max_nrhs=3)
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    ctx.dfl_build(S.gaussian_field(V, 52, nrhs=8))
    eta = S.gaussian_field(V, 53, nrhs=3)
    psi, info, st = ctx.solve(eta)
    psi = to_np(psi)
    for r in range(3):
        res = np.linalg.norm(eta[r] - orc.apply_D(L, U, A, psi[r])) / np.linalg.norm(eta[r])
        print(prec, r, info[r]["iters"], res)
        assert info[r]["converged"] and res <= 1e-10
    x_o, _ = orc.fgcr(L, U, A, Ai, eta[0], op="D", prec="sap", sap_bs=BS, ncy=5, nmr=4, tol=1e-12)
    assert np.linalg.norm(psi[0] - x_o) / np.linalg.norm(x_o) < 1e-8


@pytest.mark.parametrize("Lw,bs,ns,nrhs", [((8, 8, 8, 8), (4, 4, 4, 4), 24, 8),   # matrix-core products, 6 tiles
                                           ((8, 8, 8, 8), (4, 2, 4, 2), 12, 3),   # one site per parity and row
                                           ((4, 4, 8, 12), (2, 2, 4, 6), 16, 5),  # three sites per parity and row
                                           ((8, 8, 8, 8), (4, 4, 4, 4), 40, 2),   # Gram-Schmidt / VALU fallback
                                           ((8, 8, 8, 8), (4, 4, 2, 1), 8, 2)])   # odd rows: VALU fallback
def test_dfl_wide_bases(Q, orc, Lw, bs, ns, nrhs):
    # basis (block orthonormalisation), little operator (face products), restriction,
    # coarse apply and prolongation at the workload's Ns and rhs counts and at odd row
    # lengths, against the oracle on the same start fields
    V = int(np.prod(Lw))
    sbs = bs if bs[3] % 2 == 0 else (4, 4, 4, 4)
    ctx, U = make_ctx(Q, Lw, 0.6, 0.1357, 1.9, 61, sap_bs=sbs, ncy=2, nmr=4, sap_prec=0, dfl_Ns=ns, dfl_bs=bs,
                      dfl_nit=1, dfl_coarse_tol=1e-12, precond=Q.PRECOND_DFL, max_nrhs=nrhs)
    A, Ai = orc.clover(Lw, U, 0.1357, 1.9)
    init = S.gaussian_field(V, 62, nrhs=ns)
    ctx.dfl_build(init)
    d = orc.Deflation(Lw, bs, ns)
    d.build(U, A, Ai, sbs, 2, 4, 1, init)
    basis, little = ctx.dfl_export()
    basis, little = to_np(basis), to_np(little)
    eb, el = relerr(basis, d.basis()), relerr(little, d.little())
    print(f"{Lw} {bs} Ns {ns}: basis err {eb:.2e} little err {el:.2e}")
    assert eb < 1e-10 and el < 1e-10
    nb = np.array(Lw) // np.array(bs)
    x = np.array(np.unravel_index(np.arange(V), Lw)).T
    bid = np.ravel_multi_index((x // np.array(bs)).T, nb)
    for b in (0, d.nblk - 1):
        Wb = basis[:, bid == b].reshape(ns, -1)
        assert np.abs(Wb.conj() @ Wb.T - np.eye(ns)).max() < 1e-13
    # coarse operator on several right-hand sides (one solve = many applies)
    f = S.gaussian_field(d.nblk * ns * nrhs // 12 + 1, 63).reshape(-1)[: d.nblk * ns * nrhs].reshape(nrhs, d.nblk, ns)
    c_g, _ = ctx.dfl_coarse_solve(f, 1e-13)
    for k in range(nrhs):
        c_o, _ = d.coarse_solve(f[k], 1e-13)
        assert relerr(to_np(c_g)[k], c_o) < 1e-10
    # two-level preconditioner (restriction, coarse solve, prolongation, SAP)
    r = S.gaussian_field(V, 64, nrhs=nrhs)
    out = to_np(ctx.dfl_precond(r))
    for k in (0, nrhs - 1):
        e = relerr(out[k], d.precond(U, A, Ai, sbs, 2, 4, 1e-12, r[k]))
        print("precond err", e)
        assert e < 1e-9
