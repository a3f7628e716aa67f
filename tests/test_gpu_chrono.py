"""Chronological inversion and deflation-subspace refresh on the GPU (Sect. 3:
the solutions of earlier inversions predict the next one; Sect. 4, Fig. 1: the
deflation subspace is updated along the trajectory), against the oracle.

The gauge fields of a trajectory are stood in for by the random-link generator
at slowly growing eps with one seed, U(eps) = V diag(exp(i eps h)) V^dag, which
varies smoothly with eps."""
import numpy as np
import pytest

from paper_1011_0911_amd import synth as S
from tests.gpu_util import relerr, to_np

pytestmark = pytest.mark.gpu
L = (8, 8, 8, 8)
V = 4096
BS = (4, 4, 4, 4)
KAPPA, CSW = 0.1357, 1.9


@pytest.fixture(scope="module")
def Q():
    from paper_1011_0911_amd import qdd

    qdd.lib()
    return qdd


def ctx_of(Q, **cfg):
    return Q.Context(L, Q.default_config(**cfg))


def set_field(ctx, eps, seed=1901):
    import torch

    U = S.random_su3_links(L, eps, seed)
    ctx.set_gauge(torch.from_numpy(U))
    ctx.set_params(KAPPA, CSW)
    return U


def test_warm_start(Q, orc):
    ctx = ctx_of(Q, max_nrhs=2, sap_bs=BS, sap_prec=1, precond=Q.PRECOND_SAP)
    U = set_field(ctx, 0.6)
    A, _ = orc.clover(L, U, KAPPA, CSW)
    eta = S.gaussian_field(V, 1902, nrhs=2)
    x, info, _ = ctx.solve(eta)
    # the solution itself as guess: no iteration
    x2, info2, _ = ctx.solve_guess(eta, x)
    assert [i["iters"] for i in info2] == [0, 0] and all(i["converged"] for i in info2)
    assert np.array_equal(to_np(x2), to_np(x))
    # a perturbed guess converges to the same tolerance in fewer iterations than from 0
    g = to_np(x) + 1e-3 * S.gaussian_field(V, 1903, nrhs=2)
    x3, info3, _ = ctx.solve_guess(eta, g)
    for r in range(2):
        res = np.linalg.norm(eta[r] - orc.apply_D(L, U, A, to_np(x3)[r])) / np.linalg.norm(eta[r])
        assert info3[r]["converged"] and res <= 1e-10 and info3[r]["iters"] < info[r]["iters"]


@pytest.mark.parametrize("deflated", [False, True])
def test_chronological_guess_parity_and_gain(Q, orc, deflated):
    # four solves along the trajectory fill the history of both rhs slots; at the
    # fifth field the GPU guess equals the oracle's least-squares combination of the
    # stored solutions, and the solve from it takes fewer iterations than from 0
    kw = dict(max_nrhs=2, sap_bs=BS, sap_prec=1, precond=Q.PRECOND_SAP, chrono_nv=4)
    if deflated:
        kw.update(precond=Q.PRECOND_DFL, dfl_Ns=8, dfl_bs=BS, dfl_nit=3, dfl_refresh_nit=1)
    ctx = ctx_of(Q, **kw)
    eta = S.gaussian_field(V, 1904, nrhs=2)
    sols = []
    for k in range(4):
        set_field(ctx, 0.6 + 0.01 * k)
        if deflated:
            if k == 0:
                ctx.dfl_build(S.gaussian_field(V, 1905, nrhs=8))
            else:
                ctx.dfl_refresh()
        x, info, _ = ctx.solve(eta)
        sols.append(to_np(x))
        print(f"field {k}: iterations {[i['iters'] for i in info]}", flush=True)
    U = set_field(ctx, 0.64)
    if deflated:
        ctx.dfl_refresh()
    A, _ = orc.clover(L, U, KAPPA, CSW)
    g = to_np(ctx.chrono_guess(eta))
    for r in range(2):
        ref = orc.chrono_guess(L, U, A, np.stack([s[r] for s in sols]), eta[r])
        e = relerr(g[r], ref)
        res_g = np.linalg.norm(eta[r] - orc.apply_D(L, U, A, g[r])) / np.linalg.norm(eta[r])
        print(f"rhs {r}: guess err {e:.2e}, guess residual {res_g:.2e}", flush=True)
        assert e < 1e-9 and res_g < 1e-2
    x, info, _ = ctx.solve(eta)
    ctx.chrono_reset()
    x0, info0, _ = ctx.solve(eta)
    for r in range(2):
        res = np.linalg.norm(eta[r] - orc.apply_D(L, U, A, to_np(x)[r])) / np.linalg.norm(eta[r])
        print(f"rhs {r}: chronological {info[r]['iters']} iterations, from 0 {info0[r]['iters']}", flush=True)
        assert info[r]["converged"] and res <= 1e-10 and info[r]["iters"] < info0[r]["iters"]


def test_deflation_refresh_parity(Q, orc):
    # FP64 SAP on both sides: the refreshed basis and little operator (rounds of SAP
    # inverse iteration from the basis of the previous field) equal the oracle's
    # build at the new field started from its basis of the previous field
    kw = dict(max_nrhs=2, sap_bs=BS, ncy=2, nmr=4, sap_prec=0, dfl_Ns=6, dfl_bs=BS, dfl_nit=2,
              dfl_refresh_nit=2, precond=Q.PRECOND_DFL)
    ctx = ctx_of(Q, **kw)
    U0 = set_field(ctx, 0.6)
    init = S.gaussian_field(V, 1906, nrhs=6)
    ctx.dfl_build(init)
    A0, Ai0 = orc.clover(L, U0, KAPPA, CSW)
    d0 = orc.Deflation(L, BS, 6)
    d0.build(U0, A0, Ai0, BS, 2, 4, 2, init)
    U1 = set_field(ctx, 0.62)
    with pytest.raises(Q.QddError):  # the subspace of the old field is no longer in effect
        ctx.solve(S.gaussian_field(V, 1907)[None])
    ctx.dfl_refresh()
    A1, Ai1 = orc.clover(L, U1, KAPPA, CSW)
    d1 = orc.Deflation(L, BS, 6)
    d1.build(U1, A1, Ai1, BS, 2, 4, 2, d0.basis())
    basis, little = ctx.dfl_export()
    eb, el = relerr(to_np(basis), d1.basis()), relerr(to_np(little), d1.little())
    print(f"refresh: basis err {eb:.2e} little err {el:.2e}")
    assert eb < 1e-10 and el < 1e-10
    assert ctx.dfl_stats() == (1, 1)


def test_automatic_refresh(Q, orc):
    # a deflated solve above dfl_refresh_iters outer iterations refreshes the
    # subspace afterwards; the next solve is deflated by the refreshed subspace
    kw = dict(max_nrhs=1, sap_bs=BS, sap_prec=1, dfl_Ns=8, dfl_bs=BS, dfl_nit=3, dfl_refresh_nit=2,
              dfl_refresh_iters=1, precond=Q.PRECOND_DFL)
    ctx = ctx_of(Q, **kw)
    set_field(ctx, 0.6)
    ctx.dfl_build(S.gaussian_field(V, 1908, nrhs=8))
    eta = S.gaussian_field(V, 1909)[None]
    _, info, _ = ctx.solve(eta)
    assert info[0]["iters"] > 1 and ctx.dfl_stats() == (1, 1)
    U = set_field(ctx, 0.61)
    ctx.dfl_refresh()
    A, _ = orc.clover(L, U, KAPPA, CSW)
    x, info, _ = ctx.solve(eta)
    res = np.linalg.norm(eta[0] - orc.apply_D(L, U, A, to_np(x)[0])) / np.linalg.norm(eta[0])
    assert info[0]["converged"] and res <= 1e-10 and ctx.dfl_stats() == (1, 3)
