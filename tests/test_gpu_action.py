"""GPU parity of the mass-preconditioning calls (Eqs. 2-5) against the oracle:
the clover log determinants (log det Q_ee, log det Q_oo) and W(dm) = Q_S + dm."""
import ctypes

import numpy as np
import pytest

from paper_1011_0911_amd import synth as S
from tests.gpu_util import make_ctx, relerr, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    from paper_1011_0911_amd import qdd

    qdd.lib()
    return qdd


# 4^3x8: one partial sum per parity; 24^3x48 (the learned-stage lattice):
# 512 workgroups per parity, each looping over several site tiles with a ragged end
@pytest.mark.parametrize("L,seed", [((4, 4, 4, 8), 701), ((48, 24, 24, 24), 702)])
def test_clover_logdet_parity(Q, orc, L, seed):
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, seed)
    le, lo = ctx.clover_logdet()
    re, ro = orc.clover_logdet(L, U, 0.1357, 1.9)
    print("logdet", le, re, lo, ro)
    # every site adds about 12 log(1/(2 kappa)) ~ 16; the sums are formed in a
    # different order on each side: a few units of rounding of the total
    assert abs(le - re) < 1e-12 * abs(re) and abs(lo - ro) < 1e-12 * abs(ro)
    assert (le, lo) == ctx.clover_logdet()  # fixed summation order: bit-identical on repeat


def test_clover_logdet_closed_form(Q):
    L = (8, 4, 4, 4)
    ctx, _ = make_ctx(Q, L, 0.6, 0.125, 0.0, 703)
    le, lo = ctx.clover_logdet()
    ref = int(np.prod(L)) // 2 * 12 * np.log(4.0)  # A = 1/(2 kappa) = 4 on every component
    assert abs(le - ref) < 1e-13 * ref and abs(lo - ref) < 1e-13 * ref


@pytest.mark.parametrize("nrhs", [1, 3])
def test_apply_w_parity(Q, orc, nrhs):
    # nrhs 1: blocked even field; 3: the interleaved batch layout
    L = (8, 4, 4, 4)
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 704, max_nrhs=4)
    A, _ = orc.clover(L, U, 0.1357, 1.9)
    pe = S.gaussian_field(V // 2, 705, nrhs=nrhs)
    for dm in (0.0, 0.25):
        out = to_np(ctx.apply_w(dm, pe))
        ref = orc.apply_W(L, U, A, dm, pe)
        e = relerr(out, ref)
        print("W nrhs", nrhs, "dm", dm, "err", e)
        assert e < 1e-12


def test_apply_w_rejects_aliasing_and_bad_shift(Q):
    L = (8, 4, 4, 4)
    ctx, _ = make_ctx(Q, L, 0.6, 0.1357, 1.9, 706)
    f = ctx.pack(0, S.gaussian_field(int(np.prod(L)) // 2, 707)[None], True)
    g = ctx.empty_field(0, 1, True)
    lib = Q.lib()
    assert lib.qdd_apply_w(ctx.h, 1, 0.1, Q._ptr(f), Q._ptr(f)) == Q.QDD_EINVAL
    assert lib.qdd_apply_w(ctx.h, 1, float("nan"), Q._ptr(f), Q._ptr(g)) == Q.QDD_EINVAL
    assert lib.qdd_apply_w(ctx.h, 1, 0.1, Q._ptr(f), Q._ptr(g)) == Q.QDD_OK


@pytest.mark.parametrize("deflated", [False, True])
def test_solve_qs_eq5(Q, orc, deflated):
    # Q_S^{-1} phi through Eq. 5 with the configured solver, checked by the
    # residual of the oracle's Q_S (the paper's form from the blocks of Q).  The
    # D solve stops at relative residual 1e-10; on the even sites that becomes a
    # Q_S residual of at most about cond(A) (1 + |D_eo A_o^{-1}|) 1e-10 ~ 1e-9
    L, BS = (8, 8, 8, 8), (4, 4, 4, 4)
    V = int(np.prod(L))
    kw = dict(max_nrhs=2)
    if deflated:
        kw.update(sap_bs=BS, sap_prec=1, dfl_Ns=8, dfl_bs=BS, dfl_nit=3, precond=Q.PRECOND_DFL)
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 708, **kw)
    A, _ = orc.clover(L, U, 0.1357, 1.9)
    if deflated:
        ctx.dfl_build(S.gaussian_field(V, 709, nrhs=8))
    phi = S.gaussian_field(V // 2, 710, nrhs=2)
    x, info, st = ctx.solve_qs(phi)
    x = to_np(x)
    for r in range(2):
        res = np.linalg.norm(orc.apply_W(L, U, A, 0.0, x[r]) - phi[r]) / np.linalg.norm(phi[r])
        print("deflated", deflated, "rhs", r, "iters", info[r]["iters"], "Q_S residual", res)
        assert info[r]["converged"] and res < 1e-8
