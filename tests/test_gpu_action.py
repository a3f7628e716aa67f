"""GPU parity of the mass-preconditioning calls (Eqs. 2-5) against the oracle:
the clover log determinants (log det Q_ee, log det Q_oo), W(dm) = Q_S + dm, the
solves Q_S^{-1} (Eq. 5) and W(dm)^{-1}, and the effective action of Eq. 4."""
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


def _solver_ctx(Q, orc, L, deflated, seed, nrhs=2):
    BS = (4, 4, 4, 4)
    V = int(np.prod(L))
    kw = dict(max_nrhs=nrhs)
    if deflated:
        kw.update(sap_bs=BS, sap_prec=1, dfl_Ns=8, dfl_bs=BS, dfl_nit=3, precond=Q.PRECOND_DFL)
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, seed, **kw)
    A, _ = orc.clover(L, U, 0.1357, 1.9)
    if deflated:
        ctx.dfl_build(S.gaussian_field(V, seed + 1, nrhs=8))
    return ctx, U, A


@pytest.mark.parametrize("deflated", [False, True])
def test_solve_qs_eq5(Q, orc, deflated):
    # Q_S^{-1} phi through Eq. 5 with the configured solver; the call checks and
    # reports the residual of Q_S itself and refines until it is <= 1e-10, which
    # the oracle's Q_S (the paper's form from the blocks of Q) confirms
    L = (8, 8, 8, 8)
    V = int(np.prod(L))
    ctx, U, A = _solver_ctx(Q, orc, L, deflated, 708)
    phi = S.gaussian_field(V // 2, 710, nrhs=2)
    x, info, st = ctx.solve_qs(phi)
    x = to_np(x)
    for r in range(2):
        res = np.linalg.norm(orc.apply_W(L, U, A, 0.0, x[r]) - phi[r]) / np.linalg.norm(phi[r])
        print("deflated", deflated, "rhs", r, "iters", info[r]["iters"], "Q_S residual", res, info[r]["true_res"])
        assert info[r]["converged"] and res <= 1.001e-10
        assert abs(res - info[r]["true_res"]) < 1e-3 * res + 1e-15


@pytest.mark.parametrize("deflated", [False, True])
@pytest.mark.parametrize("dm", [0.09, 0.5])
def test_solve_w_parity(Q, orc, deflated, dm):
    # W(dm)^{-1} phi through D' = D with the even clover blocks scaled by 1 + dm:
    # the W residual under the oracle's W <= 1e-10, and the distance to the
    # oracle's solution (GMRES to 1e-12 on its W) within cond(W) (1e-10 + 1e-12)
    L = (8, 8, 8, 8)
    V = int(np.prod(L))
    ctx, U, A = _solver_ctx(Q, orc, L, deflated, 711)
    phi = S.gaussian_field(V // 2, 712, nrhs=2)
    x, info, st = ctx.solve_w(dm, phi)
    x = to_np(x)
    ref = orc.solve_W(L, U, A, dm, phi[0])
    for r in range(2):
        res = np.linalg.norm(orc.apply_W(L, U, A, dm, x[r]) - phi[r]) / np.linalg.norm(phi[r])
        print("deflated", deflated, "dm", dm, "rhs", r, "iters", info[r]["iters"], "W residual", res)
        assert info[r]["converged"] and res <= 1.001e-10
    d = np.linalg.norm(x[0] - ref) / np.linalg.norm(ref)
    print("distance to the oracle solution", d)
    assert d < 1e-8


def test_solve_w_zero_shift_is_qs(Q, orc):
    L = (8, 4, 4, 8)
    ctx, U, A = _solver_ctx(Q, orc, L, False, 713, nrhs=1)
    phi = S.gaussian_field(int(np.prod(L)) // 2, 714)
    x0, _, _ = ctx.solve_qs(phi[None])
    x1, _, _ = ctx.solve_w(0.0, phi[None])
    assert np.array_equal(to_np(x0), to_np(x1))
    with pytest.raises(Q.QddError):
        ctx.solve_w(-0.1, phi[None])


@pytest.mark.parametrize("L,deflated", [((4, 4, 4, 8), False), ((8, 8, 8, 8), True)])
def test_action_parity(Q, orc, L, deflated):
    # S_eff of Eq. 4 against the oracle's (log determinants summed per site,
    # solves by GMRES on its W): the log-det term to 1e-12, the pseudofermion
    # terms within the solver tolerance (relative error of |chi|^2 about 2 cond 1e-10)
    V = int(np.prod(L))
    ctx, U, A = _solver_ctx(Q, orc, L, deflated, 715)
    phi = S.gaussian_field(V // 2, 716, nrhs=2)
    dm = 0.09
    s, parts, c1, c2, infos = ctx.action(dm, phi[0], phi[1])
    so, po = orc.s_eff(L, U, 0.1357, 1.9, dm, phi[0], phi[1])
    print("S_eff", s, so, "parts", parts, po, "iters", [i["iters"] for i in infos])
    assert abs(parts[0] - po[0]) < 1e-12 * abs(po[0])
    assert abs(parts[1] - po[1]) < 1e-8 * po[1] and abs(parts[2] - po[2]) < 1e-8 * po[2]
    assert abs(s - so) < 1e-8 * (abs(po[0]) + po[1] + po[2])
    # the returned solutions are those of the terms
    assert np.linalg.norm(orc.apply_W(L, U, A, dm, to_np(c1)) - phi[0]) <= 1.001e-10 * np.linalg.norm(phi[0])
    assert np.linalg.norm(orc.apply_W(L, U, A, 0.0, to_np(c2)) - phi[1]) <= 1.001e-10 * np.linalg.norm(phi[1])
