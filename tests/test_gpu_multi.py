"""Several systems at once: deflation subspace shared across masses (little
operator shifted on the block diagonal) and concurrent multi-system solves."""
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


def test_dfl_share_equals_little_operator_at_new_mass(Q):
    # sharing from kappa_1 to kappa_2 must give W^dag D(kappa_2) W for the same W:
    # compare with a build at kappa_2 that starts from the shared basis itself
    L, BS = (8, 8, 8, 8), (4, 4, 4, 4)
    kw = dict(sap_bs=BS, dfl_Ns=6, dfl_bs=BS, dfl_nit=2, sap_prec=0, precond=Q.PRECOND_DFL)
    a, U = make_ctx(Q, L, 0.6, 0.1355, 1.9, 701, **kw)
    a.dfl_build(S.gaussian_field(4096, 702, nrhs=6))
    b, _ = make_ctx(Q, L, 0.6, 0.1357, 1.9, 701, **kw)
    b.dfl_share(a)
    Wa, Aa = a.dfl_export()
    Wb, Ab = b.dfl_export()
    assert np.array_equal(to_np(Wa), to_np(Wb))
    # rebuild at kappa_2 with nit = 0 from the (already block-orthonormal) basis
    c, _ = make_ctx(Q, L, 0.6, 0.1357, 1.9, 701, **dict(kw, dfl_nit=0))
    c.dfl_build(to_np(Wa))
    Wc, Ac = c.dfl_export()
    assert relerr(to_np(Ab), to_np(Ac)) < 1e-12


def _system(Q, L, kappa, seed, nrhs, **cfg):
    import torch

    V = int(np.prod(L))
    U = S.random_su3_links(L, 0.6, seed)
    c = Q.Context(L, Q.default_config(max_nrhs=nrhs, **cfg), stream=torch.cuda.Stream())
    c.set_gauge(torch.from_numpy(U))
    c.set_params(kappa, 1.9)
    return c, U


@pytest.mark.parametrize("kind", ["sap", "dfl"])
def test_solve_multi_matches_single_solves(Q, orc, kind):
    # several systems (lattice sizes, masses and batch sizes differ) solved
    # concurrently give bit for bit the solutions and iteration counts of the same
    # systems solved one at a time, and every solution has true residual <= 1e-10
    import torch

    if kind == "sap":
        systems = [((8, 8, 8, 8), 0.1350, (4, 4, 4, 4)), ((8, 8, 8, 8), 0.1357, (4, 4, 4, 4)),
                   ((8, 4, 4, 8), 0.1355, (4, 2, 2, 4))]
    else:
        systems = [((8, 8, 8, 8), 0.1357, (4, 4, 4, 4)), ((16, 8, 8, 8), 0.1355, (4, 4, 4, 4)),
                   ((8, 8, 8, 8), 0.1350, (4, 4, 4, 4))]
    ctxs, etas, refs = [], [], []
    for k, (L, kappa, bs) in enumerate(systems):
        V = int(np.prod(L))
        cfg = dict(sap_bs=bs, sap_prec=1, precond=Q.PRECOND_SAP)
        if kind == "dfl":
            cfg.update(precond=Q.PRECOND_DFL, dfl_Ns=4, dfl_bs=bs, dfl_nit=2)
        c, U = _system(Q, L, kappa, 710 + k, 2, **cfg)
        if kind == "dfl":
            c.dfl_build(S.gaussian_field(V, 730 + k, nrhs=4))
        ctxs.append(c)
        etas.append(S.gaussian_field(V, 720 + k, nrhs=1 + k % 2))
        A, _ = orc.clover(L, U, kappa, 1.9)
        refs.append((L, U, A))
    psis, infos, st = Q.solve_multi(ctxs, etas)
    assert st == 0
    torch.cuda.synchronize()
    for c, eta, psi, inf, (L, U, A) in zip(ctxs, etas, psis, infos, refs):
        single, sinf, sst = c.solve(eta)
        torch.cuda.synchronize()
        assert sst == 0
        assert torch.equal(psi, single)
        assert [i["iters"] for i in inf] == [i["iters"] for i in sinf]
        psi = to_np(psi)
        for r in range(eta.shape[0]):
            res = np.linalg.norm(eta[r] - orc.apply_D(L, U, A, psi[r])) / np.linalg.norm(eta[r])
            assert inf[r]["converged"] and res <= 1e-10


@pytest.mark.parametrize("kind", ["sap1", "sap2", "sap3", "f16v3", "f16v4", "none"])
def test_solve_group_matches_single_solves(Q, orc, kind):
    # one launch per stage over all systems (lattice sizes, masses, batch sizes and
    # Schwarz block shapes of one volume differ, every FP32 Schwarz variant; one system needs far fewer
    # iterations and leaves the lockstep cycles early): every system gets bit for
    # bit the solution and iteration counts of its own solve, true residual <= 1e-10
    import torch

    systems = [((8, 8, 8, 8), 0.1357, (4, 4, 4, 4), 3), ((16, 8, 8, 8), 0.1355, (4, 4, 4, 4), 1),
               ((8, 4, 8, 16), 0.1350, (4, 2, 4, 8), 2), ((8, 8, 8, 8), 0.1200, (4, 4, 4, 4), 2)]
    ctxs, etas, refs = [], [], []
    for k, (L, kappa, bs, nr) in enumerate(systems):
        V = int(np.prod(L))
        cfg = dict(sap_bs=bs, sap_prec=2 if kind.startswith("f16") else 1, precond=Q.PRECOND_SAP, nkv=6, nmx=400)
        if kind == "none":
            cfg.update(precond=Q.PRECOND_NONE, nkv=12, nmx=2000)
        c, U = _system(Q, L, kappa, 740 + k, nr, **cfg)
        if kind in ("sap2", "sap3"):
            c.set_launch(Q.KERNEL_SAP, Q.F32, 0, int(kind[-1]), 0, 0)
        if kind == "f16v4":
            c.set_launch(Q.KERNEL_SAP, Q.F16, 0, 4, 0, 0)
        ctxs.append(c)
        etas.append(S.gaussian_field(V, 750 + k, nrhs=nr))
        A, _ = orc.clover(L, U, kappa, 1.9)
        refs.append((L, U, A))
    print(f"group solve {kind}: {[s[0] for s in systems]}", flush=True)
    psis, infos, st = Q.solve_group(ctxs, etas)
    assert st == 0
    torch.cuda.synchronize()
    for c, eta, psi, inf, (L, U, A) in zip(ctxs, etas, psis, infos, refs):
        single, sinf, sst = c.solve(eta)
        torch.cuda.synchronize()
        assert sst == 0
        assert [i["iters"] for i in inf] == [i["iters"] for i in sinf]
        assert torch.equal(psi, single)
        psi = to_np(psi)
        for r in range(eta.shape[0]):
            res = np.linalg.norm(eta[r] - orc.apply_D(L, U, A, psi[r])) / np.linalg.norm(eta[r])
            assert inf[r]["converged"] and res <= 1e-10 and abs(inf[r]["true_res"] - res) < 1e-11


def test_solve_group_twice_and_rejections(Q):
    # a second grouped call on the same contexts (state left by the first) gives the
    # same result; systems that cannot be grouped are refused with a reason
    import torch

    a, _ = _system(Q, (8, 8, 8, 8), 0.1357, 761, 2, sap_bs=(4, 4, 4, 4), sap_prec=1, precond=Q.PRECOND_SAP)
    b, _ = _system(Q, (8, 4, 8, 16), 0.1350, 762, 2, sap_bs=(4, 2, 4, 8), sap_prec=1, precond=Q.PRECOND_SAP)
    ea, eb = S.gaussian_field(4096, 763, nrhs=2), S.gaussian_field(4096, 764, nrhs=1)
    p1, i1, s1 = Q.solve_group([a, b], [ea, eb])
    p2, i2, s2 = Q.solve_group([a, b], [ea, eb])
    torch.cuda.synchronize()
    assert s1 == 0 and s2 == 0
    assert all(torch.equal(x, y) for x, y in zip(p1, p2))
    c, _ = _system(Q, (8, 8, 8, 8), 0.1357, 765, 2, sap_bs=(4, 4, 4, 4), sap_prec=2, precond=Q.PRECOND_SAP)
    _, _, st = Q.solve_group([a, c], [ea, ea])
    assert st == Q.QDD_EINVAL and "precisions differ" in Q.lib().qdd_last_error(a.h).decode()
    f, _ = _system(Q, (8, 8, 8, 8), 0.1357, 767, 2, sap_bs=(4, 4, 4, 4), sap_prec=0, precond=Q.PRECOND_SAP)
    _, _, st = Q.solve_group([f, a], [ea, ea])
    assert st == Q.QDD_EINVAL and "FP32 or FP16" in Q.lib().qdd_last_error(f.h).decode()
    d, _ = _system(Q, (8, 8, 8, 8), 0.1357, 766, 2, sap_bs=(4, 4, 4, 4), precond=Q.PRECOND_NONE)
    _, _, st = Q.solve_group([a, d], [ea, ea])
    assert st == Q.QDD_EINVAL and "preconditioner" in Q.lib().qdd_last_error(a.h).decode()
    _, _, st = Q.solve_group([a, a], [ea, ea])
    assert st == Q.QDD_EINVAL and "twice" in Q.lib().qdd_last_error(a.h).decode()


def test_solve_group_restarts_and_iteration_cap(Q):
    # systems with different restart lengths (restart cycles end at different
    # steps) and an iteration cap reached in the middle of a cycle: every system
    # still gets bit for bit its own solve's iterate, iteration count and status
    import torch

    L, bs = (8, 8, 8, 8), (4, 4, 4, 4)
    specs = [(0.1357, dict(nkv=2, nmx=400)), (0.1355, dict(nkv=5, nmx=400)), (0.1350, dict(nkv=6, nmx=3))]
    ctxs, etas = [], []
    for k, (kappa, extra) in enumerate(specs):
        c, _ = _system(Q, L, kappa, 770 + k, 2, sap_bs=bs, sap_prec=1, precond=Q.PRECOND_SAP, ncy=1, nmr=1, **extra)
        ctxs.append(c)
        etas.append(S.gaussian_field(4096, 780 + k, nrhs=2))
    psis, infos, st = Q.solve_group(ctxs, etas)
    torch.cuda.synchronize()
    assert st == Q.QDD_ENOCONV  # the capped system does not converge
    for k, (c, eta, psi, inf) in enumerate(zip(ctxs, etas, psis, infos)):
        single, sinf, sst = c.solve(eta, check=False)
        torch.cuda.synchronize()
        print(f"system {k}: group iters {[i['iters'] for i in inf]} restarts {[i['restarts'] for i in inf]}, "
              f"single {[i['iters'] for i in sinf]}")
        assert torch.equal(psi, single)
        for a, b in zip(inf, sinf):
            assert (a["iters"], a["restarts"], a["converged"]) == (b["iters"], b["restarts"], b["converged"])
            assert a["true_res"] == b["true_res"]
        if k < 2:
            assert sst == 0 and all(i["converged"] for i in inf)
            assert k == 1 or max(i["restarts"] for i in inf) > 0  # nkv 2: restarts for sure
        else:
            assert sst == Q.QDD_ENOCONV and all(i["iters"] == 3 and not i["converged"] for i in inf)
