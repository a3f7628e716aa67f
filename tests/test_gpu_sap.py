"""GPU parity of the Schwarz alternating procedure (two-colour SAP with
minimal-residual block solves) and of SAP-preconditioned flexible GCR against
the CPU oracle.

The GPU keeps the residual up to date incrementally (the block residual is the
MR residual on even sites and zero on odd sites; the faces are corrected from
the neighbours' last corrections) where the oracle recomputes eta - D psi after
every half-sweep: the same numbers in exact arithmetic.  Tolerances (max-abs
error / max-abs reference): FP64 1e-12, FP32 1e-5, FP16 storage 3e-3: six
quantities are stored in FP16 (the source, the links, the two clover blocks A_e
and A_o^{-1}, the residual rho and the block corrections V), each rounded with
unit 2^-11 = 4.9e-4 relative to its site maximum, so a half-sweep's result is
off by at most about 6 x 4.9e-4; the procedure contracts the error of earlier
half-sweeps, so the bound does not grow with the number of cycles (observed
3.6e-4 .. 6.0e-4 for 1 to 5 cycles)."""
import numpy as np
import pytest

from paper_1011_0911_amd import synth as S
from tests.gpu_util import make_ctx, relerr, to_np

pytestmark = pytest.mark.gpu
TOL = {0: 1e-12, 1: 1e-5, 2: 3e-3}


@pytest.fixture(scope="module")
def Q():
    from paper_1011_0911_amd import qdd

    qdd.lib()
    return qdd


# every kernel variant of each storage precision (FP64 has one): 1 per site with
# links in registers, 2 per (block, rhs), 3 (links, for FP16 also the clover,
# staged in LDS, 4 rhs per workgroup) and for FP16 4 (links staged, 2 rhs per
# workgroup); 5 rhs so that the staged variants also run a partly filled group
VARIANTS = [(0, 0), (1, 1), (1, 2), (1, 3), (2, 1), (2, 2), (2, 3), (2, 4)]


@pytest.mark.parametrize("L,bs,ncy,nmr", [((8, 8, 8, 8), (4, 4, 4, 4), 5, 4), ((8, 4, 4, 8), (2, 2, 2, 2), 3, 2),
                                          ((4, 8, 4, 4), (2, 4, 2, 2), 1, 1)])
@pytest.mark.parametrize("prec,variant", VARIANTS)
def test_sap_parity(Q, orc, L, bs, ncy, nmr, prec, variant):
    V = int(np.prod(L))
    nr = 5
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 500 + V, sap_bs=bs, ncy=ncy, nmr=nmr, sap_prec=prec, max_nrhs=nr)
    if variant:
        ctx.set_launch(Q.KERNEL_SAP, prec, 0, variant, 0, 0)
    assert ctx.get_launch(Q.KERNEL_SAP, prec)[1] == variant
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    eta = S.gaussian_field(V, 501, nrhs=nr)
    out = to_np(ctx.sap(eta))
    for r in (0, 1, nr - 1):
        ref = orc.sap(L, U, A, Ai, eta[r], bs, ncy, nmr)
        e = relerr(out[r], ref)
        print(f"SAP L={L} bs={bs} prec={prec} variant={variant} rhs={r} err={e:.2e}")
        assert e < TOL[prec], e


def test_sap_variants_rejected_where_missing(Q):
    ctx, _ = make_ctx(Q, (4, 4, 4, 4), 0.6, 0.1357, 1.9, 509, sap_bs=(2, 2, 2, 2), sap_prec=1)
    for prec, v in ((1, 4), (0, 1), (2, 5), (1, 0)):
        with pytest.raises(Q.QddError):
            ctx.set_launch(Q.KERNEL_SAP, prec, 0, v, 0, 0)
    with pytest.raises(Q.QddError):
        ctx.set_launch(Q.KERNEL_SAP, 1, 64, 1, 0, 0)


def test_sap_autotune_picks_a_variant(Q, orc):
    L, bs = (8, 8, 8, 8), (4, 4, 4, 4)
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 506, sap_bs=bs, sap_prec=2, precond=Q.PRECOND_SAP, max_nrhs=4)
    ms = ctx.tune_sap(4)
    v = ctx.get_launch(Q.KERNEL_SAP, 2)[1]
    print("tuned Schwarz variant", v, "ms", ms)
    assert v in (1, 2, 3, 4) and ms > 0
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    eta = S.gaussian_field(4096, 507, nrhs=4)
    out = to_np(ctx.sap(eta))
    assert relerr(out[3], orc.sap(L, U, A, Ai, eta[3], bs, 5, 4)) < TOL[2]


def test_sap_is_deterministic(Q):
    L, bs = (8, 8, 8, 8), (4, 4, 4, 4)
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 502, sap_bs=bs, sap_prec=1)
    eta = S.gaussian_field(4096, 503)
    a = to_np(ctx.sap(eta[None]))
    b = to_np(ctx.sap(eta[None]))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_sap_fgcr_solve(Q, orc, prec):
    L, bs = (8, 8, 8, 8), (4, 4, 4, 4)
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 504, sap_bs=bs, sap_prec=prec, precond=Q.PRECOND_SAP, max_nrhs=2)
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    eta = S.gaussian_field(4096, 505, nrhs=2)
    psi, info, st = ctx.solve(eta)
    psi = to_np(psi)
    x_o, info_o = orc.fgcr(L, U, A, Ai, eta[0], op="D", prec="sap", sap_bs=bs, ncy=5, nmr=4, tol=1e-10)
    print("gpu", info[0], "oracle", info_o["iters"])
    for r in range(2):
        res = np.linalg.norm(eta[r] - orc.apply_D(L, U, A, psi[r])) / np.linalg.norm(eta[r])
        assert info[r]["converged"] and res <= 1e-10
    if prec == 0:
        assert abs(info[0]["iters"] - info_o["iters"]) <= 1
    else:
        assert info[0]["iters"] <= info_o["iters"] + 3
    # both solutions agree within the conditioning of the residual tolerance
    assert np.linalg.norm(psi[0] - x_o) / np.linalg.norm(x_o) < 1e-8
