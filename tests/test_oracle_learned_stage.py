"""Pins of the oracle's learned preconditioner stage inside the two-level
deflated preconditioner, v = C r + N(r1) + M_sap(r2) with r1 = r - D C r and
r2 = r1 - D N(r1) (N dropped when |r2| > |r1|).  The solver context is the
locally deflated Schwarz-preconditioned GCR of Sect. 3-4 (Table 1); the stage
itself is this library's extension.

* zero weights give N = 0, so the flexible GCR iterates are those of the plain
  deflated solver, bit for bit;
* with an accepted, non-zero N the output equals the composition rebuilt from a
  dense little operator W^dag D W (dense LU instead of the coarse GCR), the
  network applied to r1 and the Schwarz procedure applied to r2 -- feeding r1 to
  the Schwarz procedure, or dropping a term, fails it;
* a rejected N gives exactly the plain two-level preconditioner."""
import numpy as np
import pytest

from paper_1011_0911_amd import synth as S

L = (4, 4, 4, 4)
V = 256
SAP_BS = (2, 2, 2, 2)
DFL_BS = (2, 2, 2, 2)
NS = 4
KAPPA, CSW = 0.1355, 1.9
CH = [1, 2, 1]


def stage_weights(orc, seed, scale):
    """[1, 2, 1] network: an identity path of strength 0.5*0.25 + 0.25*0.25 = 0.1875
    on d = 0 plus Gaussian perturbations of std `scale` on every weight."""
    W = S.random_weights(orc.net_nweights(CH), seed, scale)
    w1 = W[: 9 * 2 * 1 * 16].reshape(9, 2, 1, 4, 4)
    w2 = W[9 * 2 * 1 * 16:].reshape(9, 1, 2, 4, 4)
    w1[0, 0, 0] += 0.5 * np.eye(4)
    w1[0, 1, 0] += 0.25 * np.eye(4)
    w2[0, 0, 0] += 0.25 * np.eye(4)
    w2[0, 0, 1] += 0.25 * np.eye(4)
    return np.concatenate([w1.reshape(-1), w2.reshape(-1)])


@pytest.fixture(scope="module")
def setup(orc):
    U = S.random_su3_links(L, 0.5, 901)
    A, Ai = orc.clover(L, U, KAPPA, CSW)
    d = orc.Deflation(L, DFL_BS, NS)
    d.build(U, A, Ai, SAP_BS, 2, 4, 2, S.gaussian_field(V, 902, nrhs=NS))
    return U, A, Ai, d


def block_ids():
    x = np.array(np.unravel_index(np.arange(V), L)).T
    return np.ravel_multi_index((x // np.array(DFL_BS)).T, tuple(np.array(L) // np.array(DFL_BS)))


def dense_coarse(orc, U, A, d, r):
    """C r = W (W^dag D W)^{-1} W^dag r with the block-restricted basis written
    out as a dense (12 V) x (nblk Ns) matrix and the little system solved by LU."""
    basis = d.basis().reshape(NS, V, 12)
    bid = block_ids()
    nblk = int(bid.max()) + 1
    Wm = np.zeros((V, 12, nblk, NS), complex)
    for b in range(nblk):
        for k in range(NS):
            Wm[bid == b, :, b, k] = basis[k, bid == b]
    Wm = Wm.reshape(V * 12, nblk * NS)
    DW = np.stack([orc.apply_D(L, U, A, Wm[:, j].reshape(V, 4, 3)).reshape(-1) for j in range(nblk * NS)], 1)
    Ac = Wm.conj().T @ DW
    return (Wm @ np.linalg.solve(Ac, Wm.conj().T @ r.reshape(-1))).reshape(V, 4, 3)


def test_zero_weights_give_the_plain_iterates(orc, setup):
    U, A, Ai, d = setup
    eta = S.gaussian_field(V, 903)
    W0 = np.zeros(orc.net_nweights(CH), complex)
    kw = dict(op="D", sap_bs=SAP_BS, ncy=2, nmr=4, dfl=d, coarse_tol=1e-8, nhist=40)
    x_net, i_net = orc.fgcr(L, U, A, Ai, eta, prec="net", net=(CH, W0), **kw)
    x_dfl, i_dfl = orc.fgcr(L, U, A, Ai, eta, prec="dfl", **kw)
    assert i_net["converged"] and i_net["fallbacks"] == 0
    assert i_net["iters"] == i_dfl["iters"]
    assert np.array_equal(i_net["history"], i_dfl["history"])
    assert np.array_equal(x_net, x_dfl)


def test_accepted_stage_equals_dense_composition(orc, setup):
    U, A, Ai, d = setup
    W = stage_weights(orc, 904, 0.02)
    r = S.gaussian_field(V, 905)
    out, fb = d.net_precond(U, A, Ai, SAP_BS, 2, 4, 1e-14, CH, W, r)
    Cr = dense_coarse(orc, U, A, d, r)
    r1 = r - orc.apply_D(L, U, A, Cr)
    vn = orc.net_forward(L, U, CH, W, r1[None])[0]
    r2 = r1 - orc.apply_D(L, U, A, vn)
    assert not fb and np.linalg.norm(r2) < 0.9 * np.linalg.norm(r1)  # accepted, and N does work
    ref = Cr + vn + orc.sap(L, U, A, Ai, r2, SAP_BS, 2, 4)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    assert err < 1e-10, err
    # the pin is sensitive to the placement: Schwarz on r1, or a dropped term, is far off
    for wrong in (Cr + vn + orc.sap(L, U, A, Ai, r1, SAP_BS, 2, 4), Cr + orc.sap(L, U, A, Ai, r2, SAP_BS, 2, 4),
                  vn + orc.sap(L, U, A, Ai, r2, SAP_BS, 2, 4)):
        assert np.abs(out - wrong).max() / np.abs(ref).max() > 1e-3


def test_rejected_stage_is_the_plain_preconditioner(orc, setup):
    U, A, Ai, d = setup
    W = S.random_weights(orc.net_nweights(CH), 906, 3.0)  # large random weights raise the residual
    r = S.gaussian_field(V, 907)
    out, fb = d.net_precond(U, A, Ai, SAP_BS, 2, 4, 1e-10, CH, W, r)
    assert fb
    assert np.array_equal(out, d.precond(U, A, Ai, SAP_BS, 2, 4, 1e-10, r))
