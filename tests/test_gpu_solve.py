"""GPU solves against the oracle: unpreconditioned FP64 flexible GCR on Dhat
(the plain-method workload, 4^4) and on the full D."""
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


def dense(apply, n_in, shape_in):
    cols = []
    for k in range(n_in):
        e = np.zeros(n_in, complex)
        e[k] = 1
        cols.append(apply(e.reshape(shape_in)).reshape(-1))
    return np.array(cols).T


def test_plain_fgcr_on_dhat_config1(Q, orc):
    L = (4, 4, 4, 4)
    ctx, U = make_ctx(Q, L, 0.3, 0.13, 1.9, S.gauge_seed(1))
    A, Ai = orc.clover(L, U, 0.13, 1.9)
    eta = S.gaussian_field(256, S.source_seed(1))[S.even_sites(L)]
    psi, info, st = ctx.solve_dhat(eta[None])
    psi = to_np(psi)[0]
    r = eta - orc.apply_Dhat(L, U, A, Ai, psi)
    res = np.linalg.norm(r) / np.linalg.norm(eta)
    print("gpu", info[0], "true res (oracle D)", res)
    assert info[0]["converged"] and res <= 1e-10
    x_o, info_o = orc.fgcr(L, U, A, Ai, eta, op="Dhat", tol=1e-10)
    assert abs(info[0]["iters"] - info_o["iters"]) <= 1
    Dh = dense(lambda f: orc.apply_Dhat(L, U, A, Ai, f), 128 * 12, (128, 4, 3))
    xd = np.linalg.solve(Dh, eta.reshape(-1)).reshape(eta.shape)
    cond = np.linalg.cond(Dh)
    assert np.linalg.norm(psi - xd) / np.linalg.norm(xd) < 2 * cond * 1e-10


def test_plain_fgcr_full_D_batched(Q, orc):
    L = (4, 4, 4, 8)
    V = 512
    ctx, U = make_ctx(Q, L, 0.5, 0.1355, 1.9, 401, max_nrhs=3)
    A, Ai = orc.clover(L, U, 0.1355, 1.9)
    eta = S.gaussian_field(V, 402, nrhs=3)
    eta[1] *= 1e-3  # different scales converge independently
    psi, info, st = ctx.solve(eta)
    psi = to_np(psi)
    for r in range(3):
        res = np.linalg.norm(eta[r] - orc.apply_D(L, U, A, psi[r])) / np.linalg.norm(eta[r])
        assert info[r]["converged"] and res <= 1e-10 and abs(info[r]["true_res"] - res) < 1e-11
    # GPU stage times (HIP events): every stage ran, and together they fit in the wall time
    g = info[0]["gpu_ms"]
    assert all(v >= 0 for v in g) and g[1] > 0 and g[2] > 0 and g[3] > 0 and sum(g) <= info[0]["t_ms"][0]


def test_nonconvergence_reported(Q):
    L = (4, 4, 4, 4)
    ctx, U = make_ctx(Q, L, 0.3, 0.13, 1.9, 403, nmx=3)
    eta = S.gaussian_field(256, 404)
    psi, info, st = ctx.solve(eta[None], check=False)
    assert st == Q.QDD_ENOCONV and not info[0]["converged"] and info[0]["iters"] == 3
