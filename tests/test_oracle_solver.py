"""Pins of the oracle's solver pieces: flexible GCR, MR block solves, the
two-colour Schwarz procedure and local deflation (Sect. 3-4 of the paper name
the locally deflated Schwarz-preconditioned GCR; its steps are this library's
reading, pinned here against dense linear algebra and exact identities)."""
import numpy as np
import pytest

from paper_1011_0911_amd import synth as S


def dense(apply, n_in, shape_in):
    cols = []
    for k in range(n_in):
        e = np.zeros(n_in, complex)
        e[k] = 1
        cols.append(apply(e.reshape(shape_in)).reshape(-1))
    return np.array(cols).T


def setup_field(orc, L, eps, kappa, seed, csw=1.9):
    U = S.random_su3_links(L, eps, seed)
    A, Ai = orc.clover(L, U, kappa, csw)
    return U, A, Ai


# ---------------------------------------------------------------- FGCR
def test_fgcr_dhat_matches_dense_lu_4x4(orc):
    L = (4, 4, 4, 4)
    U, A, Ai = setup_field(orc, L, 0.3, 0.13, S.gauge_seed(1))
    eta = S.gaussian_field(256, S.source_seed(1))[S.even_sites(L)]
    x, info = orc.fgcr(L, U, A, Ai, eta, op="Dhat", tol=1e-10)
    assert info["converged"] and info["relres"] <= 1e-10
    Dh = dense(lambda f: orc.apply_Dhat(L, U, A, Ai, f), 128 * 12, (128, 4, 3))
    xd = np.linalg.solve(Dh, eta.reshape(-1)).reshape(eta.shape)
    cond = np.linalg.cond(Dh)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 2 * cond * 1e-10


def test_fgcr_full_D_matches_dense_lu(orc):
    L = (4, 4, 2, 2)
    V = 64
    U, A, Ai = setup_field(orc, L, 0.5, 0.1355, 7)
    eta = S.gaussian_field(V, 8)
    x, info = orc.fgcr(L, U, A, Ai, eta, op="D", tol=1e-12)
    assert info["converged"]
    Dm = dense(lambda f: orc.apply_D(L, U, A, f), V * 12, (V, 4, 3))
    xd = np.linalg.solve(Dm, eta.reshape(-1)).reshape(eta.shape)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


def test_fgcr_unpreconditioned_equals_gmres_residuals(orc):
    # M = 1 and no restart: GCR minimises |eta - D psi| over the Krylov space,
    # exactly as GMRES; the GMRES residuals come from a least-squares solve over
    # an orthonormal Krylov basis built here with numpy.
    L = (2, 2, 2, 4)
    V = 32
    U, A, Ai = setup_field(orc, L, 0.5, 0.1355, 17)
    eta = S.gaussian_field(V // 2, 18)
    n = 20
    _, info = orc.fgcr(L, U, A, Ai, eta, op="Dhat", nkv=64, nmx=n, tol=1e-30, nhist=n + 1)
    Dh = dense(lambda f: orc.apply_Dhat(L, U, A, Ai, f), V // 2 * 12, (V // 2, 4, 3))
    b = eta.reshape(-1)
    Q = [b / np.linalg.norm(b)]
    gm = [1.0]
    for k in range(1, n + 1):
        w = Dh @ Q[-1]
        for _ in range(2):
            for q in Q:
                w = w - np.vdot(q, w) * q
        Q.append(w / np.linalg.norm(w))
        K = np.array(Q[:k]).T
        AK = Dh @ K
        y, *_ = np.linalg.lstsq(AK, b, rcond=None)
        gm.append(np.linalg.norm(b - AK @ y) / np.linalg.norm(b))
    hist = info["history"]
    assert len(hist) == n + 1
    assert np.allclose(hist, gm, rtol=1e-8, atol=1e-14)
    assert np.all(np.diff(hist) <= 1e-14)
    # without a restart the back-substituted update reproduces the recursive
    # residual: the solve stops after the first cycle at the GMRES iteration count
    tol = 1e-6
    k_gm = next(k for k, v in enumerate(gm) if v <= tol)
    x, info2 = orc.fgcr(L, U, A, Ai, eta, op="Dhat", nkv=64, nmx=64, tol=tol)
    assert info2["converged"] and info2["restarts"] == 0 and info2["iters"] == k_gm
    assert np.linalg.norm(b - Dh @ x.reshape(-1)) / np.linalg.norm(b) <= tol


def test_fgcr_restarts_reach_tolerance_and_zero_source(orc):
    L = (4, 4, 4, 4)
    U, A, Ai = setup_field(orc, L, 0.3, 0.13, S.gauge_seed(1))
    eta = S.gaussian_field(256, 3)
    x, info = orc.fgcr(L, U, A, Ai, eta, op="D", nkv=4, tol=1e-10)
    assert info["converged"] and info["restarts"] > 0
    r = eta - orc.apply_D(L, U, A, x)
    assert np.linalg.norm(r) / np.linalg.norm(eta) <= 1e-10
    x0, info0 = orc.fgcr(L, U, A, Ai, np.zeros_like(eta), op="D")
    assert info0["converged"] and info0["iters"] == 0 and not x0.any()
    _, info1 = orc.fgcr(L, U, A, Ai, eta, op="D", nmx=3)
    assert not info1["converged"] and info1["status"] == -4


# ---------------------------------------------------------------- MR / SAP
def block_index_sets(L, bs):
    x = np.array(np.unravel_index(np.arange(int(np.prod(L))), L)).T
    bc = x // np.array(bs)
    nb = np.array(L) // np.array(bs)
    bid = np.ravel_multi_index(bc.T, nb)
    col = bc.sum(1) % 2
    return bid, col, int(np.prod(nb))


def dense_block_inverse_op(Dm, L, bs, colour):
    """B_c = sum_{blocks of colour c} P D_Lambda^{-1} P with D_Lambda = P D P (Dirichlet)."""
    bid, col, nblk = block_index_sets(L, bs)
    n = Dm.shape[0]
    B = np.zeros((n, n), complex)
    for b in range(nblk):
        sites = np.where(bid == b)[0]
        if col[sites[0]] != colour:
            continue
        idx = (sites[:, None] * 12 + np.arange(12)).ravel()
        B[np.ix_(idx, idx)] = np.linalg.inv(Dm[np.ix_(idx, idx)])
    return B


def test_sap_error_propagation_with_exact_block_solves(orc):
    # with (numerically) exact block solves, 1 - M_sap D = [(1 - B_1 D)(1 - B_0 D)]^ncy
    L, bs = (4, 4, 2, 2), (2, 2, 1, 1)
    V = 64
    U, A, Ai = setup_field(orc, L, 0.5, 0.1355, 27)
    Dm = dense(lambda f: orc.apply_D(L, U, A, f), V * 12, (V, 4, 3))
    B0 = dense_block_inverse_op(Dm, L, bs, 0)
    B1 = dense_block_inverse_op(Dm, L, bs, 1)
    I = np.eye(V * 12)
    eta = S.gaussian_field(V, 28)
    for ncy in (1, 3):
        E = np.linalg.matrix_power((I - B1 @ Dm) @ (I - B0 @ Dm), ncy)
        Msap = (I - E) @ np.linalg.inv(Dm)
        psi = orc.sap(L, U, A, Ai, eta, bs, ncy, 200)
        ref = (Msap @ eta.reshape(-1)).reshape(eta.shape)
        assert np.linalg.norm(psi - ref) / np.linalg.norm(ref) < 1e-11


def test_mr_block_residual_decreases_with_nmr(orc):
    # the block residual |rho_L - D_L v| after one half sweep is non-increasing in nmr
    # and tends to zero (MR on a positive-real block operator)
    L, bs = (4, 4, 4, 4), (2, 2, 2, 2)
    V = 256
    U, A, Ai = setup_field(orc, L, 0.5, 0.1355, 37)
    eta = S.gaussian_field(V, 38)
    bid, col, _ = block_index_sets(L, bs)
    black = col == 0
    prev = np.inf
    for nmr in (1, 2, 4, 8, 32, 128):
        psi, rho = orc.sap_half_sweep(L, U, A, Ai, bs, nmr, 0, eta, np.zeros_like(eta), eta.copy())
        res = np.linalg.norm(rho[black])
        assert res <= prev * (1 + 1e-12)
        prev = res
    assert prev / np.linalg.norm(eta[black]) < 1e-8
    assert not psi[~black].any()


def test_mr_single_step_is_the_minimal_residual_step(orc):
    # one MR step on the block Schur complement: the new even-site residual
    # r1 = b - alpha Dhat_L b is orthogonal to Dhat_L b (that is what "minimal
    # residual" means), and the odd sites are solved exactly
    L, bs = (4, 4, 4, 4), (2, 2, 2, 2)
    V = 256
    U, A, Ai = setup_field(orc, L, 0.5, 0.1355, 39)
    eta = S.gaussian_field(V, 40)
    psi, rho = orc.sap_half_sweep(L, U, A, Ai, bs, 1, 0, eta, np.zeros_like(eta), eta.copy())
    bid, col, nblk = block_index_sets(L, bs)
    par = np.array(np.unravel_index(np.arange(V), L)).sum(0) % 2
    for blk in [b for b in range(nblk) if col[np.where(bid == b)[0][0]] == 0][:3]:
        sites = np.where(bid == blk)[0]
        idx = (sites[:, None] * 12 + np.arange(12)).ravel()
        cols = []
        for j in idx:
            e = np.zeros(V * 12, complex)
            e[j] = 1
            cols.append(orc.apply_D(L, U, A, e.reshape(V, 4, 3)).reshape(-1)[idx])
        DL = np.array(cols).T
        ev = np.repeat(par[sites] == 0, 12)
        Dee, Deo, Doe, Doo = DL[np.ix_(ev, ev)], DL[np.ix_(ev, ~ev)], DL[np.ix_(~ev, ev)], DL[np.ix_(~ev, ~ev)]
        rl = eta.reshape(-1)[idx]
        bvec = rl[ev] - Deo @ np.linalg.solve(Doo, rl[~ev])
        Dh = Dee - Deo @ np.linalg.solve(Doo, Doe)
        p = Dh @ bvec
        r1 = rho.reshape(-1)[idx][ev]
        assert np.abs(rho.reshape(-1)[idx][~ev]).max() < 1e-13
        assert abs(np.vdot(p, r1)) < 1e-13 * np.linalg.norm(p) * np.linalg.norm(bvec)
        beta = np.vdot(p, bvec - r1) / np.vdot(p, p)
        assert np.linalg.norm(bvec - r1 - beta * p) < 1e-13 * np.linalg.norm(bvec)


# ---------------------------------------------------------------- deflation
def coarse_dense_from_little(little, L, bs):
    nb = np.array(L) // np.array(bs)
    nblk, _, Ns, _ = little.shape
    M = np.zeros((nblk * Ns, nblk * Ns), complex)
    for b in range(nblk):
        c = np.array(np.unravel_index(b, nb))
        M[b * Ns:(b + 1) * Ns, b * Ns:(b + 1) * Ns] += little[b, 0]
        for mu in range(4):
            for dirn in range(2):
                cc = c.copy()
                cc[mu] = (cc[mu] + (1 if dirn == 0 else -1)) % nb[mu]
                bb = np.ravel_multi_index(cc, nb)
                M[b * Ns:(b + 1) * Ns, bb * Ns:(bb + 1) * Ns] += little[b, 1 + 2 * mu + dirn]
    return M


@pytest.fixture(scope="module")
def dfl8(orc):
    L = (8, 8, 8, 8)
    V = 4096
    U, A, Ai = setup_field(orc, L, 0.5, 0.1355, 47)
    Ns = 6
    d = orc.Deflation(L, (4, 4, 4, 4), Ns)
    init = S.gaussian_field(V, 48, nrhs=Ns)
    d.build(U, A, Ai, (4, 4, 4, 4), 2, 4, 2, init)
    return L, U, A, Ai, d


def test_dfl_basis_block_orthonormal(dfl8):
    L, U, A, Ai, d = dfl8
    W = d.basis()
    bid, _, nblk = block_index_sets(L, (4, 4, 4, 4))
    for b in (0, 5, 15):
        Wb = W[:, bid == b].reshape(d.Ns, -1)
        assert np.abs(Wb.conj() @ Wb.T - np.eye(d.Ns)).max() < 1e-13


def test_dfl_little_operator_is_dense_WdagDW(orc, dfl8):
    L, U, A, Ai, d = dfl8
    M = coarse_dense_from_little(d.little(), L, (4, 4, 4, 4))
    n = d.nblk * d.Ns
    cols = []
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1
        f = d.prolong(e.reshape(d.nblk, d.Ns))
        cols.append(d.restrict(orc.apply_D(L, U, A, f)).reshape(-1))
    ref = np.array(cols).T
    assert np.abs(M - ref).max() < 1e-13 * np.abs(ref).max()
    c = S.gaussian_field(d.nblk * d.Ns // 12, 9).reshape(d.nblk, d.Ns)
    assert np.abs(d.coarse_apply(c).reshape(-1) - M @ c.reshape(-1)).max() < 1e-12


def test_dfl_projector_identities(orc, dfl8):
    L, U, A, Ai, d = dfl8
    eta = S.gaussian_field(4096, 49)

    def C(r):
        c, it = d.coarse_solve(d.restrict(r), 1e-14)
        assert it >= 0
        return d.prolong(c)

    def PL(r):
        return r - orc.apply_D(L, U, A, C(r))

    p1 = PL(eta)
    p2 = PL(p1)
    assert np.linalg.norm(p2 - p1) / np.linalg.norm(p1) < 1e-11
    assert np.abs(d.restrict(p1)).max() / np.abs(d.restrict(eta)).max() < 1e-11


def test_dfl_complete_subspace_solves_in_one_iteration(orc):
    # one deflation block = the whole 2^4 lattice and Ns = 192 = its dimension:
    # C = D^{-1} exactly, so M(r) = D^{-1} r and FGCR stops after one step
    L = (2, 2, 2, 2)
    V = 16
    U, A, Ai = setup_field(orc, L, 0.5, 0.1355, 57)
    d = orc.Deflation(L, (2, 2, 2, 2), 192)
    d.set_fields(U, A, S.gaussian_field(V, 58, nrhs=192))
    eta = S.gaussian_field(V, 59)
    x, info = orc.fgcr(L, U, A, Ai, eta, op="D", prec="dfl", sap_bs=(1, 1, 1, 1), ncy=1, nmr=1, dfl=d,
                       coarse_tol=1e-14, tol=1e-10)
    assert info["converged"] and info["iters"] == 1


def test_deflated_sap_gcr_reaches_tolerance(orc, dfl8):
    L, U, A, Ai, d = dfl8
    eta = S.gaussian_field(4096, 50)
    x, info = orc.fgcr(L, U, A, Ai, eta, op="D", prec="dfl", sap_bs=(4, 4, 4, 4), ncy=5, nmr=4, dfl=d,
                       coarse_tol=1e-8, tol=1e-10)
    r = eta - orc.apply_D(L, U, A, x)
    assert info["converged"] and np.linalg.norm(r) / np.linalg.norm(eta) <= 1e-10
    _, info_sap = orc.fgcr(L, U, A, Ai, eta, op="D", prec="sap", sap_bs=(4, 4, 4, 4), ncy=5, nmr=4, tol=1e-10)
    assert info_sap["converged"]
    assert info["iters"] <= info_sap["iters"]
