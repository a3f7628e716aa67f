"""The hot path at the benchmark's full sizes, against the FP64 CPU oracle.

* Dhat (Eq. 2) on the 32^3 x 64 lattice (random SU(3) links exp(i 0.6 H), kappa
  0.1357, c_sw 1.9): 8 right-hand sides in FP16 storage with the launch shape the
  benchmark uses (autotuner cache shipped with the package), plus FP32 and FP64
  with one right-hand side; every output site is compared.
* The FP16-storage Schwarz procedure with 8 right-hand sides in one call (one
  cycle), on the same lattice: every site of a sample of colour-1 blocks (at
  both time boundaries and inside) and of their face neighbours, where the
  oracle's sampled cycle gives exactly the full procedure's values.
* The deflation subspace with 24 vectors on the same lattice (start fields
  orthonormalised without inverse iteration): the basis and the little-operator
  rows (self + 8 faces) of sampled blocks.
* The 1-12-12-1 network forward pass on 24^3 x 48 at sampled sites.
* The batched solves of the 16^3 x 32 (12 rhs, FP32 Schwarz, 20 deflation
  vectors) and 32^3 x 64 (8 rhs, FP16 Schwarz, 24 vectors) workloads as the
  benchmark configures them: every solution's residual, measured again with the
  oracle's FP64 D, is at most 1e-10 and equals the solver's own figure.
* The batch-size edge cases: an empty batch and a batch above the context's
  maximum are rejected, and the maximum batch equals single-rhs applies bit for
  bit."""
import os

import numpy as np
import pytest

from paper_1011_0911_amd import synth as S
from tests.gpu_util import make_ctx, relerr, to_np

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
L = (64, 32, 32, 32)
TOL = {0: 1e-12, 1: 1e-5, 2: 5e-3}


@pytest.fixture(scope="module")
def Q():
    from paper_1011_0911_amd import qdd

    qdd.lib()
    return qdd


@pytest.fixture(scope="module")
def full(Q, orc):
    import torch

    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, S.gauge_seed(3), max_nrhs=8, nkv=1)
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    Vh = int(np.prod(L)) // 2
    src = S.gaussian_field(Vh, 2000 + 300, nrhs=8)
    yield ctx, U, A, Ai, src
    del ctx
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,nrhs", [(2, 8), (1, 1), (0, 1)])
def test_dhat_full_size_at_benchmark_launch(Q, orc, full, prec, nrhs):
    import torch

    ctx, U, A, Ai, src = full
    cache = Q.load_tune_cache(os.path.join(ROOT, "paper_1011_0911_amd", "tune_cache.json"))
    fin = ctx.pack(prec, torch.from_numpy(src[:nrhs]), True)
    fout = ctx.empty_field(prec, nrhs, True)
    ctx.autotune(Q.KERNEL_DHAT, prec, nrhs, fin, fout, reps=3, cache=cache)
    print(f"prec {prec} nrhs {nrhs} launch {ctx.get_launch(Q.KERNEL_DHAT, prec)}", flush=True)
    ctx.dw_hat(prec, nrhs, fin, fout)
    out = to_np(ctx.unpack(prec, fout, nrhs, True))
    for r in range(nrhs):
        ref = orc.apply_Dhat(L, U, A, Ai, src[r])
        e = relerr(out[r], ref)
        print(f"  rhs {r}: err {e:.2e}", flush=True)
        assert e < TOL[prec], (prec, r, e)


def ctx_on(Q, U, Lat, kappa=0.1357, **cfg):
    """A context on given links (no second link generation at full size)."""
    import torch

    c = Q.Context(Lat, Q.default_config(**cfg))
    c.set_gauge(torch.from_numpy(U))
    c.set_params(kappa, 1.9)
    return c


def sample_blocks(Lat, bs, colour, n_mid=2):
    """Blocks of one colour at the first and last time slice of blocks and inside."""
    nb = tuple(np.array(Lat) // np.array(bs))
    out = []
    for t in [0, nb[0] - 1] + [nb[0] // 3 + k for k in range(n_mid)]:
        for x1 in (0, nb[1] // 2):
            c = (t, x1, 1, 0)
            if sum(c) % 2 != colour:
                c = (t, x1, 1, 1)
            out.append(int(np.ravel_multi_index(c, nb)))
    return sorted(set(out))


def block_sites(Lat, bs, blocks):
    """lex sites of the listed blocks (and a block id per lex site)."""
    V = int(np.prod(Lat))
    x = np.array(np.unravel_index(np.arange(V), Lat)).T
    bid = np.ravel_multi_index((x // np.array(bs)).T, tuple(np.array(Lat) // np.array(bs)))
    return np.nonzero(np.isin(bid, blocks))[0], bid


@pytest.mark.parametrize("prec,variant,tol", [(2, 0, 3e-3), (1, 3, 1e-5)])
def test_sap_8rhs_full_size(Q, orc, full, prec, variant, tol):
    # one Schwarz cycle (both colours, nmr 4) on 8 right-hand sides in one call,
    # FP16 storage with the default (LDS-staged) kernel and FP32 storage with the
    # LDS-staged variant 3; FP16 tolerance 3e-3 as for the small lattices: six
    # FP16-stored quantities (source, links, both clover blocks, rho, V), unit
    # 2^-11 each
    import torch

    ctx0, U, A, Ai, _ = full
    bs = (4, 4, 4, 4)
    V = int(np.prod(L))
    c = ctx_on(Q, U, L, max_nrhs=8, sap_bs=bs, ncy=1, nmr=4, sap_prec=prec, precond=Q.PRECOND_SAP, nkv=1)
    if variant:
        c.set_launch(Q.KERNEL_SAP, prec, 0, variant, 0, 0)
    eta = S.gaussian_field(V, 2350, nrhs=8)
    print(f"[full-size SAP] prec {prec} variant {variant}, 8 rhs, 32^3x64, one cycle", flush=True)
    out = c.sap(eta)
    white = sample_blocks(L, bs, 1)
    sites, bid = block_sites(L, bs, white)
    nb = tuple(np.array(L) // np.array(bs))
    cov = set(white)
    for b in white:
        cc = np.array(np.unravel_index(b, nb))
        for mu in range(4):
            for d in (1, -1):
                e = cc.copy()
                e[mu] = (e[mu] + d) % nb[mu]
                cov.add(int(np.ravel_multi_index(e, nb)))
    allsites = np.nonzero(np.isin(bid, sorted(cov)))[0]
    got = to_np(out[:, torch.from_numpy(allsites).to(out.device)])
    del c, out
    torch.cuda.empty_cache()
    for r in range(8):
        ref = orc.sap_one_cycle_on_blocks(L, U, A, Ai, eta[r], bs, 4, white)[allsites]
        e = relerr(got[r], ref)
        print(f"  rhs {r}: err {e:.2e} over {allsites.size} sites", flush=True)
        assert e < tol, (r, e)


def test_deflation_ns24_full_size(Q, orc, full):
    # basis (block Gram-Schmidt of 24 start fields, FP64) and little operator
    # A = W^dag D W (self + 8 faces) on sampled blocks of the 32^3 x 64 lattice
    import torch

    ctx0, U, A, Ai, _ = full
    bs = (4, 4, 4, 4)
    Ns = 24
    V = int(np.prod(L))
    c = ctx_on(Q, U, L, max_nrhs=1, sap_bs=bs, sap_prec=2, dfl_Ns=Ns, dfl_bs=bs, dfl_nit=0,
               precond=Q.PRECOND_DFL, nkv=1)
    init = S.gaussian_field(V, 5003, nrhs=Ns)
    print("[full-size deflation] Ns 24, 32^3x64", flush=True)
    c.dfl_build(init)
    basis, little = c.dfl_export()
    rows = sample_blocks(L, bs, 0) + sample_blocks(L, bs, 1)
    sites, _ = block_sites(L, bs, rows)
    gb = to_np(basis[:, torch.from_numpy(sites).to(basis.device)])
    gl = to_np(little[torch.tensor(rows, device=little.device)])
    del c, basis, little
    torch.cuda.empty_cache()
    d = orc.Deflation(L, bs, Ns)
    d.set_fields_on_blocks(U, A, init, rows)
    del init
    eb = relerr(gb, d.basis()[:, sites])
    el = relerr(gl, d.little()[rows])
    print(f"  {len(rows)} blocks: basis err {eb:.2e} little err {el:.2e}", flush=True)
    assert eb < 1e-10 and el < 1e-10


def test_net_forward_24c48_full_size(Q, orc):
    # the 1-12-12-1 network of the learned workload on its 24^3 x 48 lattice, FP32
    # activations and BF16-exact weights, at sites spread over the lattice
    # (corners and both time boundaries included)
    import torch

    from tests.test_gpu_net import bf16

    L5 = (48, 24, 24, 24)
    V = int(np.prod(L5))
    ch = [1, 12, 12, 1]
    U = S.random_su3_links(L5, 0.6, S.gauge_seed(5))
    c = ctx_on(Q, U, L5, max_nrhs=1, sap_prec=1, dfl_Ns=1, precond=Q.PRECOND_DFL, use_net=1, net_nl=3, net_ch=ch,
               nkv=1)
    W = bf16(S.random_weights(c.net_num_weights(), 5004, 0.3))
    c.net_set_weights(W)
    x = S.gaussian_field(V, 5005)
    print("[full-size network] 1-12-12-1, 24^3x48", flush=True)
    out = to_np(c.net_forward(x))
    del c
    torch.cuda.empty_cache()
    sites = sorted(set([0, V - 1, 24 ** 3 - 1, V - 24 ** 3] + list(range(5, V, V // 61))))
    ref = orc.net_forward_on_sites(L5, U, ch, W, x[None], sites)
    e = relerr(out[sites], ref)
    print(f"  {len(sites)} sites: err {e:.2e}", flush=True)
    assert e < 1e-5


def _tune_from_cache(Q, c, nrhs):
    """Schwarz kernel variant for nrhs from the package's tuner cache (read only;
    a shape missing from it is timed here and not stored)."""
    cache = Q.load_tune_cache(os.path.join(ROOT, "paper_1011_0911_amd", "tune_cache.json"))
    c.tune_sap(nrhs, cache=cache)


def _check_solutions(orc, Lat, U, A, eta, psi, info, tag):
    # the solver stops on its own FP64 residual; the oracle's D measures it again
    for r in range(len(eta)):
        res = float(np.linalg.norm(eta[r] - orc.apply_D(Lat, U, A, psi[r])) / np.linalg.norm(eta[r]))
        print(f"  {tag} rhs {r}: iters {info[r]['iters']} residual (oracle D) {res:.3e} "
              f"(solver {info[r]['true_res']:.3e})", flush=True)
        assert info[r]["converged"] and res <= 1e-10, (r, res)
        assert abs(res - info[r]["true_res"]) <= 1e-13, (r, res, info[r]["true_res"])


def test_workload2_solve_full_size(Q, orc):
    # 16^3 x 32, eps 0.5, kappa 0.1355: FP32 Schwarz (4^4 blocks, 4 MR steps, 5
    # cycles), 20 deflation vectors, FP64 flexible GCR; 12 right-hand sides in one
    # batched solve, as the benchmark runs it
    import torch

    from paper_1011_0911_amd import workloads as W

    w = W.WORKLOADS[2]
    Lw, n = w["L"], w["nrhs"]
    V = int(np.prod(Lw))
    U = S.random_su3_links(Lw, w["eps"], S.gauge_seed(2))
    A, _ = orc.clover(Lw, U, w["kappa"], w["csw"])
    c = ctx_on(Q, U, Lw, kappa=w["kappa"], **W.solver_config(w, n))
    _tune_from_cache(Q, c, n)
    print("[workload 2] 16^3x32, 12 rhs, FP32 SAP, Ns 20", flush=True)
    c.dfl_build(S.gaussian_field(V, S.dfl_seed(2), nrhs=w["dfl_Ns"]))
    eta = np.stack([S.gaussian_field(V, S.source_seed(2, r)) for r in range(n)])
    psi, info, _ = c.solve(eta)
    psi = to_np(psi)
    del c
    torch.cuda.empty_cache()
    _check_solutions(orc, Lw, U, A, eta, psi, info, "w2")


def test_workload3_solve_full_size(Q, orc, full):
    # 32^3 x 64, eps 0.6, kappa 0.1357: FP16 Schwarz storage, 24 deflation vectors,
    # FP64 flexible GCR; 8 right-hand sides in one batched solve, as the benchmark
    # runs it
    import torch

    from paper_1011_0911_amd import workloads as W

    ctx0, U, A, Ai, _ = full
    w = W.WORKLOADS[3]
    n = w["nrhs"]
    V = int(np.prod(L))
    c = ctx_on(Q, U, L, kappa=w["kappa"], **W.solver_config(w, n))
    _tune_from_cache(Q, c, n)
    print("[workload 3] 32^3x64, 8 rhs, FP16 SAP, Ns 24", flush=True)
    c.dfl_build(S.gaussian_field(V, S.dfl_seed(3), nrhs=w["dfl_Ns"]))
    eta = np.stack([S.gaussian_field(V, S.source_seed(3, r)) for r in range(n)])
    psi, info, _ = c.solve(eta)
    psi = to_np(psi)
    del c
    torch.cuda.empty_cache()
    _check_solutions(orc, L, U, A, eta, psi, info, "w3")


def test_batch_size_edges(Q):
    L4 = (4, 4, 4, 4)
    ctx, U = make_ctx(Q, L4, 0.5, 0.1355, 1.9, 303, max_nrhs=64)
    for bad in (0, 65):
        with pytest.raises(Q.QddError) as e:
            ctx.dw_hat(1, bad, ctx.empty_field(1, 64, True), ctx.empty_field(1, 64, True))
        assert e.value.status == Q.QDD_EINVAL
    psi = S.gaussian_field(128, 11, nrhs=64)
    for prec in (0, 1, 2):
        ref = np.stack([to_np(ctx.apply_dhat(psi[r:r + 1], prec))[0] for r in range(64)])
        assert np.array_equal(to_np(ctx.apply_dhat(psi, prec)), ref), prec
