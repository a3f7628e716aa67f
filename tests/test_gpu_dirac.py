"""GPU parity of the clover-Wilson operator D (Eq. 1) and its Schur complement
Dhat (Eq. 2) against the FP64 CPU oracle, through the C ABI.

Tolerances (max-abs error / max-abs reference): FP64 1e-12; FP32 1e-5; FP16
storage 5e-3 (each stored operand -- spinor, link, clover, the odd-site
intermediate and the output -- is rounded to FP16 with unit roundoff 2^-11 ~
4.9e-4 relative to its site maximum; seven such roundings along the Dhat path
bound the error by ~7 u_h ~ 3.4e-3, rounded up)."""
import numpy as np
import pytest

from paper_1011_0911_amd import synth as S
from tests.gpu_util import make_ctx, relerr, to_np

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 5e-3}
LATTICES = [(4, 4, 4, 4), (6, 4, 4, 4), (8, 6, 4, 4), (4, 4, 6, 8)]


@pytest.fixture(scope="module")
def Q():
    import torch
    from paper_1011_0911_amd import qdd

    assert torch.cuda.is_available()
    qdd.lib()
    return qdd


@pytest.mark.parametrize("L", LATTICES)
@pytest.mark.parametrize("bc", [-1, 1])
def test_dw_parity_all_precisions(Q, orc, L, bc):
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.5, 0.1355, 1.9, 100 + V, bc=bc)
    A, _ = orc.clover(L, U, 0.1355, 1.9)
    psi = S.gaussian_field(V, 7)
    ref = orc.apply_D(L, U, A, psi, bc=bc)
    for prec in (0, 1, 2):
        out = to_np(ctx.apply_dw(psi[None], prec))[0]
        e = relerr(out, ref)
        print(f"D L={L} bc={bc} prec={prec} err={e:.2e}")
        assert e < TOL[prec], (prec, e)


@pytest.mark.parametrize("L", LATTICES)
def test_dhat_parity_all_precisions(Q, orc, L):
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 200 + V)
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    pe = S.gaussian_field(V // 2, 8)
    ref = orc.apply_Dhat(L, U, A, Ai, pe)
    for prec in (0, 1, 2):
        out = to_np(ctx.apply_dhat(pe[None], prec))[0]
        e = relerr(out, ref)
        print(f"Dhat L={L} prec={prec} err={e:.2e}")
        assert e < TOL[prec], (prec, e)


def test_config1_field_dhat_and_csw0(Q, orc):
    L = (4, 4, 4, 4)
    ctx, U = make_ctx(Q, L, 0.3, 0.13, 1.9, S.gauge_seed(1))
    A, Ai = orc.clover(L, U, 0.13, 1.9)
    pe = S.gaussian_field(256, S.source_seed(1))[S.even_sites(L)]
    assert relerr(to_np(ctx.apply_dhat(pe[None], 0))[0], orc.apply_Dhat(L, U, A, Ai, pe)) < 1e-12
    ctx.set_params(0.13, 0.0)
    A0, Ai0 = orc.clover(L, U, 0.13, 0.0)
    assert relerr(to_np(ctx.apply_dhat(pe[None], 0))[0], orc.apply_Dhat(L, U, A0, Ai0, pe)) < 1e-12


@pytest.mark.parametrize("kernel", [0, 1])
def test_batched_equals_single_rhs(Q, kernel):
    # for every launch shape, the batched apply equals single-rhs applies with the
    # same shape bit for bit; shapes of different kernel variants agree to the
    # last rounding (the staged variant orders its operations differently)
    L = (8, 6, 4, 4)
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.5, 0.1355, 1.9, 301, max_nrhs=5)
    n = V // 2 if kernel == 0 else V
    psi = S.gaussian_field(n, 9, nrhs=5)
    app = ctx.apply_dhat if kernel == 0 else ctx.apply_dw
    for prec in (0, 1):
        base = None
        shapes = [(64, 1, 0, 0), (128, 2, 1, 0), (256, 4, 1, 0), (192, 4, 0, 0), (128, 1, 1, 16),
                  (256, 2, 2, 32), (64, 1, 2, 16), (192, 1, 1, 64), (128, 1, 2, 0), (256, 4, 2, 0)]
        if kernel == 0:  # the LDS-staged variant (nr = 0): tiles of sb sites, block/sb lanes per site
            shapes += [(64, 0, 0, 0), (128, 0, 1, 32), (256, 0, 2, 64), (256, 0, 1, 16), (192, 0, 0, 32), (128, 0, 3, 32)]
        shapes += [(128, 1, 3, 0), (256, 1, 3, 32)]
        if kernel == 0:  # streaming loads / stores for the single-use data (xcd + 4, + 8), compressed links (+ 16)
            shapes += [(256, 1, 4, 32), (128, 1, 14, 0), (64, 1, 11, 16), (256, 1, 8, 0), (256, 1, 16, 32),
                       (128, 1, 27, 0), (64, 1, 22, 16)]
        for block, nr, xcd, sb in shapes:
            if nr == 0 and 108 * (sb or block) * (16 if prec == 0 else 8) > 65536:
                continue  # staged tile does not fit the LDS budget in this precision
            ctx.set_launch(kernel, prec, block, nr, xcd, sb)
            ref = np.stack([to_np(app(psi[r:r + 1], prec))[0] for r in range(5)])
            out = to_np(app(psi, prec))
            assert np.array_equal(out, ref), (prec, block, nr, xcd, sb)
            if base is None:
                base = out
            assert relerr(out, base) <= (1e-15 if prec == 0 else 1e-6), (prec, block, nr, xcd, sb)
        ctx.set_launch(kernel, prec, 256, 1, 1, 0)


def test_compressed_links_parity(Q, orc):
    # links read as two rows with the third rebuilt (and the antiperiodic time
    # sign of the boundary links put back): Dhat against the oracle in every
    # precision, batched and single right-hand side
    L = (8, 4, 4, 6)
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 307, max_nrhs=3)
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    psi = S.gaussian_field(V // 2, 15, nrhs=3)
    ref = np.stack([orc.apply_Dhat(L, U, A, Ai, psi[r]) for r in range(3)])
    for prec in (0, 1, 2):
        for block, xcd, sb in ((256, 16, 32), (128, 31, 0)):
            ctx.set_launch(0, prec, block, 1, xcd, sb)
            assert relerr(to_np(ctx.apply_dhat(psi, prec)), ref) < TOL[prec], (prec, block, xcd)
            assert relerr(to_np(ctx.apply_dhat(psi[1:2], prec))[0], ref[1]) < TOL[prec], (prec, block, xcd)
        ctx.set_launch(0, prec, 256, 1, 1, 0)


@pytest.mark.parametrize("nrhs", [4, 8, 6])
def test_rhs_vector_variant(Q, orc, nrhs):
    # walk field + 32: a lane loads nr consecutive right-hand sides of a component
    # in one word (FP32 nr 2; FP16 nr 2, 4).  Against the oracle, and equal bit
    # for bit to the one-rhs-per-lane kernels (same per-rhs arithmetic and order);
    # 6 rhs with nr 4 leaves the vector condition unmet and takes the plain path.
    # Ragged lattice (192 even sites) so the last tile is partly empty.
    L = (6, 4, 4, 4)
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 308, max_nrhs=nrhs)
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    pe = S.gaussian_field(V // 2, 13, nrhs=nrhs)
    ref = np.stack([orc.apply_Dhat(L, U, A, Ai, pe[r]) for r in range(nrhs)])
    for prec, nrs in ((1, (2,)), (2, (2, 4))):
        for nr in nrs:
            for block, xcd, sb in ((256, 32 + 1, 0), (128, 32 + 3 + 8, 32), (256, 32 + 2 + 16, 64), (64, 32 + 24, 16)):
                if (block // (sb or block)) * nr > 2 * nrhs:
                    continue
                # the one-rhs-per-lane kernel with the same link storage and access bits
                ctx.set_launch(0, prec, 256, 1, xcd - 32, 0)
                scalar = to_np(ctx.apply_dhat(pe, prec))
                ctx.set_launch(0, prec, block, nr, xcd, sb)
                out = to_np(ctx.apply_dhat(pe, prec))
                e = relerr(out, ref)
                assert e < TOL[prec], (prec, nr, block, xcd, sb, e)
                assert np.array_equal(out, scalar), (prec, nr, block, xcd, sb, relerr(out, scalar))
        ctx.set_launch(0, prec, 256, 1, 1, 0)
    with pytest.raises(Q.QddError):  # no rhs-vector loads in FP64 (a 16-byte element already)
        ctx.set_launch(0, 0, 256, 2, 33, 0)
    with pytest.raises(Q.QddError):  # nor for 4 FP32 right-hand sides (32 bytes)
        ctx.set_launch(0, 1, 256, 4, 33, 0)


def test_staged_variant_parity_and_limits(Q, orc):
    # the staged Dhat against the oracle in every precision on a ragged lattice
    # (192 even sites: not a multiple of the 64- or 128-site tiles)
    L = (6, 4, 4, 4)
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 304, max_nrhs=3)
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    pe = S.gaussian_field(V // 2, 12, nrhs=3)
    ref = np.stack([orc.apply_Dhat(L, U, A, Ai, pe[r]) for r in range(3)])
    for prec, sb in ((0, 32), (1, 64), (2, 128)):
        ctx.set_launch(0, prec, 256 if sb < 128 else 128, 0, 1, sb)
        e = relerr(to_np(ctx.apply_dhat(pe, prec)), ref)
        assert e < TOL[prec], (prec, e)
    # tiles whose links + clover exceed 64 KiB of LDS, and the full D, are rejected
    for kernel, prec, block, sb in ((0, 0, 64, 64), (0, 1, 128, 128), (1, 1, 64, 0)):
        with pytest.raises(Q.QddError) as e:
            ctx.set_launch(kernel, prec, block, 0, 1, sb)
        assert e.value.status == Q.QDD_EINVAL
    # streaming access (xcd + 4, + 8) and compressed links (+ 16) exist for the
    # one-rhs-per-lane Dhat kernels only
    for kernel, nr, xcd in ((1, 1, 4), (0, 0, 5), (0, 2, 8), (0, 2, 16), (0, 1, 32), (0, 1, -1)):
        with pytest.raises(Q.QddError) as e:
            ctx.set_launch(kernel, 1, 128, nr, xcd, 32)
        assert e.value.status == Q.QDD_EINVAL


def test_dw_several_masses_in_one_launch(Q, orc):
    # out_r = D(kappa_r) psi_r: the clover diagonal 1/(2 kappa) is the only kappa dependence
    L = (8, 4, 4, 4)
    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.5, 0.1355, 1.9, 305, max_nrhs=3)
    kappas = [0.1350, 0.1357, 0.13]
    psi = S.gaussian_field(V, 13, nrhs=3)
    ref = np.stack([orc.apply_D(L, U, orc.clover(L, U, k, 1.9)[0], psi[r]) for r, k in enumerate(kappas)])
    for prec in (0, 1, 2):
        e = relerr(to_np(ctx.apply_dw_masses(psi, kappas, prec)), ref)
        assert e < TOL[prec], (prec, e)
    with pytest.raises(Q.QddError) as err:
        ctx.apply_dw_masses(psi, [0.1355, -1.0, 0.13])
    assert err.value.status == Q.QDD_EINVAL


def test_pack_unpack_roundtrip(Q):
    L = (4, 4, 4, 8)
    ctx, U = make_ctx(Q, L, 0.5, 0.1355, 1.9, 302, max_nrhs=2)
    psi = S.gaussian_field(512, 10, nrhs=2)
    for even in (0, 1):
        src = psi[:, :256] if even else psi
        for prec, tol in ((0, 0.0), (1, 1e-7), (2, 1e-3)):
            f = ctx.pack(prec, src, even)
            back = to_np(ctx.unpack(prec, f, 2, even))
            assert relerr(back, src) <= tol, (even, prec)


def test_state_and_singular_errors(Q):
    import torch

    L = (4, 4, 4, 4)
    c = Q.Context(L)
    with pytest.raises(Q.QddError) as e:
        c.apply_dhat(np.zeros((1, 128, 4, 3), complex))
    assert e.value.status == Q.QDD_ESTATE
    c.set_gauge(torch.from_numpy(S.random_su3_links(L, 0.6, 5)))
    with pytest.raises(Q.QddError) as e:
        c.set_params(0.1357, 200.0)
    assert e.value.status == Q.QDD_ESINGULAR
    c.set_params(0.1357, 1.9)


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (8, 6, 4, 4)])
def test_fp16_against_quantised_inputs(Q, orc, L):
    # FP16 storage against the oracle fed the same FP16-rounded spinor, links and
    # clover blocks: D (one kernel, FP32 arithmetic) then differs only by the
    # rounding of its output, at most half an FP16 unit of the site's scale; Dhat
    # also rounds its odd-site intermediate t_o = A_o^{-1} H psi_e, emulated here
    # from the FP64 t_o: a component whose FP32 value rounds the other way moves by
    # one unit (2 u_h of its site's scale) and reaches an even neighbour through
    # -1/4 (1 -+ gamma) U, of norm <= 1/2, so by at most u_h times the scale of t_o.
    # Such flips are rare: nearly every site is within the output rounding alone.
    from tests.fp16_util import U_H, q16_clover, q16_links, q16_spinor

    V = int(np.prod(L))
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 500 + V)
    A, Ai = orc.clover(L, U, 0.1357, 1.9)
    Uq, Aq, Aiq = q16_links(U), q16_clover(A), q16_clover(Ai)
    # D on a full field
    psi = S.gaussian_field(V, 501)
    ref = orc.apply_D(L, Uq, Aq, q16_spinor(psi))
    out = to_np(ctx.apply_dw(psi[None], 2))[0]
    site_err = np.abs(out - ref).reshape(V, 12).max(1)
    site_max = np.abs(ref).reshape(V, 12).max(1)
    e_d = (site_err / site_max).max()
    print(f"D FP16 vs quantised inputs {L}: max error / site scale {e_d:.3e} (u_h {U_H:.3e}), "
          f"global {relerr(out, ref):.2e}")
    assert np.all(site_err <= 1.01 * U_H * site_max + 1e-6 * np.abs(ref).max())
    # Dhat
    ev = S.even_sites(L)
    od = np.setdiff1d(np.arange(V), ev)
    pe = S.gaussian_field(V // 2, 502)
    peq = q16_spinor(pe)
    full = np.zeros((V, 4, 3), np.complex128)
    full[ev] = peq
    h_o = -2.0 * orc.apply_D(L, Uq, Aq, full)[od]                      # (H psi_e) on the odd sites
    t_o = np.einsum("vab,vb->va", Aiq[od], h_o.reshape(-1, 12)).reshape(-1, 4, 3)
    t_q = q16_spinor(t_o)
    tf = np.zeros((V, 4, 3), np.complex128)
    tf[od] = t_q
    ref_h = (np.einsum("vab,vb->va", Aq[ev], peq.reshape(-1, 12)).reshape(-1, 4, 3)
             + 0.5 * orc.apply_D(L, Uq, Aq, tf)[ev])                   # A_e psi_e - 1/4 H t_o
    out_h = to_np(ctx.apply_dhat(pe[None], 2))[0]
    Vh = V // 2
    err_h = np.abs(out_h - ref_h).reshape(Vh, 12).max(1)
    smax_h = np.abs(ref_h).reshape(Vh, 12).max(1)
    t_scale = np.abs(t_o).max()
    out_bound = 1.01 * U_H * smax_h + 1e-6 * np.abs(ref_h).max()
    print(f"Dhat FP16 vs quantised inputs {L}: max error / site scale {(err_h / smax_h).max():.3e}, "
          f"sites beyond the output rounding {(err_h > out_bound).mean():.2%}, global {relerr(out_h, ref_h):.2e} "
          f"(unquantised inputs {relerr(out_h, orc.apply_Dhat(L, U, A, Ai, pe)):.2e})")
    assert (err_h > out_bound).mean() <= 0.02
    assert np.all(err_h <= out_bound + 2 * U_H * t_scale)
    assert relerr(out_h, ref_h) < 1e-3
