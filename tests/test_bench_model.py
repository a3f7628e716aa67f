"""The benchmark's byte models (CPU): the per-site bytes of the two Dhat passes
and of an ideal single pass, checked against the reals each pass touches by
definition (Eq. 2 split into t_o = A_o^{-1} H_oe psi_e and out = A_e psi_e -
1/4 H_eo t_o; links 8 x 18 reals, or 8 x 12 when two rows are read; Hermitian
6x6 clover blocks as 36 reals each)."""
import bench


def test_two_pass_single_rhs():
    # pass A: psi_e 24 + links 144 + A_o^{-1} 72 + t_o 24; pass B: t_o 24 + links
    # 144 + psi_e 24 + A_e 72 + out 24 -> 552 reals per even site
    assert sum(bench.bytes_per_site(0, 1)) == 552 * 8
    assert sum(bench.bytes_per_site(1, 1)) == 552 * 4
    # FP16 storage adds one FP32 scale per spinor access: 2 in pass A, 3 in pass B
    assert sum(bench.bytes_per_site(2, 1)) == 552 * 2 + 5 * 4


def test_compressed_links_and_batches():
    # two link rows read: 8 x 12 reals per pass instead of 8 x 18
    assert sum(bench.bytes_per_site(0, 1, True)) == (552 - 2 * 48) * 8
    # 8 rhs in FP16: spinors scale with the batch, links and clover do not
    a, b = bench.bytes_per_site(2, 8, True)
    assert a == (48 * 8 + 96 + 72) * 2 + 8 * 8 == 1168
    assert b == (72 * 8 + 96 + 72) * 2 + 12 * 8 == 1584


def test_ideal_single_pass():
    # psi_e in and out once per rhs, links once, both clover blocks once
    assert bench.fused_bytes_per_site(0, 1) == 336 * 8
    assert bench.fused_bytes_per_site(1, 1) == 336 * 4
    assert bench.fused_bytes_per_site(2, 8, True) == (48 * 8 + 96 + 144) * 2 + 8 * 8
    # never more than the two passes
    for prec in (0, 1, 2):
        for n in (1, 4, 8, 12):
            for comp in (False, True):
                assert bench.fused_bytes_per_site(prec, n, comp) < sum(bench.bytes_per_site(prec, n, comp))
