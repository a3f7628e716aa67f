"""The no-allocation Dhat entry point (qdd_dw_hat_static): the odd-site
intermediate in the library's static device scratch instead of the context
workspace.  Same kernels as qdd_dw_hat, so the results must be bit-identical;
two calls in a row, the second with a smaller input, and a request above the
scratch size rejected on the host."""
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


def _pair(Q, ctx, prec, src):
    import torch

    nrhs = src.shape[0]
    fin = ctx.pack(prec, torch.from_numpy(src), True)
    ref = ctx.empty_field(prec, nrhs, True)
    out = ctx.empty_field(prec, nrhs, True)
    ctx.dw_hat(prec, nrhs, fin, ref)
    out.fill_(0xAB)
    ctx.dw_hat_static(prec, nrhs, fin, out)
    torch.cuda.synchronize()
    return ref, out


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_static_scratch_dhat_equals_workspace_dhat(Q, orc, prec):
    import torch

    L = (8, 8, 8, 8)
    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, 1501, max_nrhs=4)
    Vh = int(np.prod(L)) // 2
    print(f"[no-alloc] prec {prec} L {L} nrhs 4 then 1", flush=True)
    # first call: a batch of 4 (interleaved layout)
    src = S.gaussian_field(Vh, 1502, nrhs=4)
    ref, out = _pair(Q, ctx, prec, src)
    assert torch.equal(ref, out)
    if prec == 0:
        A, Ai = orc.clover(L, U, 0.1357, 1.9)
        got = to_np(ctx.unpack(0, out, 4, True))
        for r in range(4):
            assert relerr(got[r], orc.apply_Dhat(L, U, A, Ai, src[r])) < 1e-12
    # second call, smaller input: one rhs (blocked layout, a smaller intermediate)
    src1 = S.gaussian_field(Vh, 1503, nrhs=1)
    ref, out = _pair(Q, ctx, prec, src1)
    assert torch.equal(ref, out)
    # a smaller lattice on a context of its own shares the same array
    L2 = (4, 4, 4, 8)
    ctx2, _ = make_ctx(Q, L2, 0.6, 0.1357, 1.9, 1504, max_nrhs=2)
    src2 = S.gaussian_field(int(np.prod(L2)) // 2, 1505, nrhs=2)
    ref, out = _pair(Q, ctx2, prec, src2)
    assert torch.equal(ref, out)


def test_static_scratch_size_limit(Q):
    import torch

    # 16^3 x 32: the FP64 intermediate takes 12.6 MB per rhs, so 5 rhs fit the
    # 64 MiB scratch and 6 do not
    L = (32, 16, 16, 16)
    ctx, _ = make_ctx(Q, L, 0.6, 0.1357, 1.9, 1506, max_nrhs=6, nkv=1)
    Vh = int(np.prod(L)) // 2
    print(f"[no-alloc] size limit L {L}", flush=True)
    src = S.gaussian_field(Vh, 1507, nrhs=6)
    fin = ctx.pack(0, torch.from_numpy(src), True)
    out = ctx.empty_field(0, 6, True)
    with pytest.raises(Q.QddError) as ei:
        ctx.dw_hat_static(0, 6, fin, out)
    assert ei.value.status == Q.QDD_EINVAL and "static scratch" in str(ei.value)
    ref, out5 = _pair(Q, ctx, 0, src[:5])
    assert torch.equal(ref, out5)
