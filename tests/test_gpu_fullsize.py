"""Dhat (Eq. 2) at the benchmark's full size and launch: 32^3 x 64 lattice, random
SU(3) links exp(i 0.6 H), kappa 0.1357, c_sw 1.9, 8 right-hand sides in FP16
storage with the launch shape the benchmark uses (autotuner cache shipped with
the package), plus FP32 and FP64 with one right-hand side.  Every output site is
compared with the FP64 CPU oracle (tolerances as in the small-lattice parity
tests).  Also the edge cases of the batch size: an empty batch and a batch above
the context's maximum are rejected, and the maximum batch equals single-rhs
applies bit for bit."""
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

    ctx, U = make_ctx(Q, L, 0.6, 0.1357, 1.9, S.gauge_seed(3), max_nrhs=8)
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
