"""The FP16 storage format of the GPU operands, emulated in numpy for parity
tests against oracle inputs that carry the same rounding (test infrastructure,
not the oracle).  Spinors: per site a FP32 scale s = max |Re|, |Im| over the 12
components and the components v / s rounded to FP16 (round to nearest even),
read back as FP16 -> FP32 times s.  Links and the packed Hermitian clover blocks
(6 real diagonal entries and the 15 complex entries above the diagonal of each
6x6 chiral block): FP64 -> FP32 -> FP16, no scale."""
import numpy as np

U_H = 2.0 ** -11  # unit roundoff of FP16


def q16_spinor(psi):
    """psi (..., 4, 3) complex -> the values the GPU reads back from FP16 storage."""
    v = psi.reshape(psi.shape[:-2] + (12,))
    re, im = v.real.astype(np.float32), v.imag.astype(np.float32)
    m = np.maximum(np.abs(re).max(-1), np.abs(im).max(-1))
    sc = np.where(m > 0, m, np.float32(1)).astype(np.float32)
    inv = (np.float32(1) / sc).astype(np.float32)[..., None]
    qr = (re * inv).astype(np.float16).astype(np.float32) * sc[..., None]
    qi = (im * inv).astype(np.float16).astype(np.float32) * sc[..., None]
    return (qr.astype(np.float64) + 1j * qi.astype(np.float64)).reshape(psi.shape)


def _q(x):
    return x.astype(np.float32).astype(np.float16).astype(np.float64)


def q16_links(U):
    return _q(U.real) + 1j * _q(U.imag)


def q16_clover(A):
    """A (V, 12, 12), block diagonal in the chiral basis (spins 0-1, 2-3)."""
    out = np.zeros_like(A)
    iu = np.triu_indices(6, 1)
    for b in range(2):
        M = A[:, 6 * b:6 * b + 6, 6 * b:6 * b + 6]
        Q = np.zeros_like(M)
        d = _q(np.einsum("vii->vi", M).real)
        Q[:, np.arange(6), np.arange(6)] = d
        up = M[:, iu[0], iu[1]]
        Q[:, iu[0], iu[1]] = _q(up.real) + 1j * _q(up.imag)
        Q[:, iu[1], iu[0]] = np.conj(Q[:, iu[0], iu[1]])
        out[:, 6 * b:6 * b + 6, 6 * b:6 * b + 6] = Q
    return out
