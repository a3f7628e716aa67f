"""Pins of the oracle's gauge-covariant parallel-transport network (the learned
preconditioner stage): a special case that reduces to the Wilson operator,
gauge covariance, exact adjointness of the backward pass and central finite
differences of the loss."""
import numpy as np
import pytest

from paper_1011_0911_amd import synth as S
from tests.test_oracle_operator import gauge_transform


def wilson_weights(orc, m4):
    """One layer, 1 -> 1 channel, whose output is D_W psi + (m4 - 4) psi = D(c_sw=0) psi."""
    g = orc.gamma()
    W = np.zeros((9, 1, 1, 4, 4), complex)
    W[0, 0, 0] = m4 * np.eye(4)
    for mu in range(4):
        W[1 + 2 * mu, 0, 0] = -0.5 * (np.eye(4) - g[mu])
        W[2 + 2 * mu, 0, 0] = -0.5 * (np.eye(4) + g[mu])
    return W.reshape(-1)


@pytest.mark.parametrize("bc", [-1, 1])
def test_net_layer_reproduces_wilson_operator(orc, bc):
    L = (4, 4, 4, 6)
    V = int(np.prod(L))
    U = S.random_su3_links(L, 0.5, 61)
    A, _ = orc.clover(L, U, 0.13, 0.0)
    psi = S.gaussian_field(V, 62)
    out = orc.net_layer_forward(L, U, 1, 1, wilson_weights(orc, 1 / 0.26), psi[None], bc=bc)[0]
    ref = orc.apply_D(L, U, A, psi, bc=bc)
    assert np.abs(out - ref).max() < 1e-13


def test_net_gauge_covariance(orc):
    L = (4, 4, 4, 4)
    V = 256
    U = S.random_su3_links(L, 0.6, 71)
    Lam = S.random_gauge_transform(L, 72)
    Ut = gauge_transform(U, Lam, L)
    ch = [1, 3, 2, 1]
    W = S.random_weights(orc.net_nweights(ch), 73, 0.3)
    r = S.gaussian_field(V, 74)
    out = orc.net_forward(L, U, ch, W, r[None])[0]
    outt = orc.net_forward(L, Ut, ch, W, np.einsum("xab,xsb->xsa", Lam, r)[None])[0]
    assert np.abs(outt - np.einsum("xab,xsb->xsa", Lam, out)).max() < 1e-12


def test_net_layer_backward_is_exact_adjoint(orc):
    # <gy, layer(x)> = <layer^dag gy, x> for the input gradient, and the weight
    # gradient contracts to the same number: sum conj(gW) W = <gy, layer(x)>
    L = (4, 4, 2, 4)
    V = int(np.prod(L))
    U = S.random_su3_links(L, 0.5, 81)
    cin, cout = 2, 3
    W = S.random_weights(9 * cin * cout * 16, 82, 0.5)
    x = S.gaussian_field(V, 83, nrhs=cin)
    gy = S.gaussian_field(V, 84, nrhs=cout)
    y = orc.net_layer_forward(L, U, cin, cout, W, x)
    gx, gW = orc.net_layer_backward(L, U, cin, cout, W, x, gy)
    lhs = np.vdot(gy, y)
    assert abs(lhs - np.vdot(gx, x)) / abs(lhs) < 1e-13
    assert abs(lhs - np.vdot(gW, W)) / abs(lhs) < 1e-13


def test_net_loss_gradient_finite_differences(orc):
    L = (2, 2, 2, 4)
    V = int(np.prod(L))
    U = S.random_su3_links(L, 0.6, 91)
    ch = [1, 2, 2, 1]
    W = S.random_weights(orc.net_nweights(ch), 92, 0.3)
    r = S.gaussian_field(V, 93, nrhs=3)
    e = S.gaussian_field(V, 94, nrhs=3)
    loss, grad = orc.net_loss_grad(L, U, ch, W, r, e)
    rng = np.random.default_rng(95)
    h = 1e-5
    for k in rng.choice(len(W), 12, replace=False):
        for part in (1.0, 1j):
            Wp, Wm = W.copy(), W.copy()
            Wp[k] += h * part
            Wm[k] -= h * part
            fd = (orc.net_loss_grad(L, U, ch, Wp, r, e, with_grad=False)[0]
                  - orc.net_loss_grad(L, U, ch, Wm, r, e, with_grad=False)[0]) / (2 * h)
            an = grad[k].real if part == 1.0 else grad[k].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, part, fd, an)


def test_net_loss_is_scale_invariant_and_zero_at_exact_inverse(orc):
    # with W = 0 the network outputs zero, so the loss is exactly 1
    L = (2, 2, 2, 2)
    V = 16
    U = S.random_su3_links(L, 0.5, 96)
    ch = [1, 2, 1]
    W = np.zeros(orc.net_nweights(ch), complex)
    r = S.gaussian_field(V, 97, nrhs=2)
    e = S.gaussian_field(V, 98, nrhs=2)
    loss, _ = orc.net_loss_grad(L, U, ch, W, r, e, with_grad=False)
    assert abs(loss - 1.0) < 1e-14
    loss2, _ = orc.net_loss_grad(L, U, ch, W, 7.0 * r, 7.0 * e, with_grad=False)
    assert abs(loss2 - 1.0) < 1e-14
