"""Plain FP64 CPU oracle of the clover-Wilson operator and its deflated SAP-GCR solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline timing of the benchmark may import this package; the HIP library and
its Python binding never do.  It shares no code with the HIP path.

Every array is complex128 in the canonical layouts of `paper_1011_0911_amd.synth`
(links (V,4,3,3), spinors (V,4,3), even fields (V/2,4,3) indexed by lex >> 1,
clover (V,12,12)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i = ctypes.POINTER(ctypes.c_int)
_vp = ctypes.c_void_p
_l = ctypes.POINTER(ctypes.c_int64)


def build() -> None:
    """Compile the oracle with g++ (CPU only)."""
    subprocess.check_call(["sh", os.path.join(_HERE, "build.sh")])


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        sig = {
            "orc_set_threads": (None, [ctypes.c_int]),
            "orc_get_threads": (ctypes.c_int, []),
            "orc_clover": (ctypes.c_int64, [_i, ctypes.c_int, _d, ctypes.c_double, ctypes.c_double, _d, _d]),
            "orc_field_strength": (None, [_i, ctypes.c_int, _d, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _d]),
            "orc_gamma": (None, [_d]),
            "orc_apply_D": (None, [_i, ctypes.c_int, _d, _d, _d, _d]),
            "orc_apply_Dhat": (None, [_i, ctypes.c_int, _d, _d, _d, _d, _d]),
            "orc_sap": (None, [_i, ctypes.c_int, _d, _d, _d, _i, ctypes.c_int, ctypes.c_int, _d, _d]),
            "orc_sap_half_sweep": (None, [_i, ctypes.c_int, _d, _d, _d, _i, ctypes.c_int, ctypes.c_int, _d, _d, _d]),
            "orc_sap_one_cycle_on_blocks": (ctypes.c_int, [_i, ctypes.c_int, _d, _d, _d, _i, ctypes.c_int, _d, _l,
                                                           ctypes.c_int, _d]),
            "orc_dfl_set_fields_on_blocks": (None, [_vp, _d, _d, _d, _l, ctypes.c_int]),
            "orc_net_forward_on_sites": (None, [_i, ctypes.c_int, _d, ctypes.c_int, _i, _d, _d, _l, ctypes.c_int,
                                                _d]),
            "orc_dfl_new": (_vp, [_i, ctypes.c_int, _i, ctypes.c_int]),
            "orc_dfl_free": (None, [_vp]),
            "orc_dfl_nblocks": (ctypes.c_int64, [_vp]),
            "orc_dfl_build": (None, [_vp, _d, _d, _d, _i, ctypes.c_int, ctypes.c_int, ctypes.c_int, _d]),
            "orc_dfl_set_fields": (None, [_vp, _d, _d, _d]),
            "orc_dfl_get_basis": (None, [_vp, _d]),
            "orc_dfl_get_little": (None, [_vp, _d]),
            "orc_dfl_restrict": (None, [_vp, _d, _d]),
            "orc_dfl_prolong": (None, [_vp, _d, _d]),
            "orc_dfl_coarse_apply": (None, [_vp, _d, _d]),
            "orc_dfl_coarse_solve": (ctypes.c_int, [_vp, _d, _d, ctypes.c_double]),
            "orc_dfl_precond": (None, [_vp, _d, _d, _d, _i, ctypes.c_int, ctypes.c_int, ctypes.c_double, _d, _d]),
            "orc_dfl_net_precond": (ctypes.c_int, [_vp, _d, _d, _d, _i, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                   ctypes.c_int, _i, _d, _d, _d]),
            "orc_fgcr": (ctypes.c_int, [_i, ctypes.c_int, _d, _d, _d, ctypes.c_int, ctypes.c_int, _i, ctypes.c_int,
                                        ctypes.c_int, _vp, ctypes.c_double, ctypes.c_int, _i, _d, _d, _d,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_double, _i, _d, _d, ctypes.c_int, _i]),
            "orc_block_bicgstab": (None, [_i, ctypes.c_int, _d, _d, _d, _i, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_int64, _d, _d, ctypes.c_double, ctypes.c_int, _i,
                                          ctypes.POINTER(ctypes.c_double)]),
            "orc_clover_force": (None, [_i, ctypes.c_int, _d, ctypes.c_double, _d, _d]),
            "orc_hop_force": (None, [_i, ctypes.c_int, _d, _d, _d, ctypes.c_double, _d]),
            "orc_hop_adj": (None, [_i, ctypes.c_int, _d, _d, _d]),
            "orc_force_components": (None, [ctypes.c_int64, _d, ctypes.POINTER(ctypes.c_double)]),
            "orc_net_layer_forward": (None, [_i, ctypes.c_int, _d, ctypes.c_int, ctypes.c_int, _d, _d, _d]),
            "orc_net_layer_backward": (None, [_i, ctypes.c_int, _d, ctypes.c_int, ctypes.c_int, _d, _d, _d, _d, _d]),
            "orc_net_forward": (None, [_i, ctypes.c_int, _d, ctypes.c_int, _i, _d, _d, _d]),
            "orc_net_loss_grad": (ctypes.c_double, [_i, ctypes.c_int, _d, ctypes.c_int, _i, _d, ctypes.c_int, _d, _d, _d]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _c(a: np.ndarray):
    assert a.dtype == np.complex128 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(_d)


def _lvec(v):
    return (ctypes.c_int64 * len(v))(*[int(x) for x in v])


def _ivec(v):
    arr = (ctypes.c_int * len(v))(*[int(x) for x in v])
    return arr


def _cc(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def gamma() -> np.ndarray:
    """gamma_0..gamma_3 and gamma_5 of the oracle's basis, shape (5,4,4)."""
    out = np.zeros((5, 4, 4), np.complex128)
    lib().orc_gamma(_c(out))
    return out


def clover(L, U, kappa, csw, bc=-1):
    """A(x) (12x12 per site, Eq. 1 diagonal part) and its inverse."""
    U = _cc(U)
    V = U.shape[0]
    A = np.zeros((V, 12, 12), np.complex128)
    Ai = np.zeros((V, 12, 12), np.complex128)
    nbad = lib().orc_clover(_ivec(L), bc, _c(U), kappa, csw, _c(A), _c(Ai))
    if nbad:
        raise ArithmeticError(f"{nbad} singular clover blocks")
    return A, Ai


def field_strength(L, U, x, mu, nu, bc=-1):
    F = np.zeros((3, 3), np.complex128)
    lib().orc_field_strength(_ivec(L), bc, _c(_cc(U)), int(x), mu, nu, _c(F))
    return F


def apply_D(L, U, A, psi, bc=-1):
    psi = _cc(psi)
    out = np.zeros_like(psi)
    lib().orc_apply_D(_ivec(L), bc, _c(_cc(U)), _c(_cc(A)), _c(psi), _c(out))
    return out


def apply_Dhat(L, U, A, Ai, pe, bc=-1):
    pe = _cc(pe)
    out = np.zeros_like(pe)
    lib().orc_apply_Dhat(_ivec(L), bc, _c(_cc(U)), _c(_cc(A)), _c(_cc(Ai)), _c(pe), _c(out))
    return out


def sap(L, U, A, Ai, eta, bs, ncy, nmr, bc=-1):
    eta = _cc(eta)
    out = np.zeros_like(eta)
    lib().orc_sap(_ivec(L), bc, _c(_cc(U)), _c(_cc(A)), _c(_cc(Ai)), _ivec(bs), ncy, nmr, _c(eta), _c(out))
    return out


def sap_half_sweep(L, U, A, Ai, bs, nmr, col, eta, psi, rho, bc=-1):
    """In place on copies: returns (psi, rho) after one colour half-sweep."""
    psi = _cc(psi).copy()
    rho = _cc(rho).copy()
    lib().orc_sap_half_sweep(_ivec(L), bc, _c(_cc(U)), _c(_cc(A)), _c(_cc(Ai)), _ivec(bs), nmr, col,
                             _c(_cc(eta)), _c(psi), _c(rho))
    return psi, rho


def sap_one_cycle_on_blocks(L, U, A, Ai, eta, bs, nmr, blocks, bc=-1):
    """One Schwarz cycle (ncy = 1) evaluated on the listed colour-1 blocks and their
    face neighbours only; equals sap(..., ncy=1, ...) there (zero elsewhere)."""
    eta = _cc(eta)
    out = np.zeros_like(eta)
    st = lib().orc_sap_one_cycle_on_blocks(_ivec(L), bc, _c(_cc(U)), _c(_cc(A)), _c(_cc(Ai)), _ivec(bs), nmr,
                                           _c(eta), _lvec(blocks), len(blocks), _c(out))
    if st != 0:
        raise ValueError("blocks must be of colour 1 with colour-0 face neighbours")
    return out


def net_forward_on_sites(L, U, ch, W, x, sites, bc=-1):
    """Network output (one channel) at the listed sites only, shape (len(sites), 4, 3)."""
    out = np.zeros((len(sites), 4, 3), np.complex128)
    lib().orc_net_forward_on_sites(_ivec(L), bc, _c(_cc(U)), len(ch) - 1, _ivec(ch), _c(_cc(W)), _c(_cc(x)),
                                   _lvec(sites), len(sites), _c(out))
    return out


class Deflation:
    """Local deflation subspace + little Dirac operator (oracle)."""

    def __init__(self, L, bs, Ns, bc=-1):
        self.L = tuple(L)
        self.bc = bc
        self.Ns = Ns
        self.V = int(np.prod(L))
        self.h = lib().orc_dfl_new(_ivec(L), bc, _ivec(bs), Ns)
        self.nblk = int(lib().orc_dfl_nblocks(self.h))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_dfl_free(self.h)
            self.h = None

    def build(self, U, A, Ai, sap_bs, ncy, nmr, nit, init):
        init = _cc(init)
        assert init.shape == (self.Ns, self.V, 4, 3)
        lib().orc_dfl_build(self.h, _c(_cc(U)), _c(_cc(A)), _c(_cc(Ai)), _ivec(sap_bs), ncy, nmr, nit, _c(init))

    def set_fields(self, U, A, fields):
        lib().orc_dfl_set_fields(self.h, _c(_cc(U)), _c(_cc(A)), _c(_cc(fields)))

    def set_fields_on_blocks(self, U, A, fields, blocks):
        """set_fields restricted to the listed blocks: their basis (with their face
        neighbours') is orthonormalised and their little-operator rows computed."""
        lib().orc_dfl_set_fields_on_blocks(self.h, _c(_cc(U)), _c(_cc(A)), _c(_cc(fields)), _lvec(blocks),
                                           len(blocks))

    def basis(self):
        out = np.zeros((self.Ns, self.V, 4, 3), np.complex128)
        lib().orc_dfl_get_basis(self.h, _c(out))
        return out

    def little(self):
        out = np.zeros((self.nblk, 9, self.Ns, self.Ns), np.complex128)
        lib().orc_dfl_get_little(self.h, _c(out))
        return out

    def restrict(self, r):
        c = np.zeros((self.nblk, self.Ns), np.complex128)
        lib().orc_dfl_restrict(self.h, _c(_cc(r)), _c(c))
        return c

    def prolong(self, c):
        out = np.zeros((self.V, 4, 3), np.complex128)
        lib().orc_dfl_prolong(self.h, _c(_cc(c)), _c(out))
        return out

    def coarse_apply(self, c):
        out = np.zeros((self.nblk, self.Ns), np.complex128)
        lib().orc_dfl_coarse_apply(self.h, _c(_cc(c)), _c(out))
        return out

    def coarse_solve(self, f, tol):
        c = np.zeros((self.nblk, self.Ns), np.complex128)
        it = lib().orc_dfl_coarse_solve(self.h, _c(_cc(f)), _c(c), tol)
        return c, it

    def precond(self, U, A, Ai, sap_bs, ncy, nmr, coarse_tol, r):
        out = np.zeros((self.V, 4, 3), np.complex128)
        lib().orc_dfl_precond(self.h, _c(_cc(U)), _c(_cc(A)), _c(_cc(Ai)), _ivec(sap_bs), ncy, nmr, coarse_tol,
                              _c(_cc(r)), _c(out))
        return out

    def net_precond(self, U, A, Ai, sap_bs, ncy, nmr, coarse_tol, ch, W, r):
        """Two-level preconditioner with the network stage N (channels ch, weights W):
        returns (C r + N(r1) + M_sap(r2), fallback), r1 = r - D C r, r2 = r1 - D N(r1);
        on fallback (|r2| > |r1| or not finite) N is dropped and r2 = r1."""
        out = np.zeros((self.V, 4, 3), np.complex128)
        fb = lib().orc_dfl_net_precond(self.h, _c(_cc(U)), _c(_cc(A)), _c(_cc(Ai)), _ivec(sap_bs), ncy, nmr,
                                       coarse_tol, len(ch) - 1, _ivec(ch), _c(_cc(W)), _c(_cc(r)), _c(out))
        return out, bool(fb)


def fgcr(L, U, A, Ai, eta, *, op="D", prec="none", sap_bs=(4, 4, 4, 4), ncy=5, nmr=4, dfl=None,
         coarse_tol=1e-12, net=None, nkv=16, nmx=2048, tol=1e-10, nhist=0, bc=-1):
    """Flexible GCR on D (op='D') or Dhat (op='Dhat').

    prec: 'none' | 'sap' | 'dfl' (deflated SAP) | 'net' (deflated SAP + network
    stage, net = (channels, weights)).  Returns (psi, info dict)."""
    eta = _cc(eta)
    psi = np.zeros_like(eta)
    opk = {"D": 0, "Dhat": 1}[op]
    pk = {"none": 0, "sap": 1, "dfl": 2, "net": 3}[prec]
    info = (ctypes.c_int * 3)()
    relres = ctypes.c_double()
    fb = ctypes.c_int()
    hist = np.zeros(max(nhist, 1))
    ch = _ivec(net[0]) if net is not None else _ivec([1])
    nl = len(net[0]) - 1 if net is not None else 0
    w = _cc(net[1]) if net is not None else np.zeros(1, np.complex128)
    st = lib().orc_fgcr(_ivec(L), bc, _c(_cc(U)), _c(_cc(A)), _c(_cc(Ai)), opk, pk, _ivec(sap_bs), ncy, nmr,
                        dfl.h if dfl is not None else None, coarse_tol, nl, ch, _c(w), _c(eta), _c(psi),
                        nkv, nmx, tol, info, ctypes.byref(relres), hist.ctypes.data_as(_d), nhist,
                        ctypes.byref(fb))
    return psi, {"iters": info[0], "restarts": info[1], "converged": bool(info[2]), "relres": relres.value,
                 "status": st, "history": hist[: min(nhist, info[0] + 1)], "fallbacks": fb.value}


def net_layer_forward(L, U, cin, cout, W, x, bc=-1):
    x = _cc(x)
    V = int(np.prod(L))
    out = np.zeros((cout, V, 4, 3), np.complex128)
    lib().orc_net_layer_forward(_ivec(L), bc, _c(_cc(U)), cin, cout, _c(_cc(W)), _c(x), _c(out))
    return out


def net_layer_backward(L, U, cin, cout, W, x, gy, bc=-1):
    V = int(np.prod(L))
    gx = np.zeros((cin, V, 4, 3), np.complex128)
    gW = np.zeros(9 * cout * cin * 16, np.complex128)
    lib().orc_net_layer_backward(_ivec(L), bc, _c(_cc(U)), cin, cout, _c(_cc(W)), _c(_cc(x)), _c(_cc(gy)),
                                 _c(gx), _c(gW))
    return gx, gW


def net_forward(L, U, ch, W, x, bc=-1):
    V = int(np.prod(L))
    out = np.zeros((ch[-1], V, 4, 3), np.complex128)
    lib().orc_net_forward(_ivec(L), bc, _c(_cc(U)), len(ch) - 1, _ivec(ch), _c(_cc(W)), _c(_cc(x)), _c(out))
    return out


def net_nweights(ch):
    return sum(9 * ch[i] * ch[i + 1] * 16 for i in range(len(ch) - 1))


def net_loss_grad(L, U, ch, W, r, e, with_grad=True, bc=-1):
    r = _cc(r)
    e = _cc(e)
    nb = r.shape[0]
    grad = np.zeros(net_nweights(ch), np.complex128) if with_grad else None
    loss = lib().orc_net_loss_grad(_ivec(L), bc, _c(_cc(U)), len(ch) - 1, _ivec(ch), _c(_cc(W)), nb, _c(r), _c(e),
                                   _c(grad) if with_grad else None)
    return loss, grad


# ----------------------------------------------------------- mass preconditioning
# Eq. 2-5: Q = gamma5 D, its even-odd blocks Q_xy = gamma5 D_xy, the Schur
# complement Q_S = 1 - Q_ee^{-1} Q_eo Q_oo^{-1} Q_oe, W(dm) = Q_S + dm, and the
# determinant factors det Q_ee, det Q_oo.  Written from those definitions with
# the full operator of apply_D and numpy's dense solves; nothing here goes
# through the Schur-complement kernels (apply_Dhat).

def parity(L):
    """(x0 + x1 + x2 + x3) mod 2 of every site in lex order."""
    x = np.indices(tuple(int(l) for l in L)).reshape(4, -1)
    return (x.sum(0) & 1).astype(np.int64)


def _sites(L):
    """lex indices of the even and of the odd sites; the even field index of
    an even site is lex >> 1, which numbers them 0 .. V/2 - 1 in lex order."""
    par = parity(L)
    ev, od = np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]
    assert np.array_equal(ev >> 1, np.arange(ev.size)) and np.array_equal(od >> 1, np.arange(od.size))
    return ev, od


def gamma5_12():
    """gamma5 on the 12 components k = 3 spin + colour of a site."""
    return np.kron(gamma()[4], np.eye(3))


def clover_logdet(L, U, kappa, csw, bc=-1):
    """(log det Q_ee, log det Q_oo) of Eq. 2: Q_ee = gamma5 A_e is site-diagonal
    and det gamma5 = 1 on a site's 12 components, so log det Q_ee is the sum of
    log det A(x) over the even sites (likewise odd).  A(x) is Hermitian positive
    definite for these fields; a non-positive determinant raises."""
    A, _ = clover(L, U, kappa, csw, bc)
    sign, ld = np.linalg.slogdet(A)
    if np.any(np.abs(sign - 1.0) > 1e-9):
        raise ArithmeticError("clover block with a non-positive determinant")
    par = parity(L)
    return float(ld[par == 0].sum()), float(ld[par == 1].sum())


def apply_W(L, U, A, dm, pe, bc=-1):
    """W(dm) pe = Q_S pe + dm pe (Eq. 3), Q_S = 1 - Q_ee^{-1} Q_eo Q_oo^{-1} Q_oe
    (Eq. 2), on even fields pe (..., V/2, 4, 3); A: the clover of clover()."""
    pe = _cc(pe)
    lead = pe.shape[:-3]
    pe2 = pe.reshape((-1,) + pe.shape[-3:])
    V = int(np.prod(L))
    ev, od = _sites(L)
    g5 = gamma5_12()
    Qee = g5[None] @ A[ev]  # gamma5 A on the even sites
    Qoo = g5[None] @ A[od]
    out = np.empty_like(pe2)
    for r in range(pe2.shape[0]):
        full = np.zeros((V, 4, 3), np.complex128)
        full[ev] = pe2[r]
        t = apply_D(L, U, A, full, bc).reshape(V, 12)  # D_oe pe on the odd sites
        q = (g5 @ t[od].T).T                           # Q_oe pe
        q = np.linalg.solve(Qoo, q[..., None])[..., 0]  # Q_oo^{-1} Q_oe pe
        full = np.zeros((V, 4, 3), np.complex128)
        full[od] = q.reshape(-1, 4, 3)
        t = apply_D(L, U, A, full, bc).reshape(V, 12)  # D_eo (...) on the even sites
        q = (g5 @ t[ev].T).T                           # Q_eo Q_oo^{-1} Q_oe pe
        q = np.linalg.solve(Qee, q[..., None])[..., 0]
        out[r] = pe2[r] - q.reshape(-1, 4, 3) + dm * pe2[r]
    return out.reshape(lead + pe.shape[-3:])


def solve_W(L, U, A, dm, phi, tol=1e-12, bc=-1):
    """chi with W(dm) chi = phi (Eq. 3) for even fields phi (..., V/2, 4, 3): W is
    built as a dense matrix from apply_W on unit vectors and solved by LU when it
    has at most 1536 rows; larger systems use restarted GMRES (scipy) on the
    operator apply_W to relative residual tol.  dm = 0 gives Q_S^{-1} phi."""
    phi = _cc(phi)
    lead = phi.shape[:-3]
    p2 = phi.reshape((-1,) + phi.shape[-3:])
    n = p2[0].size
    out = np.empty_like(p2)
    if n <= 1536:
        eye = np.eye(n, dtype=np.complex128).reshape((n,) + p2.shape[1:])
        Wd = apply_W(L, U, A, dm, eye, bc).reshape(n, n).T
        for r in range(p2.shape[0]):
            out[r] = np.linalg.solve(Wd, p2[r].reshape(-1)).reshape(p2.shape[1:])
    else:
        from scipy.sparse.linalg import LinearOperator, gmres

        op = LinearOperator((n, n), dtype=np.complex128,
                            matvec=lambda v: apply_W(L, U, A, dm, v.reshape(p2.shape[1:]), bc).reshape(-1))
        for r in range(p2.shape[0]):
            x, info = gmres(op, p2[r].reshape(-1), rtol=tol, atol=0.0, restart=200, maxiter=50)
            if info != 0:
                raise ArithmeticError(f"GMRES on W did not reach {tol}")
            out[r] = x.reshape(p2.shape[1:])
    return out.reshape(lead + phi.shape[-3:])


def s_eff(L, U, kappa, csw, dm, phi1, phi2, tol=1e-12, bc=-1):
    """The effective action of Eq. 4 with two pseudofermion fields (even fields):
    S = -2 (log det Q_ee + log det Q_oo) + |W^{-1}(dm) phi1|^2 + |(1 + dm Q_S^{-1}) phi2|^2,
    reading the dm/Q_S of Eq. 4 as dm Q_S^{-1}.  Returns (S, (the log-det term,
    the phi1 term, the phi2 term))."""
    le, lo = clover_logdet(L, U, kappa, csw, bc)
    A, _ = clover(L, U, kappa, csw, bc)
    chi1 = solve_W(L, U, A, dm, phi1, tol, bc)
    chi2 = solve_W(L, U, A, 0.0, phi2, tol, bc)
    t0 = -2.0 * (le + lo)
    t1 = float(np.vdot(chi1, chi1).real)
    t2 = float(np.vdot(_cc(phi2) + dm * chi2, _cc(phi2) + dm * chi2).real)
    return t0 + t1 + t2, (t0, t1, t2)


def solve_W_adj(L, U, A, dm, v, tol=1e-12, bc=-1):
    """chi with W(dm)^dag chi = v for even fields v (..., V/2, 4, 3): the conjugate
    transpose of the dense W of solve_W, by LU, up to 1536 rows; larger systems
    use GMRES on W^dag x = gamma5 A_e W(gamma5 A_e^{-1} x), which is the adjoint
    because Dhat + dm A_e = A_e W is gamma5-Hermitian and A_e commutes with gamma5."""
    v = _cc(v)
    lead = v.shape[:-3]
    p2 = v.reshape((-1,) + v.shape[-3:])
    n = p2[0].size
    out = np.empty_like(p2)
    if n <= 1536:
        eye = np.eye(n, dtype=np.complex128).reshape((n,) + p2.shape[1:])
        Wd = apply_W(L, U, A, dm, eye, bc).reshape(n, n).T
        for r in range(p2.shape[0]):
            out[r] = np.linalg.solve(Wd.conj().T, p2[r].reshape(-1)).reshape(p2.shape[1:])
    else:
        from scipy.sparse.linalg import LinearOperator, gmres

        ev, _ = _sites(L)
        g5 = gamma5_12()
        Ae = A[ev]
        Aei = np.linalg.inv(Ae)

        def adj(x):
            t = (Aei @ x.reshape(-1, 12)[..., None])[..., 0] @ g5.T
            w = apply_W(L, U, A, dm, t.reshape(p2.shape[1:]), bc).reshape(-1, 12)
            return ((Ae @ w[..., None])[..., 0] @ g5.T).reshape(-1)

        op = LinearOperator((n, n), dtype=np.complex128, matvec=adj)
        for r in range(p2.shape[0]):
            x, info = gmres(op, p2[r].reshape(-1), rtol=tol, atol=0.0, restart=200, maxiter=50)
            if info != 0:
                raise ArithmeticError(f"GMRES on W^dag did not reach {tol}")
            out[r] = x.reshape(p2.shape[1:])
    return out.reshape(lead + v.shape[-3:])


# ----------------------------------------------------------- Dirichlet block solves
def block_solve(L, U, A, Ai, bs, eta, tol=1e-12, maxit=1000, blocks=None, bc=-1):
    """D_Lambda psi = eta on every block of extent bs (or on the listed blocks,
    lexicographic block index with the last direction fastest) by BiCGstab on the
    even-odd reduced block operator (the DD-HMC block inversions of Sect. 3).
    Returns (psi, iterations per listed block, |r|/|b| per listed block); psi is zero
    outside the listed blocks."""
    U, A, Ai, eta = _cc(U), _cc(A), _cc(Ai), _cc(eta)
    V = U.shape[0]
    nb = [L[i] // bs[i] for i in range(4)]
    if blocks is None:
        blocks = np.arange(int(np.prod(nb)))
    blks = np.ascontiguousarray(blocks, dtype=np.int64)
    psi = np.zeros((V, 4, 3), np.complex128)
    it = np.zeros(blks.size, np.int32)
    res = np.zeros(blks.size, np.float64)
    lib().orc_block_bicgstab(_ivec(L), bc, _c(U), _c(A), _c(Ai), _ivec(bs),
                             blks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), blks.size, _c(eta), _c(psi),
                             float(tol), int(maxit), it.ctypes.data_as(_i),
                             res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return psi, it, res


# ----------------------------------------------------------- forces
# Sect. 2: the molecular-dynamics evolution of the mass-preconditioned HMC moves
# the links with the derivatives of the effective action of Eq. 4.  A link is
# varied as U_mu(x) -> exp(eps w) U_mu(x), w traceless anti-Hermitian; the force
# component f^a is the derivative of S_eff along the generator T^a = i lambda^a/2.
#
# With D = A - H/2 (H the hopping sum), Dhat_s = Dhat + s A_e and W = A_e^{-1} Dhat_s:
#   S_1 = |W^{-1} phi1|^2, psi = W^{-1} phi1, X = Dhat_s^{-dag} psi (s = dm):
#     dS_1 = -2 Re[X^dag dDhat_s psi - X^dag dA_e phi1]
#   S_2 = |(1 + dm Q_S^{-1}) phi2|^2, xi = Q_S^{-1} phi2, v = phi2 + dm xi,
#     X = Dhat^{-dag} v: dS_2 = -2 dm Re[X^dag dDhat xi - X^dag dA_e phi2]
#   dDhat_s = (1+s) dA_e - 1/4 d(H_eo A_o^{-1} H_oe), so with Y_o = A_o^{-1} H_oe Y and
#   X_o = A_o^{-1} H_eo^dag X, a term -2c Re[X^dag dDhat_s Y - X^dag dA_e phi] is
#     -2c Re[X^dag dA_e ((1+s) Y - phi)] - c/2 Re[X_o^dag dA_o Y_o]
#     + c/2 Re[X^dag dH_eo Y_o] + c/2 Re[X_o^dag dH_oe Y]
#   S_det = -2 sum_x log det A(x): dS_det = Re sum_x tr(-2 A(x)^{-1} dA(x)).

def clover_force(L, U, csw, K, bc=-1):
    """Per-link matrices M (V, 4, 3, 3) of the quantity sum_x Re tr(K(x) A(x)),
    K (V, 12, 12) a weight per site."""
    U = _cc(U)
    M = np.zeros((U.shape[0], 4, 3, 3), np.complex128)
    lib().orc_clover_force(_ivec(L), bc, _c(U), float(csw), _c(_cc(K)), _c(M))
    return M


def hop_force(L, U, X, Y, coef, M, bc=-1):
    """Adds to M the per-link matrices of coef Re sum_x X(x)^dag (H Y)(x) (full fields)."""
    lib().orc_hop_force(_ivec(L), bc, _c(_cc(U)), _c(_cc(X)), _c(_cc(Y)), float(coef), _c(M))


def hop_adj(L, U, X, bc=-1):
    """H^dag X for a full field X (V, 4, 3)."""
    X = _cc(X)
    out = np.zeros_like(X)
    lib().orc_hop_adj(_ivec(L), bc, _c(_cc(U)), _c(X), _c(out))
    return out


def force_components(M):
    """f^a = Re tr(T^a M), T^a = i lambda^a / 2, for per-link matrices M (..., 3, 3)."""
    M = _cc(M)
    n = M.size // 9
    f = np.zeros(M.shape[:-2] + (8,), np.float64)
    lib().orc_force_components(n, _c(M), f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return f


def force(L, U, kappa, csw, dm, phi1, phi2, parts=7, tol=1e-12, bc=-1):
    """Force components f (V, 4, 8) of S_eff (Eq. 4, the terms of s_eff):
    bit 0 of parts the log-det term, bit 1 the phi1 term, bit 2 the phi2 term."""
    U = _cc(U)
    V = U.shape[0]
    A, Ai = clover(L, U, kappa, csw, bc)
    ev, od = _sites(L)
    K = np.zeros((V, 12, 12), np.complex128)
    M = np.zeros((V, 4, 3, 3), np.complex128)
    if parts & 1:
        K += -2.0 * Ai
    terms = []
    if parts & 2:
        psi = solve_W(L, U, A, dm, phi1, tol, bc)
        terms.append((1.0, dm, psi, _cc(phi1), psi))
    if parts & 4 and dm != 0:
        xi = solve_W(L, U, A, 0.0, phi2, tol, bc)
        terms.append((dm, 0.0, xi, _cc(phi2), _cc(phi2) + dm * xi))
    for c, s, Y, phi, w in terms:
        # X = Dhat_s^{-dag} w = A_e^{-1} W(s)^{-dag} w
        Xe = (Ai[ev] @ solve_W_adj(L, U, A, s, w, tol, bc).reshape(-1, 12)[..., None])[..., 0]
        Xf = np.zeros((V, 12), np.complex128)
        Yf = np.zeros((V, 12), np.complex128)
        Xf[ev], Yf[ev] = Xe, Y.reshape(-1, 12)
        # (H Y)_o = -2 (D Y)_o for Y supported on the even sites
        HY = -2.0 * apply_D(L, U, A, Yf.reshape(V, 4, 3), bc).reshape(V, 12)
        Yo = np.zeros((V, 12), np.complex128)
        Yo[od] = (Ai[od] @ HY[od][..., None])[..., 0]
        HX = hop_adj(L, U, Xf.reshape(V, 4, 3), bc).reshape(V, 12)
        Xo = np.zeros((V, 12), np.complex128)
        Xo[od] = (Ai[od] @ HX[od][..., None])[..., 0]
        Yt = (1.0 + s) * Y.reshape(-1, 12) - phi.reshape(-1, 12)
        K[ev] += -2.0 * c * Yt[:, :, None] * Xe.conj()[:, None, :]
        K[od] += -0.5 * c * Yo[od][:, :, None] * Xo[od].conj()[:, None, :]
        hop_force(L, U, Xf.reshape(V, 4, 3), Yo.reshape(V, 4, 3), 0.5 * c, M, bc)
        hop_force(L, U, Xo.reshape(V, 4, 3), Yf.reshape(V, 4, 3), 0.5 * c, M, bc)
    M += clover_force(L, U, csw, K, bc)
    return force_components(M)


# ----------------------------------------------------------- chronological inversion
# Sect. 3: the solutions of earlier inversions predict the next one (the
# chronological inversion method the paper cites).  Reading: the prediction is
# the combination of the stored solutions with the smallest residual,
# min_c |eta - D sum_i c_i psi_i|, a linear least-squares problem in the vectors
# D psi_i.

def chrono_guess(L, U, A, prev, eta, bc=-1):
    """sum_i c_i prev_i minimising |eta - D sum_i c_i prev_i| (numpy least squares
    on the columns D prev_i); prev: (k, V, 4, 3), eta: (V, 4, 3)."""
    prev = _cc(prev)
    M = np.stack([apply_D(L, U, A, p, bc).reshape(-1) for p in prev], 1)
    c = np.linalg.lstsq(M, _cc(eta).reshape(-1), rcond=None)[0]
    return np.tensordot(c, prev, 1)
