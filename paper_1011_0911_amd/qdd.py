"""Python binding of the qdd C ABI (include/qdd.h): argument marshalling only.

PyTorch provides device memory (the workspace and the fields) and the stream;
every step of the computation runs in the HIP library libqdd.so.  If the
library has not been built this module raises on load -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqdd.so")

F64, F32, F16 = 0, 1, 2
PRECOND_NONE, PRECOND_SAP, PRECOND_DFL = 0, 1, 2
KERNEL_DHAT, KERNEL_DW, KERNEL_SAP = 0, 1, 2
# candidate set of the autotuner (cached choices of an older set are re-measured)
TUNER_VERSION = "t5"

QDD_OK, QDD_EINVAL, QDD_ESTATE, QDD_ESINGULAR, QDD_ENOCONV, QDD_EHIP, QDD_ENOWS = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "QDD_OK", -1: "QDD_EINVAL", -2: "QDD_ESTATE", -3: "QDD_ESINGULAR", -4: "QDD_ENOCONV",
          -5: "QDD_EHIP", -6: "QDD_ENOWS"}


class QddError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4), ("bc_time", ctypes.c_int)]


class Config(ctypes.Structure):
    _fields_ = [
        ("max_nrhs", ctypes.c_int),
        ("sap_bs", ctypes.c_int * 4), ("ncy", ctypes.c_int), ("nmr", ctypes.c_int), ("sap_prec", ctypes.c_int),
        ("dfl_Ns", ctypes.c_int), ("dfl_bs", ctypes.c_int * 4), ("dfl_nit", ctypes.c_int),
        ("dfl_coarse_tol", ctypes.c_double), ("dfl_coarse_nmx", ctypes.c_int),
        ("nkv", ctypes.c_int), ("nmx", ctypes.c_int), ("tol", ctypes.c_double), ("precond", ctypes.c_int),
        ("use_net", ctypes.c_int), ("net_nl", ctypes.c_int), ("net_ch", ctypes.c_int * 8),
        ("net_terms", ctypes.c_int),
        ("chrono_nv", ctypes.c_int), ("dfl_refresh_iters", ctypes.c_int), ("dfl_refresh_nit", ctypes.c_int),
        ("force", ctypes.c_int),
        ("blk_bs", ctypes.c_int * 4),
    ]


class BlockInfo(ctypes.Structure):
    _fields_ = [("nblk", ctypes.c_int), ("converged", ctypes.c_int), ("breakdowns", ctypes.c_int),
                ("iters_max", ctypes.c_int), ("res_max", ctypes.c_double), ("t_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("fallbacks", ctypes.c_int), ("true_res", ctypes.c_double), ("t_ms", ctypes.c_double * 8),
                ("gpu_ms", ctypes.c_double * 4)]

    def as_dict(self):
        return {"iters": self.iters, "restarts": self.restarts, "converged": bool(self.converged),
                "fallbacks": self.fallbacks, "true_res": self.true_res, "t_ms": list(self.t_ms),
                "gpu_ms": list(self.gpu_ms)}


_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double

# exported symbol -> (restype, argtypes); the test-suite checks this list against include/qdd.h
SIGNATURES = {
    "qdd_config_default": (None, [ctypes.POINTER(Config)]),
    "qdd_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Geom), ctypes.POINTER(Config)]),
    "qdd_create": (_i, [ctypes.POINTER(Geom), ctypes.POINTER(Config), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "qdd_destroy": (None, [_vp]),
    "qdd_last_error": (ctypes.c_char_p, [_vp]),
    "qdd_set_gauge": (_i, [_vp, _vp]),
    "qdd_set_params": (_i, [_vp, _d, _d]),
    "qdd_field_bytes": (ctypes.c_size_t, [_vp, _i, _i, _i]),
    "qdd_pack_field": (_i, [_vp, _i, _i, _i, _vp, _vp]),
    "qdd_unpack_field": (_i, [_vp, _i, _i, _i, _vp, _vp]),
    "qdd_dw_hat": (_i, [_vp, _i, _i, _vp, _vp]),
    "qdd_dw_hat_static": (_i, [_vp, _i, _i, _vp, _vp]),
    "qdd_clover_logdet": (_i, [_vp, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "qdd_apply_w": (_i, [_vp, _i, _d, _vp, _vp]),
    "qdd_dw": (_i, [_vp, _i, _i, _vp, _vp]),
    "qdd_dw_masses": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "qdd_sap": (_i, [_vp, _i, _vp, _vp]),
    "qdd_dfl_build": (_i, [_vp, _vp]),
    "qdd_dfl_export": (_i, [_vp, _vp, _vp]),
    "qdd_dfl_coarse_solve": (_i, [_vp, _i, _vp, _vp, _d, ctypes.POINTER(_i)]),
    "qdd_dfl_precond": (_i, [_vp, _i, _vp, _vp]),
    "qdd_dfl_share": (_i, [_vp, _vp]),
    "qdd_solve_multi": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(_i), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                             ctypes.POINTER(_vp)]),
    "qdd_solve_group": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(_i), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                             ctypes.POINTER(_vp)]),
    "qdd_solve": (_i, [_vp, _i, _vp, _vp, _vp]),
    "qdd_solve_guess": (_i, [_vp, _i, _vp, _vp, _vp]),
    "qdd_chrono_reset": (_i, [_vp]),
    "qdd_chrono_guess": (_i, [_vp, _i, _vp, _vp]),
    "qdd_dfl_refresh": (_i, [_vp]),
    "qdd_dfl_stats": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "qdd_net_num_weights": (_i, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    "qdd_net_set_weights": (_i, [_vp, _vp]),
    "qdd_net_get_weights": (_i, [_vp, _vp]),
    "qdd_net_set_terms": (_i, [_vp, _i]),
    "qdd_net_set_calls": (_i, [_vp, _i]),
    "qdd_net_forward": (_i, [_vp, _vp, _vp]),
    "qdd_net_loss_grad": (_i, [_vp, _i, _vp, _vp, ctypes.POINTER(_d), _vp]),
    "qdd_net_train_step": (_i, [_vp, _i, _vp, _vp, ctypes.c_float, ctypes.POINTER(_d)]),
    "qdd_solve_harvest": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _i, ctypes.POINTER(_i), _vp]),
    "qdd_solve_dhat": (_i, [_vp, _i, _vp, _vp, _vp]),
    "qdd_solve_qs": (_i, [_vp, _i, _vp, _vp, _vp]),
    "qdd_solve_w": (_i, [_vp, _i, _d, _vp, _vp, _vp]),
    "qdd_action": (_i, [_vp, _d, _vp, _vp, _vp, _vp, ctypes.POINTER(_d), ctypes.POINTER(_d), _vp]),
    "qdd_force": (_i, [_vp, _d, _vp, _vp, _i, _vp, _vp]),
    "qdd_block_solve": (_i, [_vp, _i, _vp, _vp, _d, _i, _vp, _vp, _vp]),
    "qdd_set_launch": (_i, [_vp, _i, _i, _i, _i, _i, _i]),
    "qdd_get_launch": (_i, [_vp, _i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i),
                            ctypes.POINTER(_i)]),
    "qdd_dw_hat_timed": (_i, [_vp, _i, _i, _vp, _vp, _i, ctypes.POINTER(ctypes.c_float),
                              ctypes.POINTER(ctypes.c_float)]),
    "qdd_copy": (_i, [_vp, _vp, ctypes.c_size_t, _vp]),
    "qdd_autotune": (_i, [_vp, _i, _i, _i, _vp, _vp, _i, ctypes.POINTER(ctypes.c_float)]),
}


def lib():
    """Loads libqdd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1011_0911_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def default_config(**kw) -> Config:
    c = Config()
    lib().qdd_config_default(ctypes.byref(c))
    for k, v in kw.items():
        if k in ("sap_bs", "dfl_bs", "net_ch", "blk_bs"):
            arr = getattr(c, k)
            for j, x in enumerate(v):
                arr[j] = int(x)
        else:
            setattr(c, k, v)
    return c


def make_geom(L, bc=-1) -> Geom:
    g = Geom()
    for j in range(4):
        g.L[j] = int(L[j])
    g.bc_time = int(bc)
    return g


def workspace_bytes(L, cfg: Config, bc=-1) -> int:
    g = make_geom(L, bc)
    return int(lib().qdd_workspace_bytes(ctypes.byref(g), ctypes.byref(cfg)))


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One qdd context: workspace, gauge field, clover field, deflation subspace."""

    def __init__(self, L, cfg: Config | None = None, bc: int = -1, device="cuda:0", stream=None):
        self.L = tuple(int(x) for x in L)
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        self.Vh = self.V // 2
        self.cfg = cfg if cfg is not None else default_config()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        g = make_geom(self.L, bc)
        nbytes = lib().qdd_workspace_bytes(ctypes.byref(g), ctypes.byref(self.cfg))
        if nbytes == 0:
            raise QddError(QDD_EINVAL, lib().qdd_last_error(None).decode())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        st = lib().qdd_create(ctypes.byref(g), ctypes.byref(self.cfg), _ptr(self.ws), nbytes,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != QDD_OK:
            raise QddError(st, lib().qdd_last_error(None).decode())
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.qdd_destroy(self.h)
            self.h = None

    # -- helpers
    def _check(self, st):
        if st != QDD_OK:
            raise QddError(st, lib().qdd_last_error(self.h).decode())

    def _c128(self, a) -> torch.Tensor:
        t = torch.as_tensor(a)
        t = t.to(device=self.device, dtype=torch.complex128).contiguous()
        return t

    # -- set-up
    def set_gauge(self, U):
        self._U = self._c128(U)
        assert self._U.numel() == self.V * 36
        self._check(lib().qdd_set_gauge(self.h, _ptr(self._U)))

    def set_params(self, kappa: float, csw: float):
        self._check(lib().qdd_set_params(self.h, float(kappa), float(csw)))

    # -- packed fields
    def field_bytes(self, prec, nrhs, even_only):
        return int(lib().qdd_field_bytes(self.h, prec, nrhs, int(even_only)))

    def pack(self, prec, canon, even_only):
        c = self._c128(canon)
        per = (self.Vh if even_only else self.V) * 12
        nrhs = c.numel() // per
        out = torch.empty(self.field_bytes(prec, nrhs, even_only), dtype=torch.uint8, device=self.device)
        self._check(lib().qdd_pack_field(self.h, prec, nrhs, int(even_only), _ptr(c), _ptr(out)))
        return out

    def unpack(self, prec, field, nrhs, even_only):
        n = (self.Vh if even_only else self.V)
        out = torch.empty((nrhs, n, 4, 3), dtype=torch.complex128, device=self.device)
        self._check(lib().qdd_unpack_field(self.h, prec, nrhs, int(even_only), _ptr(field), _ptr(out)))
        return out

    def empty_field(self, prec, nrhs, even_only):
        return torch.empty(self.field_bytes(prec, nrhs, even_only), dtype=torch.uint8, device=self.device)

    # -- operators on packed fields
    def dw_hat(self, prec, nrhs, fin, fout):
        self._check(lib().qdd_dw_hat(self.h, prec, nrhs, _ptr(fin), _ptr(fout)))

    def dw_hat_static(self, prec, nrhs, fin, fout):
        """As dw_hat, with the odd-site intermediate in the library's static device
        scratch (no workspace use; for callers that cannot allocate)."""
        self._check(lib().qdd_dw_hat_static(self.h, prec, nrhs, _ptr(fin), _ptr(fout)))

    def clover_logdet(self):
        """(log det Q_ee, log det Q_oo) of the current operator (Eq. 2)."""
        le, lo = _d(), _d()
        self._check(lib().qdd_clover_logdet(self.h, ctypes.byref(le), ctypes.byref(lo)))
        return le.value, lo.value

    def apply_w_packed(self, nrhs, dm, fin, fout):
        """fout = W(dm) fin = Q_S fin + dm fin (Eq. 3) on packed FP64 even fields."""
        self._check(lib().qdd_apply_w(self.h, nrhs, float(dm), _ptr(fin), _ptr(fout)))

    def apply_w(self, dm, psi_e):
        """W(dm) on canonical even fields (pack, apply, unpack)."""
        c = self._c128(psi_e)
        nrhs = c.numel() // (self.Vh * 12)
        fi = self.pack(F64, c, True)
        fo = self.empty_field(F64, nrhs, True)
        self.apply_w_packed(nrhs, dm, fi, fo)
        return self.unpack(F64, fo, nrhs, True)

    def dw(self, prec, nrhs, fin, fout):
        self._check(lib().qdd_dw(self.h, prec, nrhs, _ptr(fin), _ptr(fout)))

    # -- canonical convenience wrappers (pack -> apply -> unpack)
    def apply_dhat(self, psi_e, prec=F64):
        c = self._c128(psi_e)
        nrhs = c.numel() // (self.Vh * 12)
        fi = self.pack(prec, c, True)
        fo = self.empty_field(prec, nrhs, True)
        self.dw_hat(prec, nrhs, fi, fo)
        return self.unpack(prec, fo, nrhs, True)

    def dw_masses(self, prec, nrhs, kappas, fin, fout):
        """out_r = D(kappas[r]) in_r on packed full fields, one launch."""
        k = (ctypes.c_double * nrhs)(*[float(v) for v in kappas])
        self._check(lib().qdd_dw_masses(self.h, prec, nrhs, ctypes.cast(k, ctypes.c_void_p), _ptr(fin), _ptr(fout)))

    def apply_dw_masses(self, psi, kappas, prec=F64):
        c = self._c128(psi)
        nrhs = c.numel() // (self.V * 12)
        fi = self.pack(prec, c, False)
        fo = self.empty_field(prec, nrhs, False)
        self.dw_masses(prec, nrhs, kappas, fi, fo)
        return self.unpack(prec, fo, nrhs, False)

    def apply_dw(self, psi, prec=F64):
        c = self._c128(psi)
        nrhs = c.numel() // (self.V * 12)
        fi = self.pack(prec, c, False)
        fo = self.empty_field(prec, nrhs, False)
        self.dw(prec, nrhs, fi, fo)
        return self.unpack(prec, fo, nrhs, False)

    # -- solver
    def sap(self, eta):
        c = self._c128(eta)
        nrhs = c.numel() // (self.V * 12)
        out = torch.empty((nrhs, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        self._check(lib().qdd_sap(self.h, nrhs, _ptr(c), _ptr(out)))
        return out

    def dfl_build(self, init):
        c = self._c128(init)
        assert c.numel() == self.cfg.dfl_Ns * self.V * 12
        self._check(lib().qdd_dfl_build(self.h, _ptr(c)))

    def dfl_nblocks(self):
        n = 1
        for j in range(4):
            n *= self.L[j] // self.cfg.dfl_bs[j]
        return n

    def dfl_export(self):
        """(basis (Ns,V,4,3), little operator (nblk,9,Ns,Ns)) as device complex128 tensors."""
        Ns = self.cfg.dfl_Ns
        basis = torch.empty((Ns, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        little = torch.empty((self.dfl_nblocks(), 9, Ns, Ns), dtype=torch.complex128, device=self.device)
        self._check(lib().qdd_dfl_export(self.h, _ptr(basis), _ptr(little)))
        return basis, little

    def dfl_share(self, src: "Context"):
        self._check(lib().qdd_dfl_share(self.h, src.h))

    def dfl_coarse_solve(self, f, tol):
        c_in = self._c128(f)
        nrhs = c_in.numel() // (self.dfl_nblocks() * self.cfg.dfl_Ns)
        out = torch.empty_like(c_in)
        it = ctypes.c_int()
        self._check(lib().qdd_dfl_coarse_solve(self.h, nrhs, _ptr(c_in), _ptr(out), float(tol), ctypes.byref(it)))
        return out, it.value

    def dfl_precond(self, r):
        c = self._c128(r)
        nrhs = c.numel() // (self.V * 12)
        out = torch.empty((nrhs, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        self._check(lib().qdd_dfl_precond(self.h, nrhs, _ptr(c), _ptr(out)))
        return out

    def solve(self, eta, check=True):
        c = self._c128(eta)
        nrhs = c.numel() // (self.V * 12)
        out = torch.empty((nrhs, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        info = (SolveInfo * nrhs)()
        st = lib().qdd_solve(self.h, nrhs, _ptr(c), _ptr(out), info)
        if check:
            self._check(st)
        return out, [i.as_dict() for i in info], st

    def solve_guess(self, eta, guess, check=True):
        """Solve starting from the initial guess (canonical full fields)."""
        c = self._c128(eta)
        nrhs = c.numel() // (self.V * 12)
        out = self._c128(guess).clone().reshape(nrhs, self.V, 4, 3)
        info = (SolveInfo * nrhs)()
        st = lib().qdd_solve_guess(self.h, nrhs, _ptr(c), _ptr(out), info)
        if check:
            self._check(st)
        return out, [i.as_dict() for i in info], st

    def chrono_guess(self, eta):
        c = self._c128(eta)
        nrhs = c.numel() // (self.V * 12)
        out = torch.empty((nrhs, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        self._check(lib().qdd_chrono_guess(self.h, nrhs, _ptr(c), _ptr(out)))
        return out

    def chrono_reset(self):
        self._check(lib().qdd_chrono_reset(self.h))

    def dfl_refresh(self):
        self._check(lib().qdd_dfl_refresh(self.h))

    def dfl_stats(self):
        b, r = ctypes.c_int(), ctypes.c_int()
        self._check(lib().qdd_dfl_stats(self.h, ctypes.byref(b), ctypes.byref(r)))
        return b.value, r.value

    def solve_qs(self, phi_e, check=True):
        """Q_S^{-1} phi_e (Eq. 5) on canonical even fields through the configured solver."""
        c = self._c128(phi_e)
        nrhs = c.numel() // (self.Vh * 12)
        out = torch.empty((nrhs, self.Vh, 4, 3), dtype=torch.complex128, device=self.device)
        info = (SolveInfo * nrhs)()
        st = lib().qdd_solve_qs(self.h, nrhs, _ptr(c), _ptr(out), info)
        if check:
            self._check(st)
        return out, [i.as_dict() for i in info], st

    def solve_w(self, dm, phi_e, check=True):
        """W(dm)^{-1} phi_e (Eq. 3) on canonical even fields; info carries the W residual."""
        c = self._c128(phi_e)
        nrhs = c.numel() // (self.Vh * 12)
        out = torch.empty((nrhs, self.Vh, 4, 3), dtype=torch.complex128, device=self.device)
        info = (SolveInfo * nrhs)()
        st = lib().qdd_solve_w(self.h, nrhs, float(dm), _ptr(c), _ptr(out), info)
        if check:
            self._check(st)
        return out, [i.as_dict() for i in info], st

    def action(self, dm, phi1, phi2):
        """S_eff of Eq. 4: returns (S, (log-det term, phi1 term, phi2 term), chi1 =
        W^{-1}(dm) phi1, chi2 = Q_S^{-1} phi2, infos of the two solves)."""
        p1, p2 = self._c128(phi1), self._c128(phi2)
        assert p1.numel() == p2.numel() == self.Vh * 12
        c1 = torch.empty((self.Vh, 4, 3), dtype=torch.complex128, device=self.device)
        c2 = torch.empty_like(c1)
        s = _d()
        parts = (_d * 3)()
        info = (SolveInfo * 2)()
        self._check(lib().qdd_action(self.h, float(dm), _ptr(p1), _ptr(p2), _ptr(c1), _ptr(c2), ctypes.byref(s),
                                     parts, info))
        return s.value, tuple(parts), c1, c2, [i.as_dict() for i in info]

    def force(self, dm, phi1, phi2, terms=7):
        """Link derivatives of S_eff (Eq. 4, as action()): f (V, 4, 8) float64, f[lex, mu, a]
        along T^a = i lambda^a / 2; terms: bit 0 log-det, bit 1 phi1, bit 2 phi2 term.
        Returns (f, infos of the four solves)."""
        p1, p2 = self._c128(phi1), self._c128(phi2)
        assert p1.numel() == p2.numel() == self.Vh * 12
        f = torch.empty((self.V, 4, 8), dtype=torch.float64, device=self.device)
        info = (SolveInfo * 4)()
        self._check(lib().qdd_force(self.h, float(dm), _ptr(p1), _ptr(p2), int(terms), _ptr(f), info))
        return f, [i.as_dict() for i in info]

    def block_solve(self, eta, tol=1e-10, maxit=1000, check=True):
        """Dirichlet block solves D_Lambda psi = eta on every block of extent
        config.blk_bs (BiCGstab on each block): returns (psi (nrhs, V, 4, 3), iterations
        (nrhs, nblk), |r|/|b| (nrhs, nblk), summary dict, status)."""
        c = self._c128(eta)
        nrhs = c.numel() // (self.V * 12)
        nblk = 1
        for j in range(4):  # (no block extents: the library rejects the call)
            nblk *= self.L[j] // self.cfg.blk_bs[j] if self.cfg.blk_bs[j] else 1
        out = torch.empty((nrhs, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        it = (ctypes.c_int * (nrhs * nblk))()
        res = (ctypes.c_double * (nrhs * nblk))()
        info = BlockInfo()
        st = lib().qdd_block_solve(self.h, nrhs, _ptr(c), _ptr(out), float(tol), int(maxit), it, res,
                                   ctypes.byref(info))
        if check:
            self._check(st)
        return (out, torch.tensor(it[:], dtype=torch.int32).reshape(nrhs, nblk),
                torch.tensor(res[:], dtype=torch.float64).reshape(nrhs, nblk), info.as_dict(), st)

    def solve_dhat(self, eta_e, check=True):
        c = self._c128(eta_e)
        nrhs = c.numel() // (self.Vh * 12)
        out = torch.empty((nrhs, self.Vh, 4, 3), dtype=torch.complex128, device=self.device)
        info = (SolveInfo * nrhs)()
        st = lib().qdd_solve_dhat(self.h, nrhs, _ptr(c), _ptr(out), info)
        if check:
            self._check(st)
        return out, [i.as_dict() for i in info], st

    # -- learned stage
    def net_num_weights(self):
        n = ctypes.c_int64()
        self._check(lib().qdd_net_num_weights(self.h, ctypes.byref(n)))
        return n.value

    def net_set_weights(self, w):
        """w: complex weights (numpy or torch), stored as FP32 complex."""
        t = torch.as_tensor(w).to(device=self.device, dtype=torch.complex64).contiguous()
        assert t.numel() == self.net_num_weights()
        self._check(lib().qdd_net_set_weights(self.h, _ptr(t)))

    def net_set_terms(self, terms: int):
        """BF16 terms per activation in later network applications (3 exact, 2, 1)."""
        self._check(lib().qdd_net_set_terms(self.h, int(terms)))

    def net_set_calls(self, calls: int):
        """Network stage only in the first `calls` preconditioner applications of
        each solve (0 = every application)."""
        self._check(lib().qdd_net_set_calls(self.h, int(calls)))

    def net_get_weights(self):
        t = torch.empty(self.net_num_weights(), dtype=torch.complex64, device=self.device)
        self._check(lib().qdd_net_get_weights(self.h, _ptr(t)))
        return t

    def net_forward(self, x):
        c = self._c128(x)
        out = torch.empty((self.V, 4, 3), dtype=torch.complex128, device=self.device)
        self._check(lib().qdd_net_forward(self.h, _ptr(c), _ptr(out)))
        return out

    def net_loss_grad(self, r, e, with_grad=True):
        rc, ec = self._c128(r), self._c128(e)
        nb = rc.numel() // (self.V * 12)
        loss = ctypes.c_double()
        g = torch.empty(self.net_num_weights(), dtype=torch.complex64, device=self.device) if with_grad else None
        self._check(lib().qdd_net_loss_grad(self.h, nb, _ptr(rc), _ptr(ec), ctypes.byref(loss),
                                            _ptr(g) if g is not None else None))
        return loss.value, g

    def net_train_step(self, r_pairs, e_pairs, nb, lr):
        loss = ctypes.c_double()
        self._check(lib().qdd_net_train_step(self.h, nb, _ptr(r_pairs), _ptr(e_pairs), float(lr), ctypes.byref(loss)))
        return loss.value

    def pair_buffers(self, n):
        """Device buffers for n (residual, error) pairs: packed FP32 full fields (the
        error buffer has FP64-sized slots for the harvest; its FP32 pairs sit at the front)."""
        return (torch.empty(n * self.field_bytes(F32, 1, False), dtype=torch.uint8, device=self.device),
                torch.empty(n * self.field_bytes(F64, 1, False), dtype=torch.uint8, device=self.device))

    def solve_harvest(self, eta, rbuf, ebuf, max_pairs, check=True):
        """Solves the right-hand sides of eta (one field or a batch) and records the
        (residual, error) pairs of their outer iterations.  Returns
        (psi, infos, npairs, pair_rhs)."""
        c = self._c128(eta)
        m = c.numel() // (self.V * 12)
        out = torch.empty((m, self.V, 4, 3), dtype=torch.complex128, device=self.device)
        info = (SolveInfo * m)()
        npairs = ctypes.c_int()
        rhs = (ctypes.c_int * int(max_pairs))()
        st = lib().qdd_solve_harvest(self.h, m, _ptr(c), _ptr(out), info, _ptr(rbuf), _ptr(ebuf), int(max_pairs),
                                     ctypes.byref(npairs), ctypes.cast(rhs, ctypes.c_void_p))
        if check:
            self._check(st)
        return out, [i.as_dict() for i in info], npairs.value, list(rhs[:npairs.value])

    def set_launch(self, kernel, prec, block, nr, xcd, sb=0):
        self._check(lib().qdd_set_launch(self.h, kernel, prec, block, nr, xcd, sb))

    def get_launch(self, kernel, prec):
        b, n, x, s = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(lib().qdd_get_launch(self.h, kernel, prec, ctypes.byref(b), ctypes.byref(n), ctypes.byref(x),
                                         ctypes.byref(s)))
        return b.value, n.value, x.value, s.value

    def autotune(self, kernel, prec, nrhs, fin, fout, reps=5, cache=None):
        """Picks the fastest launch shape (C++ timing loop in the library).  With a
        cache dict, a previously measured choice for the same key is reused."""
        key = (f"{TUNER_VERSION}/{kernel}/{prec}/{nrhs}/{'x'.join(map(str, self.L))}/"
               f"{torch.cuda.get_device_properties(self.device).gcnArchName}")
        if kernel == KERNEL_SAP:  # the variants' relative cost depends on the block and the MR steps
            key += f"/bs{'x'.join(str(b) for b in self.cfg.sap_bs)}/nmr{self.cfg.nmr}"
        if cache is not None and key in cache:
            b, n, x, s = cache[key]["launch"]
            self.set_launch(kernel, prec, b, n, x, s)
            return cache[key]["ms"]
        ms = ctypes.c_float()
        self._check(lib().qdd_autotune(self.h, kernel, prec, nrhs, _ptr(fin), _ptr(fout), int(reps), ctypes.byref(ms)))
        if cache is not None:
            cache[key] = {"launch": list(self.get_launch(kernel, prec)), "ms": ms.value}
        return ms.value

    def tune_sap(self, nrhs, reps=2, cache=None):
        """Picks the fastest Schwarz half-sweep kernel variant for the configured SAP
        precision and a batch of nrhs (timed on whole preconditioner calls with
        Gaussian sources).  Returns the mean duration of the fastest (ms), or None
        for FP64, which has a single kernel."""
        if self.cfg.sap_prec == F64:
            return None
        g = torch.Generator(device=self.device)
        g.manual_seed(9000)
        eta = torch.randn((nrhs, self.V, 12, 2), dtype=torch.float64, device=self.device, generator=g)
        fin = self.pack(F64, torch.view_as_complex(eta), False)
        fout = self.empty_field(F32, nrhs, False)
        return self.autotune(KERNEL_SAP, self.cfg.sap_prec, nrhs, fin, fout, reps=reps, cache=cache)

    def dw_hat_timed(self, prec, nrhs, fin, fout, reps):
        """Mean per-pass durations (ms) of `reps` Dhat applies, HIP events on the context stream."""
        a, b = ctypes.c_float(), ctypes.c_float()
        self._check(lib().qdd_dw_hat_timed(self.h, prec, nrhs, _ptr(fin), _ptr(fout), int(reps), ctypes.byref(a),
                                           ctypes.byref(b)))
        return a.value, b.value


def solve_multi(ctxs, etas):
    """Solves several systems concurrently (each context needs its own stream).
    Returns (psis, infos, status)."""
    return _solve_systems("qdd_solve_multi", ctxs, etas)


def solve_group(ctxs, etas):
    """Solves several systems with one launch per solver stage over all of them
    (qdd_solve_group; all on the stream of ctxs[0]).  Returns (psis, infos, status)."""
    return _solve_systems("qdd_solve_group", ctxs, etas)


def _solve_systems(entry, ctxs, etas):
    n = len(ctxs)
    H = (ctypes.c_void_p * n)(*[c.h for c in ctxs])
    nr = (ctypes.c_int * n)()
    E = (ctypes.c_void_p * n)()
    P = (ctypes.c_void_p * n)()
    I = (ctypes.c_void_p * n)()
    keep, psis, infos = [], [], []
    for k, (c, eta) in enumerate(zip(ctxs, etas)):
        t = c._c128(eta)
        m = t.numel() // (c.V * 12)
        out = torch.empty((m, c.V, 4, 3), dtype=torch.complex128, device=c.device)
        inf = (SolveInfo * m)()
        keep.append(t)
        psis.append(out)
        infos.append(inf)
        nr[k] = m
        E[k] = t.data_ptr()
        P[k] = out.data_ptr()
        I[k] = ctypes.cast(inf, ctypes.c_void_p)
    for c in ctxs:
        torch.cuda.current_stream(c.device).synchronize()
    st = getattr(lib(), entry)(H, n, nr, E, P, I)
    return psis, [[i.as_dict() for i in inf] for inf in infos], st


def load_tune_cache(path):
    import json

    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_tune_cache(path, cache):
    import json

    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    """HBM copy reference kernel (16-byte vectors) on `stream` (default: current)."""
    st = stream if stream is not None else torch.cuda.current_stream(dst.device)
    nbytes = min(dst.numel() * dst.element_size(), src.numel() * src.element_size())
    r = lib().qdd_copy(_ptr(dst), _ptr(src), nbytes - nbytes % 16, ctypes.c_void_p(st.cuda_stream))
    if r != QDD_OK:
        raise QddError(r, "qdd_copy failed")
