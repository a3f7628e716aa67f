// Preconditioners of the outer FGCR: identity, Schwarz (SAP) and the two-level
// deflated SAP, each applied to a whole right-hand-side batch.
#include "qdd_solver.h"
#include "qdd_sap.h"
#include "qdd_dfl.h"

#include <algorithm>
#include <string>
#include <vector>

using namespace qdd;

// full-field views of the SAP buffers
template <class S>
static FieldV<S> full_view(const qdd_ctx* x, size_t off, float* scale) {
  int64_t n = x->G.Vh;
  return FieldV<S>{x->ptr<typename St<S>::E>(off), scale, 24 * n, 2 * n, (int)n};
}
// the same memory seen as 2*nrhs parity vectors (for element-wise conversions)
template <class S>
static FieldV<S> vec_view(const qdd_ctx* x, const void* p, float* scale) {
  int64_t n = x->G.Vh;
  return FieldV<S>{(typename St<S>::E*)p, scale, 12 * n, n, (int)n};
}

// arguments of the half-sweeps of one context (colour and cycle flags unset)
template <class S, class P>
static SapArgs<S, P> sap_args(const qdd_ctx* x, int nrhs, typename St<P>::E* psi, int* nblk_out) {
  const Layout& lo = x->lo;
  const qdd_config& c = x->cfg;
  int64_t Vh = x->G.Vh;
  float* sc = x->ptr<float>(lo.s_scale);
  float* rho_sc = sizeof(S) == 2 ? sc : nullptr;
  float* v_sc = sizeof(S) == 2 ? sc + (size_t)c.max_nrhs * 2 * Vh : nullptr;
  SapArgs<S, P> a;
  a.g = x->G;
  int nblk = 1;
  for (int m = 0; m < 4; ++m) {
    a.bs[m] = c.sap_bs[m];
    a.nb[m] = x->G.L[m] / c.sap_bs[m];
    nblk *= a.nb[m];
  }
  a.nrhs = nrhs;
  a.nmr = c.nmr;
  a.variant = x->sap_variant[c.sap_prec];
  DevOp<S> op = x->op<S>();
  a.U = op.U;
  a.A = op.A;
  a.Ai = op.Ainv;
  a.rho = full_view<S>(x, lo.s_rho, rho_sc);
  a.V = full_view<S>(x, lo.s_v, v_sc);
  a.psi = FieldV<P>{psi, nullptr, 24 * Vh, 2 * Vh, (int)Vh};
  a.poff = 12 * Vh;
  a.spoff = Vh;
  a.col = a.first = a.do_bnd = a.write_v = 0;
  *nblk_out = nblk;
  return a;
}

// psi (P storage, full fields, rhs stride 24 Vh) = M_sap eta (FP64 internal full fields)
template <class S, class P>
static qdd_status sap_run(qdd_ctx* x, int nrhs, const double2* eta, typename St<P>::E* psi) {
  const qdd_config& c = x->cfg;
  int nblk = 1;
  SapArgs<S, P> a = sap_args<S, P>(x, nrhs, psi, &nblk);
  HCK(x, launch_field_convert<double, S>(vec_view<double>(x, eta, nullptr), vec_view<S>(x, a.rho.p, a.rho.scale),
                                          2 * nrhs, x->st));
  for (int cy = 0; cy < c.ncy; ++cy)
    for (int col = 0; col < 2; ++col) {
      a.col = col;
      a.first = cy == 0;
      a.do_bnd = !(cy == 0 && col == 0);
      a.write_v = !(cy == c.ncy - 1 && col == 1);
      // the face corrections by a coalesced kernel of their own (1-2 % faster than
      // inside the half-sweep, which then skips them)
      if (a.do_bnd) {
        HCK(x, launch_sap_face<S, P>(a, x->st));
        a.do_bnd = 0;
      }
      HCK(x, launch_sap_half<S, P>(a, nblk / 2, x->st));
    }
  return QDD_OK;
}

// the same for ns systems with FP32 or FP16 storage (psi FP32), every step one
// launch over the systems that still take part in it (systems may differ in
// lattice, mass, batch size, block shape of equal volume and cycle count)
template <class S>
static qdd_status sap_grp_run(qdd_ctx* const* xs, const int* nrhs, const double2* const* eta, void* const* psi,
                              int ns, hipStream_t st) {
  qdd_ctx* x0 = xs[0];
  std::vector<SapArgs<S, float>> a(ns), sel;
  std::vector<FieldV<double>> cin(ns);
  std::vector<FieldV<S>> cvo(ns);
  std::vector<int> nvec(ns);
  int ncy = 0;
  for (int s = 0; s < ns; ++s) {
    int nblk = 0;
    a[s] = sap_args<S, float>(xs[s], nrhs[s], (float2*)psi[s], &nblk);
    cin[s] = vec_view<double>(xs[s], eta[s], nullptr);
    cvo[s] = vec_view<S>(xs[s], a[s].rho.p, a[s].rho.scale);
    nvec[s] = 2 * nrhs[s];
    ncy = std::max(ncy, xs[s]->cfg.ncy);
  }
  HCK(x0, launch_field_convert_grp<double, S>(cin.data(), cvo.data(), nvec.data(), ns, st));
  for (int cy = 0; cy < ncy; ++cy)
    for (int col = 0; col < 2; ++col) {
      sel.clear();
      for (int s = 0; s < ns; ++s) {
        const int nc = xs[s]->cfg.ncy;
        if (cy >= nc) continue;
        SapArgs<S, float> b = a[s];
        b.col = col;
        b.first = cy == 0;
        b.do_bnd = !(cy == 0 && col == 0);
        b.write_v = !(cy == nc - 1 && col == 1);
        sel.push_back(b);
      }
      if (cy > 0 || col > 0) HCK(x0, launch_sap_face_grp<S, float>(sel.data(), (int)sel.size(), st));
      for (auto& b : sel) b.do_bnd = 0;
      HCK(x0, launch_sap_half_grp<S, float>(sel.data(), (int)sel.size(), st));
    }
  return QDD_OK;
}

qdd_status sap_apply_grp(qdd_ctx* const* xs, const int* nrhs, const double2* const* eta, void* const* psi, int ns,
                         hipStream_t st) {
  if (ns < 1 || ns > kGrpMax) {
    xs[0]->fail("grouped Schwarz: 1 to %d systems", kGrpMax);
    return QDD_EINVAL;
  }
  switch (xs[0]->cfg.sap_prec) {
    case QDD_F32: return sap_grp_run<float>(xs, nrhs, eta, psi, ns, st);
    case QDD_F16: return sap_grp_run<__half>(xs, nrhs, eta, psi, ns, st);
    default: xs[0]->fail("grouped Schwarz: FP32 or FP16 storage"); return QDD_EINVAL;
  }
}

// dispatch on the configured SAP precision; psi storage: FP64 for F64, else FP32
qdd_status sap_apply(qdd_ctx* x, int nrhs, const double2* eta, void* psi) {
  switch (x->cfg.sap_prec) {
    case QDD_F64: return sap_run<double, double>(x, nrhs, eta, (double2*)psi);
    case QDD_F32: return sap_run<float, float>(x, nrhs, eta, (float2*)psi);
    default: return sap_run<__half, float>(x, nrhs, eta, (float2*)psi);
  }
}

qdd_status make_solver_ops(qdd_ctx* x, int nrhs, FgcrOps& F) {
  int64_t n = (int64_t)24 * x->G.Vh;
  F.n = n;
  F.nrhs = nrhs;
  F.op = [x, nrhs](const double2* in, double2* out) -> qdd_status {
    HCK(x, x->dw(QDD_F64, nrhs, (void*)in, out));
    return QDD_OK;
  };
  F.phi32 = x->lo.phi32;
  switch (x->cfg.precond) {
    case QDD_PRECOND_NONE:
      F.prec = [x, nrhs, n](const double2* r, void* phi) -> qdd_status {
        HCK(x, hipMemcpyAsync(phi, r, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, x->st));
        return QDD_OK;
      };
      return QDD_OK;
    case QDD_PRECOND_SAP:
      F.prec = [x, nrhs](const double2* r, void* phi) -> qdd_status { return sap_apply(x, nrhs, r, phi); };
      return QDD_OK;
    case QDD_PRECOND_DFL:
      return dfl_make_precond(x, nrhs, F);
  }
  x->fail("unknown preconditioner");
  return QDD_EINVAL;
}

extern "C" qdd_status qdd_sap(qdd_ctx* x, int nrhs, const double* eta_c, double* psi_c) {
  if (!x || !eta_c || !psi_c || nrhs < 1 || nrhs > x->cfg.max_nrhs) {
    if (x) x->fail("qdd_sap: invalid arguments");
    return QDD_EINVAL;
  }
  std::string why;
  if (!valid_sap_blocks(&x->geom, &x->cfg, &why)) {
    x->fail("qdd_sap: %s", why.c_str());
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_sap before qdd_set_params"); return QDD_ESTATE; }
  const Layout& lo = x->lo;
  double2* eta = x->ptr<double2>(lo.s_tmp);
  PackedView pe = x->packed(QDD_F64, nrhs, 0, eta);
  HCK(x, launch_pack_spinor<double>(x->G, eta_c, pe.f64, nrhs, 0, pe.poff, pe.spoff, x->st));
  void* out = x->cfg.sap_prec == QDD_F64 ? (void*)x->ptr<double2>(lo.res) : (void*)x->ptr<float2>(lo.phi);
  qdd_status s = sap_apply(x, nrhs, eta, out);
  if (s != QDD_OK) return s;
  if (x->cfg.sap_prec == QDD_F64) {
    PackedView po = x->packed(QDD_F64, nrhs, 0, out);
    HCK(x, launch_unpack_spinor<double>(x->G, po.f64, psi_c, nrhs, 0, po.poff, po.spoff, x->st));
  } else {
    PackedView po = x->packed(QDD_F32, nrhs, 0, out);
    HCK(x, launch_unpack_spinor<float>(x->G, po.f32, psi_c, nrhs, 0, po.poff, po.spoff, x->st));
  }
  return QDD_OK;
}
