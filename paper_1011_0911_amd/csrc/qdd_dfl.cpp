// Local deflation, host side: subspace build (SAP inverse iteration, block
// orthonormalisation, little Dirac operator), the little-operator GCR and the
// two-level preconditioner M(r) = C r + M_sap(r - D C r), C = W A^{-1} W^dag
// (W the block-orthonormal basis, A = W^dag D W the little Dirac operator).
#include "qdd_dfl.h"
#include "qdd_dfl_kernels.h"

#include <cmath>
#include <cstring>
#include <vector>

using namespace qdd;

static DflGeo dfl_geo(const qdd_ctx* x) {
  DflGeo d;
  d.nblk = 1;
  for (int m = 0; m < 4; ++m) {
    d.bs[m] = x->cfg.dfl_bs[m];
    d.nb[m] = x->G.L[m] / d.bs[m];
    d.nblk *= d.nb[m];
  }
  return d;
}

// precision of the deflation correction inside the preconditioner
static bool dfl_fp64(const qdd_ctx* x) { return x->cfg.sap_prec == QDD_F64; }

// ------------------------------------------------------------------ coarse GCR
// Solves A c = f (little operator, FP64) for nrhs right-hand sides with restarted
// GCR to relative residual tol; f, c: [rhs][nblk*Ns].  Returns the iterations.
static qdd_status coarse_gcr(qdd_ctx* x, int nrhs, const double2* f, double2* c, double tol, int nmx, int* its) {
  const Layout& lo = x->lo;
  hipStream_t st = x->st;
  DflGeo d = dfl_geo(x);
  int Ns = x->cfg.dfl_Ns;
  int64_t nc = (int64_t)d.nblk * Ns, slot = (int64_t)x->cfg.max_nrhs * nc;
  double2* base = x->ptr<double2>(lo.dfl_cvec);
  double2 *r = base + 2 * slot, *t = base + 3 * slot, *P = base + 4 * slot, *Q = base + (4 + kCoarseKv) * slot;
  double2* Am = x->ptr<double2>(lo.dfl_A);
  double2 *part = x->ptr<double2>(lo.cpart), *coef = x->ptr<double2>(lo.ccoef), *rn2 = x->ptr<double2>(lo.crn2);
  double2* alpha = x->ptr<double2>(lo.calpha);
  double* binv = x->ptr<double>(lo.cbinv);
  double* bnrm = binv + x->cfg.max_nrhs;
  int* active = x->ptr<int>(lo.cactive);
  int64_t ls = (int64_t)nrhs * nc;  // stride between Krylov vectors of the batch
  std::vector<double2> h(nrhs);
  std::vector<double> fn(nrhs);
  std::vector<int> act(nrhs);
  HCK(x, launch_dots<double2>(f, 0, nc, 1, f, nc, nc, nrhs, part, rn2, st));
  HCK(x, hipMemcpyAsync(h.data(), rn2, nrhs * sizeof(double2), hipMemcpyDeviceToHost, st));
  HCK(x, hipStreamSynchronize(st));
  for (int i = 0; i < nrhs; ++i) {
    fn[i] = std::sqrt(h[i].x);
    act[i] = fn[i] > 0;
  }
  HCK(x, hipMemsetAsync(c, 0, (size_t)nrhs * nc * sizeof(double2), st));
  HCK(x, hipMemcpyAsync(r, f, (size_t)nrhs * nc * sizeof(double2), hipMemcpyDeviceToDevice, st));
  int it = 0;
  while (true) {
    bool any = false;
    for (int i = 0; i < nrhs; ++i) any |= act[i];
    if (!any || it >= nmx) break;
    HCK(x, hipMemcpyAsync(active, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    int j = 0;
    for (; j < kCoarseKv && it < nmx; ++j, ++it) {
      double2 *pj = P + j * ls, *qj = Q + j * ls;
      HCK(x, hipMemcpyAsync(pj, r, (size_t)nrhs * nc * sizeof(double2), hipMemcpyDeviceToDevice, st));
      HCK(x, launch_coarse_apply(d, Am, Ns, pj, qj, nc, nrhs, st));
      if (j > 0)
        for (int pass = 0; pass < 2; ++pass) {
          HCK(x, launch_dots<double2>(Q, ls, nc, j, qj, nc, nc, nrhs, part, coef, st));
          HCK(x, launch_axpy_multi<double2>(qj, nc, Q, ls, nc, j, coef, j, -1.0, nc, nrhs, nullptr, st));
          HCK(x, launch_axpy_multi<double2>(pj, nc, P, ls, nc, j, coef, j, -1.0, nc, nrhs, nullptr, st));
        }
      HCK(x, launch_dots<double2>(qj, 0, nc, 1, qj, nc, nc, nrhs, part, rn2, st));
      HCK(x, launch_norm_finish(rn2, bnrm, binv, nrhs, st));
      HCK(x, launch_axpby(qj, nc, qj, nc, binv, nullptr, nc, nrhs, nullptr, st));
      HCK(x, launch_axpby(pj, nc, pj, nc, binv, nullptr, nc, nrhs, nullptr, st));
      HCK(x, launch_dots<double2>(qj, 0, nc, 1, r, nc, nc, nrhs, part, alpha, st));
      HCK(x, launch_axpy_multi<double2>(r, nc, qj, 0, nc, 1, alpha, 1, -1.0, nc, nrhs, active, st));
      HCK(x, launch_axpy_multi<double2>(c, nc, pj, 0, nc, 1, alpha, 1, 1.0, nc, nrhs, active, st));
      HCK(x, launch_dots<double2>(r, 0, nc, 1, r, nc, nc, nrhs, part, rn2, st));
      HCK(x, hipMemcpyAsync(h.data(), rn2, nrhs * sizeof(double2), hipMemcpyDeviceToHost, st));
      HCK(x, hipStreamSynchronize(st));
      bool changed = false, any2 = false;
      for (int i = 0; i < nrhs; ++i) {
        if (!act[i]) continue;
        if (!(std::sqrt(std::fabs(h[i].x)) > tol * fn[i]) || !std::isfinite(h[i].x)) {
          act[i] = 0;
          changed = true;
        }
        any2 |= act[i];
      }
      if (!any2) {
        ++it;
        ++j;
        break;
      }
      if (changed) HCK(x, hipMemcpyAsync(active, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    }
    bool any3 = false;
    for (int i = 0; i < nrhs; ++i) any3 |= act[i];
    if (!any3) break;
    // restart from the true residual r = f - A c
    HCK(x, launch_coarse_apply(d, Am, Ns, c, t, nc, nrhs, st));
    HCK(x, launch_sub(r, f, t, nc, nc, nrhs, st));
  }
  if (its) *its = it;
  return QDD_OK;
}

// ------------------------------------------------------------------ build
// nit rounds of SAP inverse iteration on the fields in W (normalised after each
// round), block orthonormalisation and the little operator
static qdd_status dfl_build_from_W(qdd_ctx* x, int nit) {
  const Layout& lo = x->lo;
  const Geo& G = x->G;
  hipStream_t st = x->st;
  DflGeo d = dfl_geo(x);
  int Ns = x->cfg.dfl_Ns, nr = x->cfg.max_nrhs;
  int64_t vs = (int64_t)24 * G.Vh;
  double2* W = x->ptr<double2>(lo.dfl_W);
  // SAP inverse iteration, nr fields at a time, each normalised after every round
  double2 *part = x->ptr<double2>(lo.part), *rn2 = x->ptr<double2>(lo.rn2);
  double *bn = x->ptr<double>(lo.bhist), *binv = x->ptr<double>(lo.binv);
  void* tmp = x->ptr<void>(lo.phi);
  for (int it = 0; it < nit; ++it)
    for (int l0 = 0; l0 < Ns; l0 += nr) {
      int nb = std::min(nr, Ns - l0);
      double2* w = W + l0 * vs;
      qdd_status s = sap_apply(x, nb, w, tmp);
      if (s != QDD_OK) return s;
      if (x->cfg.sap_prec == QDD_F64) {
        HCK(x, hipMemcpyAsync(w, tmp, (size_t)nb * vs * sizeof(double2), hipMemcpyDeviceToDevice, st));
      } else {
        FieldV<float> a{(float2*)tmp, nullptr, vs, vs, (int)(vs / 12)};
        FieldV<double> b{w, nullptr, vs, vs, (int)(vs / 12)};
        HCK(x, launch_field_convert<float, double>(a, b, nb, st));
      }
      HCK(x, launch_dots<double2>(w, 0, vs, 1, w, vs, vs, nb, part, rn2, st));
      HCK(x, launch_norm_finish(rn2, bn, binv, nb, st));
      HCK(x, launch_axpby(w, vs, w, vs, binv, nullptr, vs, nb, nullptr, st));
    }
  // block orthonormalisation (the little-operator storage is its work space)
  double2* Am = x->ptr<double2>(lo.dfl_A);
  HCK(x, launch_block_orth(G, d, W, vs, Ns, Am, st));
  // little operator: self (hops inside blocks) and the 8 face couplings; a face
  // term is non-zero only on that face of every block
  double2* F = x->ptr<double2>(lo.dfl_init);
  for (int mode = 0; mode < 9; ++mode) {
    HCK(x, launch_dfl_hops(G, d, x->op<double>(), W, vs, F, Ns, mode, st));
    HCK(x, launch_block_dots<double2, double2>(G, d, W, vs, Ns, F, vs, Ns, Am + (int64_t)mode * Ns * Ns,
                                               (int64_t)9 * Ns * Ns, Ns, 1, st, mode));
  }
  if (!dfl_fp64(x)) {
    HCK(x, launch_convert(W, x->ptr<float2>(lo.dfl_W32), (int64_t)Ns * vs, st));
    if (block_major_ok(d)) HCK(x, launch_to_blocks(G, d, W, vs, Ns, x->ptr<float2>(lo.dfl_W32b), st));
  }
  HCK(x, hipStreamSynchronize(st));
  x->have_dfl = true;
  return QDD_OK;
}

extern "C" qdd_status qdd_dfl_build(qdd_ctx* x, const double* init) {
  if (!x || !init) {
    if (x) x->fail("qdd_dfl_build: invalid arguments");
    return QDD_EINVAL;
  }
  if (x->cfg.dfl_Ns <= 0) { x->fail("qdd_dfl_build: dfl_Ns is 0"); return QDD_EINVAL; }
  if (!x->have_clover) { x->fail("qdd_dfl_build before qdd_set_params"); return QDD_ESTATE; }
  double2* W = x->ptr<double2>(x->lo.dfl_W);
  PackedView pw = x->packed(QDD_F64, x->cfg.dfl_Ns, 0, W);
  HCK(x, launch_pack_spinor<double>(x->G, init, pw.f64, x->cfg.dfl_Ns, 0, pw.poff, pw.spoff, x->st));
  qdd_status s = dfl_build_from_W(x, x->cfg.dfl_nit);
  if (s == QDD_OK) {
    x->dfl_builds++;
    x->have_basis = true;
  }
  return s;
}

// Refresh of the subspace for the current operator (after the gauge field or the
// mass changed): dfl_refresh_nit rounds of SAP inverse iteration started from the
// current basis, then orthonormalisation and little operator as in a build.
qdd_status dfl_refresh_impl(qdd_ctx* x) {
  qdd_status s = dfl_build_from_W(x, x->cfg.dfl_refresh_nit);
  if (s == QDD_OK) x->dfl_refreshes++;
  return s;
}

extern "C" qdd_status qdd_dfl_refresh(qdd_ctx* x) {
  if (!x) return QDD_EINVAL;
  if (x->cfg.dfl_Ns <= 0) { x->fail("qdd_dfl_refresh: dfl_Ns is 0"); return QDD_EINVAL; }
  if (!x->have_clover) { x->fail("qdd_dfl_refresh before qdd_set_params"); return QDD_ESTATE; }
  if (!x->have_basis) { x->fail("qdd_dfl_refresh before a subspace was built or shared"); return QDD_ESTATE; }
  return dfl_refresh_impl(x);
}

extern "C" qdd_status qdd_dfl_stats(const qdd_ctx* x, int* builds, int* refreshes) {
  if (!x) return QDD_EINVAL;
  if (builds) *builds = x->dfl_builds;
  if (refreshes) *refreshes = x->dfl_refreshes;
  return QDD_OK;
}

// ------------------------------------------------------------------ preconditioner
// c = W^dag r (per block), coarse solve, Cr = W c (precision P), t = D Cr,
// r1 = r - t (FP64), phi = Cr + M_sap(r1)
template <class EP>
static qdd_status dfl_apply(qdd_ctx* x, int nrhs, const double2* r, EP* phi, double* tcoarse) {
  const Layout& lo = x->lo;
  const Geo& G = x->G;
  hipStream_t st = x->st;
  DflGeo d = dfl_geo(x);
  int Ns = x->cfg.dfl_Ns;
  int64_t vs = (int64_t)24 * G.Vh, nc = (int64_t)d.nblk * Ns, slot = (int64_t)x->cfg.max_nrhs * nc;
  double2* cbase = x->ptr<double2>(lo.dfl_cvec);
  double2 *cf = cbase, *cc = cbase + slot;
  constexpr bool F64 = sizeof(EP) == 16;
  // restriction
  if constexpr (F64)
    HCK(x, launch_block_dots<double2, double2>(G, d, x->ptr<double2>(lo.dfl_W), vs, Ns, r, vs, nrhs, cf, Ns, 1, nc,
                                               st));
  else if (block_major_ok(d) && block_mm_fits(Ns, 1, 0, d))
    HCK(x, launch_block_dots_xb(G, d, x->ptr<float2>(lo.dfl_W32b), Ns, r, vs, nrhs, cf, Ns, 1, nc, st));
  else
    HCK(x, launch_block_dots<float2, double2>(G, d, x->ptr<float2>(lo.dfl_W32), vs, Ns, r, vs, nrhs, cf, Ns, 1, nc,
                                              st));
  int its = 0;
  qdd_status s = coarse_gcr(x, nrhs, cf, cc, x->cfg.dfl_coarse_tol, x->cfg.dfl_coarse_nmx, &its);
  if (s != QDD_OK) return s;
  x->coarse_iters += its;
  // prolongation and the deflation-corrected residual
  EP* Cr = x->ptr<EP>(lo.dfl_cr);
  EP* t = x->ptr<EP>(lo.dfl_t);
  if constexpr (F64)
    HCK(x, launch_prolong<double2, double2>(G, d, x->ptr<double2>(lo.dfl_W), vs, Ns, cc, nc, Cr, vs, nrhs, st));
  else
    HCK(x, launch_prolong<float2, float2>(G, d, x->ptr<float2>(lo.dfl_W32), vs, Ns, cc, nc, Cr, vs, nrhs, st));
  HCK(x, x->dw(F64 ? QDD_F64 : QDD_F32, nrhs, Cr, t));
  double2* r1 = x->ptr<double2>(lo.s_tmp);
  if constexpr (F64) {
    HCK(x, launch_sub(r1, r, (const double2*)t, vs, vs, nrhs, st));
  } else {
    FieldV<float> a{(float2*)t, nullptr, vs, vs, (int)(vs / 12)};
    FieldV<double> b{r1, nullptr, vs, vs, (int)(vs / 12)};
    HCK(x, launch_field_convert<float, double>(a, b, nrhs, st));
    HCK(x, launch_sub(r1, r, r1, vs, vs, nrhs, st));
  }
  (void)tcoarse;
  if constexpr (!F64) {
    // the network stage; not during a pair harvest, whose pairs are those of the plain method
    if (x->cfg.use_net && x->have_net && !x->harvest && (x->net_calls == 0 || x->net_calls_done < x->net_calls)) {
      ++x->net_calls_done;
      float2* vn = x->ptr<float2>(lo.net_tmp);
      double2* r2 = x->ptr<double2>(lo.t64);
      std::vector<int> fb;
      s = net_stage(x, nrhs, r1, vn, r2, (float2*)t, fb);
      if (s != QDD_OK) return s;
      if ((int)x->fallbacks.size() < nrhs) x->fallbacks.resize(nrhs, 0);
      for (int j = 0; j < nrhs; ++j) x->fallbacks[j] += fb[j];
      s = sap_apply(x, nrhs, r2, phi);
      if (s != QDD_OK) return s;
      HCK(x, launch_add<EP>(phi, Cr, 1.0, (int64_t)nrhs * vs, st));
      HCK(x, launch_add<EP>(phi, (const EP*)vn, 1.0, (int64_t)nrhs * vs, st));
      return QDD_OK;
    }
  }
  s = sap_apply(x, nrhs, r1, phi);
  if (s != QDD_OK) return s;
  HCK(x, launch_add<EP>(phi, Cr, 1.0, (int64_t)nrhs * vs, st));
  return QDD_OK;
}

qdd_status dfl_precond_apply(qdd_ctx* x, int nrhs, const double2* r, void* phi) {
  if (dfl_fp64(x)) return dfl_apply<double2>(x, nrhs, r, (double2*)phi, nullptr);
  return dfl_apply<float2>(x, nrhs, r, (float2*)phi, nullptr);
}

qdd_status dfl_make_precond(qdd_ctx* x, int nrhs, FgcrOps& F) {
  F.prec = [x, nrhs](const double2* r, void* phi) -> qdd_status { return dfl_precond_apply(x, nrhs, r, phi); };
  return QDD_OK;
}

// ------------------------------------------------------------------ test / inspection entry points
extern "C" qdd_status qdd_dfl_export(qdd_ctx* x, double* basis, double* little) {
  if (!x) return QDD_EINVAL;
  if (!x->have_dfl) { x->fail("qdd_dfl_export before qdd_dfl_build"); return QDD_ESTATE; }
  const Layout& lo = x->lo;
  int Ns = x->cfg.dfl_Ns;
  if (basis) {
    PackedView pw = x->packed(QDD_F64, Ns, 0, x->ptr<double2>(lo.dfl_W));
    HCK(x, launch_unpack_spinor<double>(x->G, pw.f64, basis, Ns, 0, pw.poff, pw.spoff, x->st));
  }
  if (little)
    HCK(x, hipMemcpyAsync(little, x->ptr<double2>(lo.dfl_A), (size_t)lo.nblk_dfl * 9 * Ns * Ns * sizeof(double2),
                          hipMemcpyDeviceToDevice, x->st));
  HCK(x, hipStreamSynchronize(x->st));
  return QDD_OK;
}

extern "C" qdd_status qdd_dfl_coarse_solve(qdd_ctx* x, int nrhs, const double* f, double* c, double tol, int* iters) {
  if (!x || !f || !c || nrhs < 1 || nrhs > x->cfg.max_nrhs || !(tol > 0)) {
    if (x) x->fail("qdd_dfl_coarse_solve: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_dfl) { x->fail("qdd_dfl_coarse_solve before qdd_dfl_build"); return QDD_ESTATE; }
  DflGeo d = dfl_geo(x);
  int64_t nc = (int64_t)d.nblk * x->cfg.dfl_Ns, slot = (int64_t)x->cfg.max_nrhs * nc;
  double2* cbase = x->ptr<double2>(x->lo.dfl_cvec);
  HCK(x, hipMemcpyAsync(cbase, f, (size_t)nrhs * nc * sizeof(double2), hipMemcpyDeviceToDevice, x->st));
  qdd_status s = coarse_gcr(x, nrhs, cbase, cbase + slot, tol, 100000, iters);
  if (s != QDD_OK) return s;
  HCK(x, hipMemcpyAsync(c, cbase + slot, (size_t)nrhs * nc * sizeof(double2), hipMemcpyDeviceToDevice, x->st));
  HCK(x, hipStreamSynchronize(x->st));
  return QDD_OK;
}

extern "C" qdd_status qdd_dfl_precond(qdd_ctx* x, int nrhs, const double* r_c, double* out_c) {
  if (!x || !r_c || !out_c || nrhs < 1 || nrhs > x->cfg.max_nrhs) {
    if (x) x->fail("qdd_dfl_precond: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_dfl) { x->fail("qdd_dfl_precond before qdd_dfl_build"); return QDD_ESTATE; }
  const Layout& lo = x->lo;
  double2* r = x->ptr<double2>(lo.res);
  PackedView pr = x->packed(QDD_F64, nrhs, 0, r);
  HCK(x, launch_pack_spinor<double>(x->G, r_c, pr.f64, nrhs, 0, pr.poff, pr.spoff, x->st));
  void* phi = x->ptr<void>(lo.phi);
  qdd_status s = dfl_precond_apply(x, nrhs, r, phi);
  if (s != QDD_OK) return s;
  if (dfl_fp64(x)) {
    PackedView po = x->packed(QDD_F64, nrhs, 0, phi);
    HCK(x, launch_unpack_spinor<double>(x->G, po.f64, out_c, nrhs, 0, po.poff, po.spoff, x->st));
  } else {
    PackedView po = x->packed(QDD_F32, nrhs, 0, phi);
    HCK(x, launch_unpack_spinor<float>(x->G, po.f32, out_c, nrhs, 0, po.poff, po.spoff, x->st));
  }
  HCK(x, hipStreamSynchronize(x->st));
  return QDD_OK;
}

// ------------------------------------------------------------------ subspace sharing across masses
// shift the diagonal of every block's self-coupling by delta (little operator of
// D + delta: A = W^dag (D + delta) W = W^dag D W + delta 1 for a block-orthonormal W)
__global__ void k_little_shift(double2* Am, int Ns, int nblk, double delta) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblk * Ns) return;
  int b = t / Ns, k = t % Ns;
  double2& v = Am[(((int64_t)b * 9) * Ns + k) * Ns + k];
  v.x += delta;
}

extern "C" qdd_status qdd_dfl_share(qdd_ctx* dst, const qdd_ctx* src) {
  if (!dst || !src) return QDD_EINVAL;
  if (!src->have_dfl) { dst->fail("qdd_dfl_share: source has no deflation subspace"); return QDD_ESTATE; }
  if (!dst->have_clover) { dst->fail("qdd_dfl_share before qdd_set_params"); return QDD_ESTATE; }
  for (int m = 0; m < 4; ++m)
    if (dst->geom.L[m] != src->geom.L[m] || dst->cfg.dfl_bs[m] != src->cfg.dfl_bs[m]) {
      dst->fail("qdd_dfl_share: lattice or deflation blocks differ");
      return QDD_EINVAL;
    }
  if (dst->cfg.dfl_Ns != src->cfg.dfl_Ns || dst->geom.bc_time != src->geom.bc_time ||
      (dst->cfg.sap_prec == QDD_F64) != (src->cfg.sap_prec == QDD_F64)) {
    dst->fail("qdd_dfl_share: Ns, boundary condition or deflation precision differ");
    return QDD_EINVAL;
  }
  const Layout &ld = dst->lo, &ls = src->lo;
  int Ns = dst->cfg.dfl_Ns;
  int64_t vs = (int64_t)24 * dst->G.Vh;
  DflGeo d = dfl_geo(dst);
  // the same gauge field is assumed; the caller guarantees it (the links are not compared)
  HCK(dst, hipMemcpyAsync(dst->ptr<double2>(ld.dfl_W), src->ptr<double2>(ls.dfl_W), (size_t)Ns * vs * 16,
                          hipMemcpyDeviceToDevice, dst->st));
  if (!dfl_fp64(dst)) {
    HCK(dst, hipMemcpyAsync(dst->ptr<float2>(ld.dfl_W32b), src->ptr<float2>(ls.dfl_W32b), (size_t)Ns * vs * 8,
                            hipMemcpyDeviceToDevice, dst->st));
    HCK(dst, hipMemcpyAsync(dst->ptr<float2>(ld.dfl_W32), src->ptr<float2>(ls.dfl_W32), (size_t)Ns * vs * 8,
                            hipMemcpyDeviceToDevice, dst->st));
  }
  HCK(dst, hipMemcpyAsync(dst->ptr<double2>(ld.dfl_A), src->ptr<double2>(ls.dfl_A),
                          (size_t)d.nblk * 9 * Ns * Ns * 16, hipMemcpyDeviceToDevice, dst->st));
  double delta = 1.0 / (2.0 * dst->kappa) - 1.0 / (2.0 * src->kappa);
  hipLaunchKernelGGL(k_little_shift, dim3((d.nblk * Ns + 255) / 256), dim3(256), 0, dst->st,
                     dst->ptr<double2>(ld.dfl_A), Ns, d.nblk, delta);
  HCK(dst, hipGetLastError());
  HCK(dst, hipStreamSynchronize(dst->st));
  dst->have_dfl = true;
  dst->have_basis = true;
  return QDD_OK;
}
