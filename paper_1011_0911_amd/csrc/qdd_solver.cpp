// Outer flexible GCR in FP64 (the outer solver of the paper's locally deflated
// Schwarz-preconditioned GCR, Sect. 3): phi_k = M(r_k), chi_k = D phi_k,
// classical Gram-Schmidt with one re-orthogonalisation pass, r -= c_k chi_k; at
// the end of a cycle the small triangular system is back-substituted on the host,
// psi += sum alpha_k phi_k, and the residual is recomputed with the FP64
// operator.  All right-hand sides of a batch advance together through batched
// kernels; each keeps its own coefficients and convergence flag.
#include "qdd_api_internal.h"
#include "qdd_solver.h"
#include "qdd_net.h"
#include "qdd_dfl_kernels.h"

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

using namespace qdd;

// back substitution of one right-hand side's m steps: R alpha = c with the
// Gram-Schmidt coefficients of chi_l on chi_0 .. chi_{l-1} (ah, row stride kMaxKv
// per rhs and step), the norms b_j and c_j = <chi_j, r_j>; al: kMaxKv entries
void fgcr_backsub(const double2* ah, const double* bh, const double2* chh, int nr, int i, int m, double2* al) {
  for (int j = m - 1; j >= 0; --j) {
    double sr = chh[(size_t)j * nr + i].x, si = chh[(size_t)j * nr + i].y;
    for (int l = j + 1; l < m; ++l) {
      double2 a2 = ah[((size_t)l * nr + i) * kMaxKv + j], b2 = al[l];
      sr -= a2.x * b2.x - a2.y * b2.y;
      si -= a2.x * b2.y + a2.y * b2.x;
    }
    double bj = bh[(size_t)j * nr + i];
    al[j] = bj > 0 ? double2{sr / bj, si / bj} : double2{0.0, 0.0};
  }
}

qdd_status run_fgcr(qdd_ctx* x, FgcrOps& F, const double2* eta, double2* psi, qdd_solve_info* info) {
  const Layout& lo = x->lo;
  hipStream_t st = x->st;
  int nr = F.nrhs, nkv = x->cfg.nkv, nmx = x->cfg.nmx;
  int64_t n = F.n;
  double tol = x->cfg.tol;
  double2 *r = x->ptr<double2>(lo.res), *t = x->ptr<double2>(lo.t64), *chi = x->ptr<double2>(lo.chi);
  void* phi = x->ptr<void>(lo.phi);
  double2 *part = x->ptr<double2>(lo.part), *coef = x->ptr<double2>(lo.coef);
  double2 *ahist = x->ptr<double2>(lo.ahist), *chist = x->ptr<double2>(lo.chist), *rn2 = x->ptr<double2>(lo.rn2);
  double *bhist = x->ptr<double>(lo.bhist), *binv = x->ptr<double>(lo.binv);
  double2* alpha = x->ptr<double2>(lo.alpha);
  int* active = x->ptr<int>(lo.active);
  int64_t lstride = (int64_t)nr * n;
  size_t phi_e = F.phi32 ? 8 : 16;
  auto phi_k = [&](int k) { return (void*)((char*)phi + (size_t)k * lstride * phi_e); };
  auto chi_k = [&](int k) { return chi + (size_t)k * lstride; };

  auto t0 = std::chrono::steady_clock::now();
  x->net_calls_done = 0;  // a new solve: the network stage counts its applications afresh
  std::vector<double> tstage(8, 0.0);
  StageEvents ev;
  HCK(x, ev.init());
  auto tic = [&]() { return std::chrono::steady_clock::now(); };
  auto since = [&](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
  };

  // |eta|
  std::vector<double2> h2(nr);
  std::vector<double> etan(nr), rn(nr);
  HCK(x, launch_dots<double2>(eta, 0, n, 1, eta, n, n, nr, part, rn2, st));
  HCK(x, hipMemcpyAsync(h2.data(), rn2, nr * sizeof(double2), hipMemcpyDeviceToHost, st));
  HCK(x, hipStreamSynchronize(st));
  for (int i = 0; i < nr; ++i) etan[i] = std::sqrt(h2[i].x);
  std::vector<int> act(nr), conv(nr, 0), iters(nr, 0), restarts(nr, 0);
  if (F.warm) {
    // psi holds the initial guess: r = eta - D psi
    qdd_status s0 = F.op(psi, t);
    if (s0 != QDD_OK) return s0;
    HCK(x, launch_sub(r, eta, t, n, n, nr, st));
    HCK(x, launch_dots<double2>(r, 0, n, 1, r, n, n, nr, part, rn2, st));
    HCK(x, hipMemcpyAsync(h2.data(), rn2, nr * sizeof(double2), hipMemcpyDeviceToHost, st));
    HCK(x, hipStreamSynchronize(st));
    for (int i = 0; i < nr; ++i) {
      rn[i] = std::sqrt(std::fabs(h2[i].x));
      conv[i] = !(etan[i] > 0) || rn[i] <= tol * etan[i];
      act[i] = !conv[i];
    }
  } else {
    // psi = 0, r = eta
    HCK(x, hipMemsetAsync(psi, 0, (size_t)nr * n * sizeof(double2), st));
    HCK(x, hipMemcpyAsync(r, eta, (size_t)nr * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
    for (int i = 0; i < nr; ++i) {
      rn[i] = etan[i];
      conv[i] = !(etan[i] > 0);
      act[i] = !conv[i];
    }
  }
  std::vector<double2> ah((size_t)kMaxKv * nr * kMaxKv), chh((size_t)kMaxKv * nr), al((size_t)nr * kMaxKv);
  std::vector<double> bh((size_t)kMaxKv * nr);
  bool nonfinite = false;
  int total_it = 0;
  qdd_status status = QDD_OK;
  while (true) {
    bool any = false;
    for (int i = 0; i < nr; ++i) any |= act[i];
    if (!any || total_it >= nmx) break;
    HCK(x, hipMemcpyAsync(active, act.data(), nr * sizeof(int), hipMemcpyHostToDevice, st));
    std::vector<int> ks(nr, 0);
    int k = 0;
    for (; k < nkv && total_it < nmx; ++k) {
      auto ta = tic();
      HCK(x, ev.mark(0, st));
      // phi_k = M(r)
      qdd_status s = F.prec(r, phi_k(k));
      if (s != QDD_OK) return s;
      if (F.sync_stages) HCK(x, hipStreamSynchronize(st));
      tstage[1] += since(ta);
      HCK(x, ev.mark(1, st));
      ta = tic();
      // chi_k = D phi_k
      if (F.phi32) {
        FieldV<float> src{(float2*)phi_k(k), nullptr, n, n, (int)n};
        FieldV<double> dst{t, nullptr, n, n, (int)n};
        // viewed as nr vectors of n/12 "sites" of 12 components each
        src.n = dst.n = (int)(n / 12);
        HCK(x, launch_field_convert<float, double>(src, dst, nr, st));
        s = F.op(t, chi_k(k));
      } else {
        s = F.op((const double2*)phi_k(k), chi_k(k));
      }
      if (s != QDD_OK) return s;
      if (F.sync_stages) HCK(x, hipStreamSynchronize(st));
      tstage[2] += since(ta);
      HCK(x, ev.mark(2, st));
      ta = tic();
      // Gram-Schmidt against chi_0 .. chi_{k-1}, two passes; every update sweep
      // also forms the next inner products (the same sums as separate launches)
      double2* ak = ahist + (size_t)k * nr * kMaxKv;
      HCK(x, hipMemsetAsync(ak, 0, (size_t)nr * kMaxKv * sizeof(double2), st));
      if (k > 0) {
        HCK(x, launch_dots<double2>(chi, lstride, n, k, chi_k(k), n, n, nr, part, coef, st));
        HCK(x, launch_acc_coef(ak, kMaxKv, coef, k, nr, st));
        // pass 1 update + pass 2 products
        HCK(x, launch_sub_dots(chi_k(k), n, chi, lstride, n, k, coef, k, nullptr, 0, n, nr, part, coef, st));
        HCK(x, launch_acc_coef(ak, kMaxKv, coef, k, nr, st));
        // pass 2 update + |chi_k|^2
        HCK(x, launch_sub_dots(chi_k(k), n, chi, lstride, n, k, coef, k, nullptr, 1, n, nr, part, rn2, st));
      } else {
        HCK(x, launch_dots<double2>(chi_k(k), 0, n, 1, chi_k(k), n, n, nr, part, rn2, st));
      }
      HCK(x, launch_norm_finish(rn2, bhist + (size_t)k * nr, binv, nr, st));
      // chi_k /= |chi_k| + c_k = <chi_k, r>; r -= c_k chi_k + |r|^2
      HCK(x, launch_scale_dot(chi_k(k), n, binv, r, n, n, nr, part, chist + (size_t)k * nr, st));
      HCK(x, launch_sub_dots(r, n, chi_k(k), 0, n, 1, chist + (size_t)k * nr, 1, active, 1, n, nr, part, rn2, st));
      HCK(x, ev.mark(3, st));
      HCK(x, hipMemcpyAsync(h2.data(), rn2, nr * sizeof(double2), hipMemcpyDeviceToHost, st));
      HCK(x, hipStreamSynchronize(st));
      HCK(x, ev.add(0, 3));
      tstage[3] += since(ta);
      // (the iteration that converges is not captured: its iterate is the solution, e = 0)
      // capture (r_k, psi_k) of every right-hand side still iterating, with
      // psi_k = psi + sum_{j<=k} alpha_j phi_j (back-substitution over the steps so far)
      if (F.hv && F.hv->n < F.hv->max) {
        Harvest& hv = *F.hv;
        std::vector<int> cap;
        for (int i = 0; i < nr && hv.n + (int)cap.size() < hv.max; ++i)
          if (act[i] && std::sqrt(std::fabs(h2[i].x)) > tol * etan[i]) cap.push_back(i);
        if (!cap.empty()) {
          const int m = k + 1;
          HCK(x, hipMemcpyAsync(ah.data(), ahist, (size_t)m * nr * kMaxKv * sizeof(double2), hipMemcpyDeviceToHost, st));
          HCK(x, hipMemcpyAsync(bh.data(), bhist, (size_t)m * nr * sizeof(double), hipMemcpyDeviceToHost, st));
          HCK(x, hipMemcpyAsync(chh.data(), chist, (size_t)m * nr * sizeof(double2), hipMemcpyDeviceToHost, st));
          HCK(x, hipStreamSynchronize(st));
          std::fill(al.begin(), al.end(), double2{0.0, 0.0});
          for (int i : cap) fgcr_backsub(ah.data(), bh.data(), chh.data(), nr, i, m, al.data() + (size_t)i * kMaxKv);
          HCK(x, hipMemcpyAsync(alpha, al.data(), (size_t)nr * kMaxKv * sizeof(double2), hipMemcpyHostToDevice, st));
          for (int i : cap) {
            HCK(x, launch_scale_to_f<double2>(hv.r + (int64_t)hv.n * n, r + (int64_t)i * n, 1.0, n, st));
            double2* pk = (double2*)hv.e + (int64_t)hv.n * n;
            HCK(x, hipMemcpyAsync(pk, psi + (int64_t)i * n, n * sizeof(double2), hipMemcpyDeviceToDevice, st));
            const double2* ai = alpha + (size_t)i * kMaxKv;
            if (F.phi32)
              HCK(x, launch_axpy_multi<float2>(pk, n, (const float2*)phi + (int64_t)i * n, lstride, n, m, ai, kMaxKv,
                                               1.0, n, 1, nullptr, st));
            else
              HCK(x, launch_axpy_multi<double2>(pk, n, (const double2*)phi + (int64_t)i * n, lstride, n, m, ai,
                                                kMaxKv, 1.0, n, 1, nullptr, st));
            hv.rhs.push_back(i);
            hv.n++;
          }
        }
      }
      ++total_it;
      bool changed = false, any2 = false;
      for (int i = 0; i < nr; ++i) {
        if (!act[i]) continue;
        ks[i] = k + 1;
        iters[i]++;
        rn[i] = std::sqrt(std::fabs(h2[i].x));
        if (!std::isfinite(h2[i].x)) {
          nonfinite = true;
          act[i] = 0;
          changed = true;
        } else if (rn[i] <= tol * etan[i]) {
          act[i] = 0;  // recursive residual converged: stop this rhs for the cycle
          changed = true;
        }
        any2 |= act[i];
      }
      if (!any2) { ++k; break; }
      if (changed) HCK(x, hipMemcpyAsync(active, act.data(), nr * sizeof(int), hipMemcpyHostToDevice, st));
    }
    int kk = k;
    // back substitution per rhs
    auto ta = tic();
    HCK(x, hipMemcpyAsync(ah.data(), ahist, (size_t)kk * nr * kMaxKv * sizeof(double2), hipMemcpyDeviceToHost, st));
    HCK(x, hipMemcpyAsync(bh.data(), bhist, (size_t)kk * nr * sizeof(double), hipMemcpyDeviceToHost, st));
    HCK(x, hipMemcpyAsync(chh.data(), chist, (size_t)kk * nr * sizeof(double2), hipMemcpyDeviceToHost, st));
    HCK(x, hipStreamSynchronize(st));
    std::fill(al.begin(), al.end(), double2{0.0, 0.0});
    for (int i = 0; i < nr; ++i) fgcr_backsub(ah.data(), bh.data(), chh.data(), nr, i, ks[i], al.data() + (size_t)i * kMaxKv);
    HCK(x, hipMemcpyAsync(alpha, al.data(), (size_t)nr * kMaxKv * sizeof(double2), hipMemcpyHostToDevice, st));
    HCK(x, ev.mark(3, st));
    if (F.phi32)
      HCK(x, launch_axpy_multi<float2>(psi, n, (const float2*)phi, lstride, n, kk, alpha, kMaxKv, 1.0, n, nr, nullptr,
                                       st));
    else
      HCK(x, launch_axpy_multi<double2>(psi, n, (const double2*)phi, lstride, n, kk, alpha, kMaxKv, 1.0, n, nr,
                                        nullptr, st));
    // true residual r = eta - D psi
    qdd_status s = F.op(psi, t);
    if (s != QDD_OK) return s;
    HCK(x, launch_sub(r, eta, t, n, n, nr, st));
    HCK(x, launch_dots<double2>(r, 0, n, 1, r, n, n, nr, part, rn2, st));
    HCK(x, ev.mark(4, st));
    HCK(x, hipMemcpyAsync(h2.data(), rn2, nr * sizeof(double2), hipMemcpyDeviceToHost, st));
    HCK(x, hipStreamSynchronize(st));
    HCK(x, ev.add(3, 4));
    tstage[7] += since(ta);
    for (int i = 0; i < nr; ++i) {
      if (conv[i]) continue;
      rn[i] = std::sqrt(std::fabs(h2[i].x));
      if (!std::isfinite(h2[i].x)) {
        nonfinite = true;
        act[i] = 0;
      } else if (rn[i] <= tol * etan[i]) {
        conv[i] = 1;
        act[i] = 0;
      } else {
        act[i] = 1;
        restarts[i]++;
      }
    }
    if (nonfinite) break;
  }
  if (F.hv)
    // e_j = psi*_{rhs(j)} - psi_j in FP64, then packed as FP32 at the front of
    // the buffer (slot j of the FP32 output only overlaps FP64 slots that are
    // already consumed)
    for (int j = 0; j < F.hv->n; ++j) {
      HCK(x, launch_sub(t, psi + (int64_t)F.hv->rhs[j] * n, (const double2*)F.hv->e + (int64_t)j * n, n, n, 1, st));
      HCK(x, launch_scale_to_f<double2>((float2*)F.hv->e + (int64_t)j * n, t, 1.0, n, st));
    }
  double tot = since(t0);
  for (int i = 0; i < nr; ++i) {
    if (!conv[i]) status = QDD_ENOCONV;
    if (info) {
      info[i].iters = iters[i];
      info[i].restarts = conv[i] ? restarts[i] : std::max(0, restarts[i] - 1);
      info[i].converged = conv[i];
      info[i].fallbacks = F.fallbacks ? F.fallbacks[i] : 0;
      info[i].true_res = etan[i] > 0 ? rn[i] / etan[i] : 0.0;
      for (int s2 = 0; s2 < 8; ++s2) info[i].t_ms[s2] = tstage[s2];
      info[i].t_ms[0] = tot;
      for (int s2 = 4; s2 < 7; ++s2) info[i].t_ms[s2] = F.tstage ? F.tstage[s2] : 0.0;
      for (int s2 = 0; s2 < 4; ++s2) info[i].gpu_ms[s2] = ev.gpu_ms[s2];
    }
  }
  if (status != QDD_OK) x->fail(nonfinite ? "non-finite residual" : "no convergence within nmx iterations");
  return status;
}

// ------------------------------------------------------------------ entry points
extern "C" qdd_status qdd_solve_dhat(qdd_ctx* x, int nrhs, const double* eta_e, double* psi_e,
                                     qdd_solve_info* info) {
  if (!x || !eta_e || !psi_e || nrhs < 1 || nrhs > x->cfg.max_nrhs) {
    if (x) x->fail("qdd_solve_dhat: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_solve_dhat before qdd_set_params"); return QDD_ESTATE; }
  const Layout& lo = x->lo;
  int64_t n = (int64_t)12 * x->G.Vh;
  double2 *eta = x->ptr<double2>(lo.eta), *psi = x->ptr<double2>(lo.psi);
  PackedView pe = x->packed(QDD_F64, nrhs, 1, eta);
  HCK(x, launch_pack_spinor<double>(x->G, eta_e, pe.f64, nrhs, 1, pe.poff, pe.spoff, x->st));
  FgcrOps F;
  F.n = n;
  F.nrhs = nrhs;
  F.phi32 = false;
  F.op = [&](const double2* in, double2* out) -> qdd_status {
    HCK(x, x->dhat(QDD_F64, nrhs, (void*)in, out));
    return QDD_OK;
  };
  F.prec = [&](const double2* r, void* phi) -> qdd_status {
    HCK(x, hipMemcpyAsync(phi, r, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, x->st));
    return QDD_OK;
  };
  // the FGCR buffers hold full fields; with even fields only their first half is used
  qdd_status s = run_fgcr(x, F, eta, psi, info);
  PackedView pp = x->packed(QDD_F64, nrhs, 1, psi);
  HCK(x, launch_unpack_spinor<double>(x->G, pp.f64, psi_e, nrhs, 1, pp.poff, pp.spoff, x->st));
  HCK(x, hipStreamSynchronize(x->st));
  return s;
}

// ------------------------------------------------------------------ chronological inversion
// The initial guess of a solve from the solutions of earlier ones (Sect. 3, the
// chronological inversion method the paper uses for all inversions): for each
// right-hand side with k stored solutions psi_j, the images z_j = D psi_j are
// orthonormalised by Gram-Schmidt (two passes, FP64), z = q R, and the guess is
// sum_j c_j psi_j with R c = q^dag eta, the combination with the smallest
// residual |eta - D sum c_j psi_j|.  Images that are (numerically) dependent on
// the earlier ones are dropped.  The images are formed in the Krylov space.
static qdd_status chrono_guess(qdd_ctx* x, int nrhs, const double2* eta, double2* psi) {
  const Layout& lo = x->lo;
  hipStream_t st = x->st;
  const int nv = x->cfg.chrono_nv;
  const int64_t n = (int64_t)24 * x->G.Vh;
  double2* hist = x->ptr<double2>(lo.chrono);
  double2* z = x->ptr<double2>(lo.chi);
  double2 *part = x->ptr<double2>(lo.part), *coef = x->ptr<double2>(lo.coef), *rn2 = x->ptr<double2>(lo.rn2);
  HCK(x, hipMemsetAsync(psi, 0, (size_t)nrhs * n * sizeof(double2), st));
  std::vector<double2> hc(kMaxKv);
  for (int r = 0; r < nrhs; ++r) {
    const int k = std::min(x->chrono_count[r], nv);
    if (k == 0) continue;
    const double2* ps = hist + (int64_t)r * nv * n;
    HCK(x, x->dw(QDD_F64, k, (void*)ps, z));
    std::vector<double> z0(k), R((size_t)k * k, 0.0);
    std::vector<double2> Rc((size_t)k * k, double2{0.0, 0.0});
    HCK(x, launch_dots<double2>(z, 0, n, 1, z, n, n, k, part, rn2, st));
    HCK(x, hipMemcpyAsync(hc.data(), rn2, k * sizeof(double2), hipMemcpyDeviceToHost, st));
    HCK(x, hipStreamSynchronize(st));
    for (int j = 0; j < k; ++j) z0[j] = std::sqrt(hc[j].x);
    std::vector<int> keep(k, 1);
    double* binv = x->ptr<double>(lo.binv);
    for (int i = 0; i < k; ++i) {
      double2* zi = z + (int64_t)i * n;
      if (i > 0)
        for (int pass = 0; pass < 2; ++pass) {
          HCK(x, launch_dots<double2>(z, n, n, i, zi, n, n, 1, part, coef, st));
          HCK(x, hipMemcpyAsync(hc.data(), coef, i * sizeof(double2), hipMemcpyDeviceToHost, st));
          HCK(x, hipStreamSynchronize(st));
          for (int j = 0; j < i; ++j) {
            if (!keep[j]) hc[j] = double2{0.0, 0.0};
            Rc[(size_t)j * k + i].x += hc[j].x;
            Rc[(size_t)j * k + i].y += hc[j].y;
          }
          HCK(x, hipMemcpyAsync(coef, hc.data(), i * sizeof(double2), hipMemcpyHostToDevice, st));
          HCK(x, launch_axpy_multi<double2>(zi, n, z, n, n, i, coef, i, -1.0, n, 1, nullptr, st));
        }
      HCK(x, launch_dots<double2>(zi, 0, n, 1, zi, n, n, 1, part, rn2, st));
      HCK(x, hipMemcpyAsync(hc.data(), rn2, sizeof(double2), hipMemcpyDeviceToHost, st));
      HCK(x, hipStreamSynchronize(st));
      const double nrm = std::sqrt(std::fabs(hc[0].x));
      if (!(nrm > 1e-10 * z0[i])) {  // dependent on the earlier images: drop it
        keep[i] = 0;
        HCK(x, hipMemsetAsync(zi, 0, n * sizeof(double2), st));
        continue;
      }
      R[(size_t)i * k + i] = nrm;
      const double inv = 1.0 / nrm;
      HCK(x, hipMemcpyAsync(binv, &inv, sizeof(double), hipMemcpyHostToDevice, st));
      HCK(x, launch_axpby(zi, n, zi, n, binv, nullptr, n, 1, nullptr, st));
    }
    // d = q^dag eta, back substitution R c = d over the kept columns
    HCK(x, launch_dots<double2>(z, n, n, k, eta + (int64_t)r * n, n, n, 1, part, coef, st));
    HCK(x, hipMemcpyAsync(hc.data(), coef, k * sizeof(double2), hipMemcpyDeviceToHost, st));
    HCK(x, hipStreamSynchronize(st));
    std::vector<double2> c(k, double2{0.0, 0.0});
    for (int i = k - 1; i >= 0; --i) {
      if (!keep[i]) continue;
      double sr = hc[i].x, si = hc[i].y;
      for (int j = i + 1; j < k; ++j) {
        if (!keep[j]) continue;
        const double2 a = Rc[(size_t)i * k + j], b = c[j];
        sr -= a.x * b.x - a.y * b.y;
        si -= a.x * b.y + a.y * b.x;
      }
      c[i] = double2{sr / R[(size_t)i * k + i], si / R[(size_t)i * k + i]};
    }
    HCK(x, hipMemcpyAsync(coef, c.data(), k * sizeof(double2), hipMemcpyHostToDevice, st));
    HCK(x, launch_axpy_multi<double2>(psi + (int64_t)r * n, n, ps, n, n, k, coef, k, 1.0, n, 1, nullptr, st));
    HCK(x, hipStreamSynchronize(st));  // the host copies of c, R are reused by the next rhs
  }
  return QDD_OK;
}

// the solutions of this solve into the history of their rhs slots (ring buffer)
static qdd_status chrono_store(qdd_ctx* x, int nrhs, const double2* psi, const qdd_solve_info* info) {
  const int nv = x->cfg.chrono_nv;
  const int64_t n = (int64_t)24 * x->G.Vh;
  double2* hist = x->ptr<double2>(x->lo.chrono);
  for (int r = 0; r < nrhs; ++r) {
    if (info && !info[r].converged) continue;
    int& h = x->chrono_head[r];
    HCK(x, hipMemcpyAsync(hist + ((int64_t)r * nv + h) * n, psi + (int64_t)r * n, n * sizeof(double2),
                          hipMemcpyDeviceToDevice, x->st));
    h = (h + 1) % nv;
    x->chrono_count[r] = std::min(x->chrono_count[r] + 1, nv);
  }
  return QDD_OK;
}

// the chronological guess itself (inspection): psi_c = sum_j c_j psi_j for the
// source eta_c from the stored solutions, without solving
extern "C" qdd_status qdd_chrono_guess(qdd_ctx* x, int nrhs, const double* eta_c, double* psi_c) {
  if (!x || !eta_c || !psi_c || nrhs < 1 || nrhs > x->cfg.max_nrhs || x->cfg.chrono_nv < 1) {
    if (x) x->fail("qdd_chrono_guess: invalid arguments (needs chrono_nv > 0)");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_chrono_guess before qdd_set_params"); return QDD_ESTATE; }
  double2 *eta = x->ptr<double2>(x->lo.eta), *psi = x->ptr<double2>(x->lo.psi);
  PackedView pe = x->packed(QDD_F64, nrhs, 0, eta);
  HCK(x, launch_pack_spinor<double>(x->G, eta_c, pe.f64, nrhs, 0, pe.poff, pe.spoff, x->st));
  qdd_status s = chrono_guess(x, nrhs, eta, psi);
  if (s != QDD_OK) return s;
  PackedView pp = x->packed(QDD_F64, nrhs, 0, psi);
  HCK(x, launch_unpack_spinor<double>(x->G, pp.f64, psi_c, nrhs, 0, pp.poff, pp.spoff, x->st));
  HCK(x, hipStreamSynchronize(x->st));
  return QDD_OK;
}

extern "C" qdd_status qdd_chrono_reset(qdd_ctx* x) {
  if (!x) return QDD_EINVAL;
  std::fill(x->chrono_count.begin(), x->chrono_count.end(), 0);
  std::fill(x->chrono_head.begin(), x->chrono_head.end(), 0);
  return QDD_OK;
}

qdd_status dfl_refresh_impl(qdd_ctx* x);

// guess: 0 start from 0 (or the chronological guess when configured), 1 psi_c holds
// the caller's initial guess
static qdd_status solve_impl(qdd_ctx* x, int nrhs, const double* eta_c, double* psi_c, qdd_solve_info* info,
                             int guess) {
  if (!x || !eta_c || !psi_c || nrhs < 1 || nrhs > x->cfg.max_nrhs) {
    if (x) x->fail("qdd_solve: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_solve before qdd_set_params"); return QDD_ESTATE; }
  if (x->cfg.precond == QDD_PRECOND_DFL && !x->have_dfl) {
    x->fail("deflated solve before qdd_dfl_build");
    return QDD_ESTATE;
  }
  const Layout& lo = x->lo;
  double2 *eta = x->ptr<double2>(lo.eta), *psi = x->ptr<double2>(lo.psi);
  PackedView pe = x->packed(QDD_F64, nrhs, 0, eta);
  HCK(x, launch_pack_spinor<double>(x->G, eta_c, pe.f64, nrhs, 0, pe.poff, pe.spoff, x->st));
  FgcrOps F;
  x->fallbacks.assign(nrhs, 0);
  x->coarse_iters = 0;
  qdd_status s0 = make_solver_ops(x, nrhs, F);
  if (s0 != QDD_OK) return s0;
  F.fallbacks = x->fallbacks.data();
  F.hv = x->harvest;
  const bool chrono = x->cfg.chrono_nv > 0 && !x->harvest;
  if (guess) {
    PackedView pg = x->packed(QDD_F64, nrhs, 0, psi);
    HCK(x, launch_pack_spinor<double>(x->G, psi_c, pg.f64, nrhs, 0, pg.poff, pg.spoff, x->st));
    F.warm = true;
  } else if (chrono) {
    s0 = chrono_guess(x, nrhs, eta, psi);
    if (s0 != QDD_OK) return s0;
    F.warm = true;
  }
  std::vector<qdd_solve_info> own(nrhs);
  qdd_solve_info* inf = info ? info : own.data();
  qdd_status s = run_fgcr(x, F, eta, psi, inf);
  PackedView pp = x->packed(QDD_F64, nrhs, 0, psi);
  HCK(x, launch_unpack_spinor<double>(x->G, pp.f64, psi_c, nrhs, 0, pp.poff, pp.spoff, x->st));
  if (chrono && (s == QDD_OK || s == QDD_ENOCONV)) {
    qdd_status sc = chrono_store(x, nrhs, psi, inf);
    if (sc != QDD_OK) return sc;
  }
  HCK(x, hipStreamSynchronize(x->st));
  // refresh the deflation subspace when this solve took too many iterations
  if ((s == QDD_OK || s == QDD_ENOCONV) && x->cfg.precond == QDD_PRECOND_DFL && x->cfg.dfl_refresh_iters > 0 &&
      !x->harvest) {
    int mx = 0;
    for (int r = 0; r < nrhs; ++r) mx = std::max(mx, inf[r].iters);
    if (mx > x->cfg.dfl_refresh_iters) {
      qdd_status sr = dfl_refresh_impl(x);
      if (sr != QDD_OK) return sr;
    }
  }
  return s;
}

extern "C" qdd_status qdd_solve(qdd_ctx* x, int nrhs, const double* eta_c, double* psi_c, qdd_solve_info* info) {
  return solve_impl(x, nrhs, eta_c, psi_c, info, 0);
}

// psi_c holds the initial guess on entry
extern "C" qdd_status qdd_solve_guess(qdd_ctx* x, int nrhs, const double* eta_c, double* psi_c,
                                      qdd_solve_info* info) {
  return solve_impl(x, nrhs, eta_c, psi_c, info, 1);
}

// W(dm_r)^{-1} phi_r for nrhs even fields (Eq. 3; dm_r = 0 gives Q_S^{-1} phi_r,
// Eq. 5).  W = Q_S + dm = A_e^{-1} (Dhat + dm A_e), and Dhat + dm A_e is the Schur
// complement of D' = D with the even sites' clover term scaled by 1 + dm, so
// W^{-1} phi = [D'^{-1} (A_e phi (+) 0)]_e: flexible GCR on D' (FP64) with the
// configured preconditioner, which is built for D, and the even half of the
// solution.  The residual that counts is that of W: phi - W x is formed with the
// FP64 Dhat, the even-site inverse clover blocks and the shift, and where it is
// above tol |phi| the same solve is run on it and the correction added (at most
// two such passes).  Since the W residual is a few times the D' residual, the
// first pass stops at tol / 5 and a correction pass only at the reduction its
// residual still needs (with the same margin).  info[r]: iterations of all
// passes, the W residual.
static qdd_status solve_w_impl(qdd_ctx* x, int nrhs, const double* dm, const double* const* phi, double* const* out,
                               qdd_solve_info* info) {
  const Layout& lo = x->lo;
  const Geo& G = x->G;
  hipStream_t st = x->st;
  const int64_t n = (int64_t)24 * G.Vh, ne = (int64_t)12 * G.Vh;
  const double tol = x->cfg.tol;
  double2 *eta = x->ptr<double2>(lo.eta), *psi = x->ptr<double2>(lo.psi);
  double* ce = x->ptr<double>(lo.dw_ce);
  // scratch: canonical residuals and one W image in the Krylov space (consumed
  // before each solve overwrites it), one packed even field and its W image in
  // t64 / res, canonical corrections in s_tmp
  double2* resc = x->ptr<double2>(lo.chi);
  double2* wxc = resc + (int64_t)nrhs * ne;
  double2* xe = x->ptr<double2>(lo.t64);
  double2* we = x->ptr<double2>(lo.res);
  double2* corr = x->ptr<double2>(lo.s_tmp);
  double2 *part = x->ptr<double2>(lo.part), *rn2 = x->ptr<double2>(lo.rn2);
  const CloverV<double> A = x->op<double>().A, Ai = x->op<double>().Ainv;
  std::vector<double> ceh(nrhs), pn(nrhs), rn(nrhs);
  for (int r = 0; r < nrhs; ++r) ceh[r] = 1.0 + dm[r];
  HCK(x, hipMemcpyAsync(ce, ceh.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
  std::vector<double2> h2(nrhs);
  for (int r = 0; r < nrhs; ++r)
    HCK(x, launch_dots<double2>((const double2*)phi[r], 0, ne, 1, (const double2*)phi[r], ne, ne, 1, part, rn2 + r, st));
  HCK(x, hipMemcpyAsync(h2.data(), rn2, nrhs * sizeof(double2), hipMemcpyDeviceToHost, st));
  HCK(x, hipStreamSynchronize(st));
  for (int r = 0; r < nrhs; ++r) pn[r] = std::sqrt(h2[r].x);
  std::vector<int> need(nrhs, 1), iters(nrhs, 0), restarts(nrhs, 0), fallbacks(nrhs, 0);
  std::vector<qdd_solve_info> pi(nrhs);
  double t_ms = 0.0, pass_tol = 0.2 * tol;
  qdd_status solve_status = QDD_OK;
  struct TolGuard {  // the outer solver reads its tolerance from the configuration
    qdd_ctx* x;
    double keep;
    ~TolGuard() { x->cfg.tol = keep; }
  } guard{x, x->cfg.tol};
  for (int pass = 0; pass < 3; ++pass) {
    x->cfg.tol = pass_tol;
    // source: A_e rho_r on the even sites, 0 on the odd ones (rho = phi, then the
    // W residual; zero for the right-hand sides that need no correction)
    HCK(x, hipMemsetAsync(eta, 0, (size_t)nrhs * n * sizeof(double2), st));
    PackedView pe = x->packed(QDD_F64, nrhs, 0, eta);
    for (int r = 0; r < nrhs; ++r)
      if (need[r]) {
        FieldV<double> er = pe.f64;
        er.p += r * er.rs;
        HCK(x, launch_qs_source(G, pass == 0 ? phi[r] : (const double*)(resc + r * ne), er, A, 1, st));
      }
    FgcrOps F;
    x->fallbacks.assign(nrhs, 0);
    x->coarse_iters = 0;
    qdd_status s0 = make_solver_ops(x, nrhs, F);
    if (s0 != QDD_OK) return s0;
    F.op = [x, nrhs, ce](const double2* in, double2* o) -> qdd_status {
      HCK(x, x->dw(QDD_F64, nrhs, (void*)in, o, ce));
      return QDD_OK;
    };
    F.fallbacks = x->fallbacks.data();
    F.hv = nullptr;
    qdd_status s = run_fgcr(x, F, eta, psi, pi.data());
    if (s != QDD_OK && s != QDD_ENOCONV) return s;
    if (s == QDD_ENOCONV) solve_status = s;
    for (int r = 0; r < nrhs; ++r) {
      iters[r] += pi[r].iters;
      restarts[r] += pi[r].restarts;
      fallbacks[r] += pi[r].fallbacks;
    }
    t_ms += pi[0].t_ms[0];
    // the even half of the solution becomes (pass 0) or corrects the result
    PackedView pp = x->packed(QDD_F64, nrhs, 0, psi);
    for (int r = 0; r < nrhs; ++r) {
      if (!need[r]) continue;
      FieldV<double> v = pp.f64;
      v.p += r * v.rs;
      if (pass == 0) {
        HCK(x, launch_unpack_spinor<double>(G, v, out[r], 1, 1, pp.poff, pp.spoff, st));
      } else {
        HCK(x, launch_unpack_spinor<double>(G, v, (double*)(corr + r * ne), 1, 1, pp.poff, pp.spoff, st));
        HCK(x, launch_add<double2>((double2*)out[r], corr + r * ne, 1.0, ne, st));
      }
    }
    // W residual phi - W(dm) x
    PackedView px = x->packed(QDD_F64, 1, 1, xe), pw = x->packed(QDD_F64, 1, 1, we);
    for (int r = 0; r < nrhs; ++r) {
      HCK(x, launch_pack_spinor<double>(G, out[r], px.f64, 1, 1, px.poff, px.spoff, st));
      HCK(x, x->dhat(QDD_F64, 1, xe, we));
      HCK(x, launch_apply_w_finish(G, px.f64, pw.f64, Ai, 1, dm[r], st));
      HCK(x, launch_unpack_spinor<double>(G, pw.f64, (double*)wxc, 1, 1, pw.poff, pw.spoff, st));
      HCK(x, launch_sub(resc + r * ne, (const double2*)phi[r], wxc, ne, ne, 1, st));
    }
    HCK(x, launch_dots<double2>(resc, 0, ne, 1, resc, ne, ne, nrhs, part, rn2, st));
    HCK(x, hipMemcpyAsync(h2.data(), rn2, nrhs * sizeof(double2), hipMemcpyDeviceToHost, st));
    HCK(x, hipStreamSynchronize(st));
    bool any = false;
    pass_tol = 0.5;
    for (int r = 0; r < nrhs; ++r) {
      rn[r] = std::sqrt(std::fabs(h2[r].x));
      need[r] = !(rn[r] <= tol * pn[r]) && std::isfinite(h2[r].x);
      any |= need[r] != 0;
      if (need[r]) pass_tol = std::min(pass_tol, 0.2 * tol * pn[r] / rn[r]);
    }
    if (!any) break;
  }
  qdd_status status = QDD_OK;
  for (int r = 0; r < nrhs; ++r) {
    const bool conv = pn[r] > 0 ? rn[r] <= tol * pn[r] : true;
    if (!conv) status = QDD_ENOCONV;
    if (info) {
      info[r] = pi[r];
      info[r].iters = iters[r];
      info[r].restarts = restarts[r];
      info[r].fallbacks = fallbacks[r];
      info[r].converged = conv;
      info[r].true_res = pn[r] > 0 ? rn[r] / pn[r] : 0.0;
      info[r].t_ms[0] = t_ms;
    }
  }
  if (status != QDD_OK)
    x->fail(solve_status != QDD_OK ? "no convergence within nmx iterations" : "W residual above tol after refinement");
  return status;
}

static qdd_status solve_w_check(qdd_ctx* x, int nrhs, const char* name) {
  if (!x->have_clover) { x->fail("%s before qdd_set_params", name); return QDD_ESTATE; }
  if (x->cfg.precond == QDD_PRECOND_DFL && !x->have_dfl) {
    x->fail("%s: deflated solve before qdd_dfl_build", name);
    return QDD_ESTATE;
  }
  (void)nrhs;
  return QDD_OK;
}

// Q_S^{-1} phi = P_e Q^{-1} Q_ee P_e phi (Eq. 5)
extern "C" qdd_status qdd_solve_qs(qdd_ctx* x, int nrhs, const double* phi_c, double* out_c, qdd_solve_info* info) {
  if (!x || !phi_c || !out_c || nrhs < 1 || nrhs > x->cfg.max_nrhs) {
    if (x) x->fail("qdd_solve_qs: invalid arguments");
    return QDD_EINVAL;
  }
  qdd_status s = solve_w_check(x, nrhs, "qdd_solve_qs");
  if (s != QDD_OK) return s;
  const int64_t ne = (int64_t)24 * x->G.Vh;  // doubles per canonical even field
  std::vector<const double*> ph(nrhs);
  std::vector<double*> o(nrhs);
  std::vector<double> dm(nrhs, 0.0);
  for (int r = 0; r < nrhs; ++r) {
    ph[r] = phi_c + r * ne;
    o[r] = out_c + r * ne;
  }
  return solve_w_impl(x, nrhs, dm.data(), ph.data(), o.data(), info);
}

// W(dm)^{-1} phi (Eq. 3)
extern "C" qdd_status qdd_solve_w(qdd_ctx* x, int nrhs, double dm, const double* phi_c, double* out_c,
                                  qdd_solve_info* info) {
  if (!x || !phi_c || !out_c || nrhs < 1 || nrhs > x->cfg.max_nrhs || !std::isfinite(dm) || dm < 0) {
    if (x) x->fail("qdd_solve_w: invalid arguments");
    return QDD_EINVAL;
  }
  qdd_status s = solve_w_check(x, nrhs, "qdd_solve_w");
  if (s != QDD_OK) return s;
  const int64_t ne = (int64_t)24 * x->G.Vh;
  std::vector<const double*> ph(nrhs);
  std::vector<double*> o(nrhs);
  std::vector<double> dms(nrhs, dm);
  for (int r = 0; r < nrhs; ++r) {
    ph[r] = phi_c + r * ne;
    o[r] = out_c + r * ne;
  }
  return solve_w_impl(x, nrhs, dms.data(), ph.data(), o.data(), info);
}

// S_eff of Eq. 4 with two pseudofermions: -2 (log det Q_ee + log det Q_oo)
// + |W^{-1}(dm) phi1|^2 + |(1 + dm Q_S^{-1}) phi2|^2; the two solves run as one
// batch of two right-hand sides (masses dm and 0)
extern "C" qdd_status qdd_action(qdd_ctx* x, double dm, const double* phi1, const double* phi2, double* chi1,
                                 double* chi2, double* s_eff, double* parts, qdd_solve_info* info) {
  if (!x || !phi1 || !phi2 || !chi1 || !chi2 || !s_eff || !std::isfinite(dm) || dm < 0 || x->cfg.max_nrhs < 2 ||
      chi1 == chi2) {
    if (x) x->fail("qdd_action: invalid arguments (max_nrhs must be >= 2)");
    return QDD_EINVAL;
  }
  qdd_status s = solve_w_check(x, 2, "qdd_action");
  if (s != QDD_OK) return s;
  double le = 0, lo_ = 0;
  s = qdd_clover_logdet(x, &le, &lo_);
  if (s != QDD_OK) return s;
  const double dms[2] = {dm, 0.0};
  const double* ph[2] = {phi1, phi2};
  double* o[2] = {chi1, chi2};
  s = solve_w_impl(x, 2, dms, ph, o, info);
  if (s != QDD_OK) return s;
  // |chi1|^2 and |phi2 + dm chi2|^2 (the sum formed in the correction scratch)
  const int64_t ne = (int64_t)12 * x->G.Vh;
  hipStream_t st = x->st;
  double2* tmp = x->ptr<double2>(x->lo.s_tmp);
  double2 *part = x->ptr<double2>(x->lo.part), *rn2 = x->ptr<double2>(x->lo.rn2);
  HCK(x, hipMemcpyAsync(tmp, phi2, ne * sizeof(double2), hipMemcpyDeviceToDevice, st));
  HCK(x, launch_add<double2>(tmp, (const double2*)chi2, dm, ne, st));
  HCK(x, launch_dots<double2>((const double2*)chi1, 0, ne, 1, (const double2*)chi1, ne, ne, 1, part, rn2, st));
  HCK(x, launch_dots<double2>(tmp, 0, ne, 1, tmp, ne, ne, 1, part, rn2 + 1, st));
  double2 h[2];
  HCK(x, hipMemcpyAsync(h, rn2, sizeof(h), hipMemcpyDeviceToHost, st));
  HCK(x, hipStreamSynchronize(st));
  const double t0 = -2.0 * (le + lo_), t1 = h[0].x, t2 = h[1].x;
  if (parts) {
    parts[0] = t0;
    parts[1] = t1;
    parts[2] = t2;
  }
  *s_eff = t0 + t1 + t2;
  return QDD_OK;
}

// Forces of S_eff (Eq. 4; the molecular-dynamics forces of Sect. 2).  With
// W(s) = A_e^{-1} (Dhat + s A_e), a pseudofermion term -2c Re[X^dag d(Dhat + s A_e) Y
// - X^dag dA_e phi] has Y = W^{-1} phi (psi for phi1 with s = dm, c = 1; xi for phi2
// with s = 0, c = dm) and X = (Dhat + s A_e)^{-dag} w, w = psi or phi2 + dm xi,
// computed as g5 W(s)^{-1} A_e^{-1} g5 w (Dhat + s A_e is g5-Hermitian and A_e
// commutes with g5).  Both solves of each kind run as one batch of two.
extern "C" qdd_status qdd_force(qdd_ctx* x, double dm, const double* phi1, const double* phi2, int terms,
                                double* force, qdd_solve_info* info) {
  if (!x || !force || terms < 1 || terms > 7 || !std::isfinite(dm) || dm < 0 || !x->cfg.force ||
      ((terms & 6) && (!phi1 || !phi2 || x->cfg.max_nrhs < 2))) {
    if (x) x->fail("qdd_force: invalid arguments (needs config.force = 1; max_nrhs >= 2 for the pseudofermion terms)");
    return QDD_EINVAL;
  }
  if (!x->have_clover) {
    x->fail("qdd_force before qdd_set_params");
    return QDD_ESTATE;
  }
  const int64_t Vh = x->G.Vh, ts = 2 * 12 * Vh;  // complex entries of one term's full field
  double2 *fx = x->ptr<double2>(x->lo.frc_x), *fy = x->ptr<double2>(x->lo.frc_y);
  double2* src = x->ptr<double2>(x->lo.frc_src);
  hipStream_t st = x->st;
  const DevOp<double> op = x->op<double>();
  FrcTerms T;
  if (info)
    for (int r = 0; r < 4; ++r) info[r] = qdd_solve_info{};
  if (terms & 6) {
    qdd_status s = solve_w_check(x, 2, "qdd_force");
    if (s != QDD_OK) return s;
    const double dms[2] = {dm, 0.0};
    const double* ph[2] = {phi1, phi2};
    double* y[2] = {(double*)fy, (double*)(fy + ts)};
    s = solve_w_impl(x, 2, dms, ph, y, info);
    if (s != QDD_OK) return s;
    HCK(x, launch_force_src(x->G, op, fy, fy + ts, (const double2*)phi2, dm, src, st));
    const double* us[2] = {(const double*)src, (const double*)(src + 12 * Vh)};
    double* z[2] = {(double*)fx, (double*)(fx + ts)};
    s = solve_w_impl(x, 2, dms, us, z, info ? info + 2 : nullptr);
    if (s != QDD_OK) return s;
    HCK(x, launch_force_odd(x->G, op, 2, fx, fy, st));
    for (int t = 0; t < 2; ++t) {
      const bool on = t == 0 ? (terms & 2) != 0 : ((terms & 4) != 0 && dm != 0.0);
      if (!on) continue;
      T.X[T.nt] = fx + t * ts;
      T.Y[T.nt] = fy + t * ts;
      T.phi[T.nt] = (const double2*)(t == 0 ? phi1 : phi2);
      T.c[T.nt] = t == 0 ? 1.0 : dm;
      T.s[T.nt] = t == 0 ? dm : 0.0;
      ++T.nt;
    }
  }
  HCK(x, launch_force(x->G, op, x->ptr<double2>(x->lo.U[0]), (terms & 1) ? -2.0 : 0.0, x->csw, T,
                      x->ptr<double>(x->lo.frc_lt), force, st));
  HCK(x, hipStreamSynchronize(st));
  return QDD_OK;
}

// Plain solve of one right-hand side that records a (residual, error) pair at
// every outer iteration: r_k = eta - D psi_k (the recursive residual) and
// e_k = psi* - psi_k, both returned as packed FP32 full fields (training data of
// the network stage).  The e buffer needs FP64-sized slots: the iterates are kept
// in FP64 until psi* is known, so that the small errors keep their precision.
extern "C" qdd_status qdd_solve_harvest(qdd_ctx* x, int nrhs, const double* eta_c, double* psi_c,
                                        qdd_solve_info* info, void* r_pairs, void* e_pairs, int max_pairs,
                                        int* npairs, int* pair_rhs) {
  if (!x || !r_pairs || !e_pairs || max_pairs < 1 || !npairs) {
    if (x) x->fail("qdd_solve_harvest: invalid arguments");
    return QDD_EINVAL;
  }
  Harvest hv;
  hv.r = (float2*)r_pairs;
  hv.e = e_pairs;
  hv.max = max_pairs;
  x->harvest = &hv;
  qdd_status s = qdd_solve(x, nrhs, eta_c, psi_c, info);
  x->harvest = nullptr;
  *npairs = hv.n;
  if (pair_rhs)
    for (int j = 0; j < hv.n; ++j) pair_rhs[j] = hv.rhs[j];
  return s;
}

// ------------------------------------------------------------------ several systems at once
// Solves nsys independent systems (different lattices, masses, batch sizes):
// every context runs its flexible GCR on its own host thread and its own
// stream, so the kernels of all systems are in flight together and each system
// stops at its own convergence.  info[s] points at nrhs[s] entries (or NULL).
#include <thread>
extern "C" qdd_status qdd_solve_multi(qdd_ctx* const* ctxs, int nsys, const int* nrhs, const double* const* eta,
                                      double* const* psi, qdd_solve_info* const* info) {
  if (!ctxs || nsys < 1 || !nrhs || !eta || !psi) return QDD_EINVAL;
  for (int s = 0; s < nsys; ++s)
    for (int q = s + 1; q < nsys; ++q)
      if (ctxs[s] == ctxs[q] || (ctxs[s]->st == ctxs[q]->st && ctxs[s]->st != nullptr)) {
        ctxs[s]->fail("qdd_solve_multi: every system needs its own context and stream");
        return QDD_EINVAL;
      }
  std::vector<qdd_status> st(nsys, QDD_OK);
  std::vector<std::thread> th;
  for (int s = 0; s < nsys; ++s)
    th.emplace_back([&, s]() { st[s] = qdd_solve(ctxs[s], nrhs[s], eta[s], psi[s], info ? info[s] : nullptr); });
  for (auto& t : th) t.join();
  for (int s = 0; s < nsys; ++s)
    if (st[s] != QDD_OK) return st[s];
  return QDD_OK;
}
