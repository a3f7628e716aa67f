// Several independent systems (lattices, masses, batch sizes) solved together by
// the outer flexible GCR of the paper's Schwarz-preconditioned solver (Sect. 3),
// with every stage of an iteration issued as ONE launch over the workgroups of
// all systems that take part in it: the Schwarz face and half-sweep kernels, the
// full D, the precision conversions and each Gram-Schmidt reduction and update
// (Grp tables, qdd_kernels.h: workgroup -> (system, own workgroup number)).  The
// systems advance in lockstep through the steps of a restart cycle; a system
// whose right-hand sides have all converged (recursive residual), or that used up
// its cycle length or iteration limit, drops out of the tables until the cycle
// ends, and per-rhs masks on the device keep converged right-hand sides of a
// running system from being updated.  Every system computes exactly the
// arithmetic of its own qdd_solve (same kernels, same partial-sum blocking, same
// host back substitution), so the results agree bit for bit; what changes is
// that the small lattices fill the chip together with the large ones and that
// one host thread issues one launch per stage instead of one per system.
#include "qdd_api_internal.h"
#include "qdd_solver.h"
#include "qdd_sap.h"

#include <chrono>
#include <cmath>
#include <string>
#include <vector>

using namespace qdd;

namespace {

struct Sys {
  qdd_ctx* x;
  int nr;
  int64_t n;       // complex numbers per right-hand side (full field)
  int64_t lstride;  // between Krylov vectors
  double2 *eta, *psi, *r, *t, *chi, *part, *coef, *ahist, *chist, *rn2, *alpha;
  double *bhist, *binv;
  int* active;
  void* phi;
  bool phi32;
  std::vector<double> etan, rn;
  std::vector<int> act, conv, iters, restarts, ks;
  int total_it = 0, kk = 0;
  bool done = false, nonfinite = false;
  std::vector<double2> h2;
  void* phi_k(int k) const { return (char*)phi + (size_t)k * lstride * (phi32 ? 8 : 16); }
  double2* chi_k(int k) const { return chi + (size_t)k * lstride; }
};

// why the systems cannot be grouped ("" if they can)
std::string group_check(qdd_ctx* const* xs, int ns, const int* nrhs) {
  if (ns < 1 || ns > kGrpMax) return "1 to " + std::to_string(kGrpMax) + " systems";
  const qdd_ctx* a = xs[0];
  for (int s = 0; s < ns; ++s) {
    const qdd_ctx* x = xs[s];
    if (!x) return "null context";
    for (int q = 0; q < s; ++q)
      if (xs[q] == x) return "a context appears twice";
    if (!x->have_clover) return "a context has no qdd_set_params";
    if (nrhs[s] < 1 || nrhs[s] > x->cfg.max_nrhs) return "nrhs out of range";
    if (x->device != a->device) return "contexts on different devices";
    if (x->cfg.precond != a->cfg.precond) return "contexts with different preconditioners";
    if (x->cfg.precond != QDD_PRECOND_NONE && x->cfg.precond != QDD_PRECOND_SAP)
      return "grouped solves take the Schwarz preconditioner or none";
    if (x->cfg.precond == QDD_PRECOND_SAP) {
      if (x->cfg.sap_prec == QDD_F64) return "grouped Schwarz solves run with FP32 or FP16 storage";
      if (x->cfg.sap_prec != a->cfg.sap_prec) return "Schwarz storage precisions differ";
      const int* b = x->cfg.sap_bs;
      const int* b0 = a->cfg.sap_bs;
      if (b[0] * b[1] * b[2] * b[3] != b0[0] * b0[1] * b0[2] * b0[3]) return "Schwarz blocks of different volumes";
      const int p = x->cfg.sap_prec;
      const int v = x->sap_variant[p] ? x->sap_variant[p] : sap_default_variant(p);
      const int v0 = a->sap_variant[p] ? a->sap_variant[p] : sap_default_variant(p);
      if (v != v0) return "different Schwarz kernel variants";
    }
    if (x->lo.phi32 != a->lo.phi32) return "different preconditioner output precisions";
    if (x->cfg.chrono_nv > 0) return "chronological inversion is per context (chrono_nv must be 0)";
    if (x->harvest) return "pair capture is per context";
  }
  return "";
}

}  // namespace

extern "C" qdd_status qdd_solve_group(qdd_ctx* const* ctxs, int nsys, const int* nrhs, const double* const* eta_c,
                                      double* const* psi_c, qdd_solve_info* const* info) {
  if (!ctxs || nsys < 1 || !nrhs || !eta_c || !psi_c || !ctxs[0]) return QDD_EINVAL;
  const std::string why = group_check(ctxs, nsys, nrhs);
  if (!why.empty()) {
    ctxs[0]->fail("qdd_solve_group: %s", why.c_str());
    return QDD_EINVAL;
  }
  for (int s = 0; s < nsys; ++s)
    if (!eta_c[s] || !psi_c[s]) {
      ctxs[0]->fail("qdd_solve_group: null field");
      return QDD_EINVAL;
    }
  qdd_ctx* x0 = ctxs[0];
  hipStream_t st = x0->st;
  // work queued on the other contexts' streams (their set-up) precedes the group
  for (int s = 1; s < nsys; ++s) HCK(ctxs[s], hipStreamSynchronize(ctxs[s]->st));
  const auto t0 = std::chrono::steady_clock::now();
  double tstage[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  StageEvents ev;
  HCK(x0, ev.init());
  auto tic = []() { return std::chrono::steady_clock::now(); };
  auto since = [](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
  };

  std::vector<Sys> S(nsys);
  for (int s = 0; s < nsys; ++s) {
    Sys& y = S[s];
    qdd_ctx* x = ctxs[s];
    const Layout& lo = x->lo;
    y.x = x;
    y.nr = nrhs[s];
    y.n = (int64_t)24 * x->G.Vh;
    y.lstride = (int64_t)y.nr * y.n;
    y.eta = x->ptr<double2>(lo.eta);
    y.psi = x->ptr<double2>(lo.psi);
    y.r = x->ptr<double2>(lo.res);
    y.t = x->ptr<double2>(lo.t64);
    y.chi = x->ptr<double2>(lo.chi);
    y.phi = x->ptr<void>(lo.phi);
    y.phi32 = lo.phi32;
    y.part = x->ptr<double2>(lo.part);
    y.coef = x->ptr<double2>(lo.coef);
    y.ahist = x->ptr<double2>(lo.ahist);
    y.chist = x->ptr<double2>(lo.chist);
    y.rn2 = x->ptr<double2>(lo.rn2);
    y.alpha = x->ptr<double2>(lo.alpha);
    y.bhist = x->ptr<double>(lo.bhist);
    y.binv = x->ptr<double>(lo.binv);
    y.active = x->ptr<int>(lo.active);
    y.etan.assign(y.nr, 0.0);
    y.rn.assign(y.nr, 0.0);
    y.act.assign(y.nr, 0);
    y.conv.assign(y.nr, 0);
    y.iters.assign(y.nr, 0);
    y.restarts.assign(y.nr, 0);
    y.ks.assign(y.nr, 0);
    y.h2.assign(y.nr, double2{0.0, 0.0});
    PackedView pe = x->packed(QDD_F64, y.nr, 0, y.eta);
    HCK(x0, launch_pack_spinor<double>(x->G, eta_c[s], pe.f64, y.nr, 0, pe.poff, pe.spoff, st));
  }
  // the launch shape of the full D: that of the largest system (its tuned shape)
  int big = 0;
  for (int s = 1; s < nsys; ++s)
    if (ctxs[s]->G.V > ctxs[big]->G.V) big = s;
  const LaunchCfg dcfg = ctxs[big]->launch[1][QDD_F64];

  // ---- grouped stages over a list of systems
  auto dots = [&](const std::vector<int>& L, auto xa, int m, auto ya, auto out) -> qdd_status {
    std::vector<DotsArgs<double2>> a;
    for (int s : L) {
      const Sys& y = S[s];
      a.push_back(DotsArgs<double2>{xa(y).first, xa(y).second, y.n, m, ya(y), y.n, y.n, y.nr, 0, y.part, out(y)});
    }
    HCK(x0, launch_dots_grp<double2>(a.data(), (int)a.size(), st));
    return QDD_OK;
  };
  auto fetch_rn2 = [&](const std::vector<int>& L) -> qdd_status {
    for (int s : L)
      HCK(x0, hipMemcpyAsync(S[s].h2.data(), S[s].rn2, S[s].nr * sizeof(double2), hipMemcpyDeviceToHost, st));
    HCK(x0, hipStreamSynchronize(st));
    return QDD_OK;
  };
  // out[s] = D in[s] (FP64)
  auto apply_d = [&](const std::vector<int>& L, double2* Sys::*in, double2* Sys::*out) -> qdd_status {
    std::vector<DwArgs<double>> a;
    for (int s : L) {
      const Sys& y = S[s];
      PackedView pi = y.x->packed(QDD_F64, y.nr, 0, y.*in), po = y.x->packed(QDD_F64, y.nr, 0, y.*out);
      const DevOp<double> op = y.x->op<double>();
      a.push_back(DwArgs<double>{y.x->G, op.U, op.A, pi.f64, po.f64, pi.poff, pi.spoff, y.nr, 0, 0, 0});
    }
    HCK(x0, launch_dw_grp<double>(a.data(), (int)a.size(), dcfg, st));
    return QDD_OK;
  };
  auto r_sqnorm = [&](const std::vector<int>& L) -> qdd_status {
    return dots(
        L, [](const Sys& y) { return std::make_pair((const double2*)y.r, (int64_t)0); }, 1,
        [](const Sys& y) { return (const double2*)y.r; }, [](const Sys& y) { return y.rn2; });
  };

  // |eta|, psi = 0, r = eta
  std::vector<int> all(nsys);
  for (int s = 0; s < nsys; ++s) all[s] = s;
  {
    qdd_status q = dots(
        all, [](const Sys& y) { return std::make_pair((const double2*)y.eta, (int64_t)0); }, 1,
        [](const Sys& y) { return (const double2*)y.eta; }, [](const Sys& y) { return y.rn2; });
    if (q != QDD_OK) return q;
    for (Sys& y : S) {
      HCK(x0, hipMemsetAsync(y.psi, 0, (size_t)y.nr * y.n * sizeof(double2), st));
      HCK(x0, hipMemcpyAsync(y.r, y.eta, (size_t)y.nr * y.n * sizeof(double2), hipMemcpyDeviceToDevice, st));
    }
    q = fetch_rn2(all);
    if (q != QDD_OK) return q;
    for (Sys& y : S) {
      for (int i = 0; i < y.nr; ++i) {
        y.etan[i] = std::sqrt(y.h2[i].x);
        y.rn[i] = y.etan[i];
        y.conv[i] = !(y.etan[i] > 0);
        y.act[i] = !y.conv[i];
      }
    }
  }
  auto any_of = [](const std::vector<int>& v) {
    for (int a : v)
      if (a) return true;
    return false;
  };

  std::vector<double2> ah, chh, al;
  std::vector<double> bh;
  while (true) {
    // the systems that run a restart cycle
    std::vector<int> live;
    for (int s = 0; s < nsys; ++s) {
      Sys& y = S[s];
      if (!y.done && any_of(y.act) && y.total_it < y.x->cfg.nmx) live.push_back(s);
      else y.done = true;
    }
    if (live.empty()) break;
    for (int s : live) {
      Sys& y = S[s];
      HCK(x0, hipMemcpyAsync(y.active, y.act.data(), y.nr * sizeof(int), hipMemcpyHostToDevice, st));
      std::fill(y.ks.begin(), y.ks.end(), 0);
      y.kk = 0;
    }
    std::vector<int> run = live;
    for (int k = 0; !run.empty(); ++k) {
      // phi_k = M(r)
      auto ta = tic();
      HCK(x0, ev.mark(0, st));
      if (ctxs[0]->cfg.precond == QDD_PRECOND_SAP) {
        std::vector<qdd_ctx*> xs;
        std::vector<int> nr;
        std::vector<const double2*> e;
        std::vector<void*> p;
        for (int s : run) {
          xs.push_back(S[s].x);
          nr.push_back(S[s].nr);
          e.push_back(S[s].r);
          p.push_back(S[s].phi_k(k));
        }
        qdd_status q = sap_apply_grp(xs.data(), nr.data(), e.data(), p.data(), (int)run.size(), st);
        if (q != QDD_OK) return q;
      } else {
        for (int s : run)
          HCK(x0, hipMemcpyAsync(S[s].phi_k(k), S[s].r, (size_t)S[s].nr * S[s].n * sizeof(double2),
                                 hipMemcpyDeviceToDevice, st));
      }
      tstage[1] += since(ta);
      HCK(x0, ev.mark(1, st));
      ta = tic();
      // chi_k = D phi_k (FP64; an FP32 phi converted first)
      {
        std::vector<DwArgs<double>> a;
        std::vector<FieldV<float>> cin;
        std::vector<FieldV<double>> cout;
        std::vector<int> nv;
        for (int s : run) {
          const Sys& y = S[s];
          void* src = y.phi_k(k);
          if (y.phi32) {
            cin.push_back(FieldV<float>{(float2*)src, nullptr, y.n, y.n, (int)(y.n / 12)});
            cout.push_back(FieldV<double>{y.t, nullptr, y.n, y.n, (int)(y.n / 12)});
            nv.push_back(y.nr);
            src = y.t;
          }
          PackedView pi = y.x->packed(QDD_F64, y.nr, 0, src), po = y.x->packed(QDD_F64, y.nr, 0, y.chi_k(k));
          const DevOp<double> op = y.x->op<double>();
          a.push_back(DwArgs<double>{y.x->G, op.U, op.A, pi.f64, po.f64, pi.poff, pi.spoff, y.nr, 0, 0, 0});
        }
        if (!cin.empty())
          HCK(x0, launch_field_convert_grp<float, double>(cin.data(), cout.data(), nv.data(), (int)cin.size(), st));
        HCK(x0, launch_dw_grp<double>(a.data(), (int)a.size(), dcfg, st));
      }
      tstage[2] += since(ta);
      HCK(x0, ev.mark(2, st));
      ta = tic();
      // Gram-Schmidt against chi_0 .. chi_{k-1}, two passes, then normalise
      {
        std::vector<CoefArgs> c;
        for (int s : run) {
          const Sys& y = S[s];
          c.push_back(CoefArgs{y.ahist + (size_t)k * y.nr * kMaxKv, kMaxKv, nullptr, 0, nullptr, nullptr, nullptr,
                               y.nr});
        }
        HCK(x0, launch_coef_grp(c.data(), (int)c.size(), 0, st));
        // the update sweeps also form the next inner products (as in the
        // single-system solver, the same sums as separate launches)
        auto upd = [&](auto fill) {
          std::vector<UpdArgs> u;
          for (int s : run) u.push_back(fill(S[s]));
          return u;
        };
        qdd_status q = QDD_OK;
        if (k > 0) {
          q = dots(
              run, [](const Sys& y) { return std::make_pair((const double2*)y.chi, y.lstride); }, k,
              [k](const Sys& y) { return (const double2*)y.chi_k(k); }, [](const Sys& y) { return y.coef; });
          if (q != QDD_OK) return q;
          for (size_t j = 0; j < run.size(); ++j) {
            const Sys& y = S[run[j]];
            c[j] = CoefArgs{y.ahist + (size_t)k * y.nr * kMaxKv, kMaxKv, y.coef, k, nullptr, nullptr, nullptr, y.nr};
          }
          HCK(x0, launch_coef_grp(c.data(), (int)c.size(), 2, st));
          auto u0 = upd([k](const Sys& y) {
            return UpdArgs{y.chi_k(k), y.n, y.chi, y.lstride, y.n, k, y.coef, k, nullptr, nullptr, nullptr, 0,
                           y.n, y.nr, 0, y.part, y.coef};
          });
          HCK(x0, launch_sub_dots_grp(u0.data(), (int)u0.size(), 0, st));
          HCK(x0, launch_coef_grp(c.data(), (int)c.size(), 2, st));
          auto u1 = upd([k](const Sys& y) {
            return UpdArgs{y.chi_k(k), y.n, y.chi, y.lstride, y.n, k, y.coef, k, nullptr, nullptr, nullptr, 0,
                           y.n, y.nr, 0, y.part, y.rn2};
          });
          HCK(x0, launch_sub_dots_grp(u1.data(), (int)u1.size(), 1, st));
        } else {
          q = dots(
              run, [k](const Sys& y) { return std::make_pair((const double2*)y.chi_k(k), (int64_t)0); }, 1,
              [k](const Sys& y) { return (const double2*)y.chi_k(k); }, [](const Sys& y) { return y.rn2; });
          if (q != QDD_OK) return q;
        }
        for (size_t j = 0; j < run.size(); ++j) {
          const Sys& y = S[run[j]];
          c[j] = CoefArgs{nullptr, 0, nullptr, 0, y.rn2, y.bhist + (size_t)k * y.nr, y.binv, y.nr};
        }
        HCK(x0, launch_coef_grp(c.data(), (int)c.size(), 1, st));
        // chi_k /= |chi_k| + c_k = <chi_k, r>; r -= c_k chi_k (masked per rhs) + |r|^2
        auto u2 = upd([k](const Sys& y) {
          return UpdArgs{y.chi_k(k), y.n, nullptr, 0, 0, 1, nullptr, 1, nullptr, y.binv, y.r, y.n, y.n, y.nr, 0,
                         y.part, y.chist + (size_t)k * y.nr};
        });
        HCK(x0, launch_scale_dot_grp(u2.data(), (int)u2.size(), st));
        auto u3 = upd([k](const Sys& y) {
          return UpdArgs{y.r, y.n, y.chi_k(k), 0, y.n, 1, y.chist + (size_t)k * y.nr, 1, y.active, nullptr, nullptr,
                         0, y.n, y.nr, 0, y.part, y.rn2};
        });
        HCK(x0, launch_sub_dots_grp(u3.data(), (int)u3.size(), 1, st));
        HCK(x0, ev.mark(3, st));
        q = fetch_rn2(run);
        if (q != QDD_OK) return q;
        HCK(x0, ev.add(0, 3));
      }
      tstage[3] += since(ta);
      // per-rhs convergence of the recursive residual; systems leave the cycle
      std::vector<int> next;
      for (int s : run) {
        Sys& y = S[s];
        ++y.total_it;
        y.kk = k + 1;
        bool changed = false;
        for (int i = 0; i < y.nr; ++i) {
          if (!y.act[i]) continue;
          y.ks[i] = k + 1;
          y.iters[i]++;
          y.rn[i] = std::sqrt(std::fabs(y.h2[i].x));
          if (!std::isfinite(y.h2[i].x)) {
            y.nonfinite = true;
            y.act[i] = 0;
            changed = true;
          } else if (y.rn[i] <= y.x->cfg.tol * y.etan[i]) {
            y.act[i] = 0;
            changed = true;
          }
        }
        const bool more = any_of(y.act) && k + 1 < y.x->cfg.nkv && y.total_it < y.x->cfg.nmx;
        if (more) {
          next.push_back(s);
          if (changed) HCK(x0, hipMemcpyAsync(y.active, y.act.data(), y.nr * sizeof(int), hipMemcpyHostToDevice, st));
        }
      }
      run.swap(next);
    }
    // end of the cycle: back substitution per rhs, psi += sum alpha_j phi_j, and
    // the true residual r = eta - D psi
    auto ta = tic();
    for (int s : live) {
      Sys& y = S[s];
      const int kk = y.kk;
      ah.resize((size_t)kk * y.nr * kMaxKv);
      bh.resize((size_t)kk * y.nr);
      chh.resize((size_t)kk * y.nr);
      al.assign((size_t)y.nr * kMaxKv, double2{0.0, 0.0});
      HCK(x0, hipMemcpyAsync(ah.data(), y.ahist, ah.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
      HCK(x0, hipMemcpyAsync(bh.data(), y.bhist, bh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HCK(x0, hipMemcpyAsync(chh.data(), y.chist, chh.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
      HCK(x0, hipStreamSynchronize(st));
      for (int i = 0; i < y.nr; ++i)
        fgcr_backsub(ah.data(), bh.data(), chh.data(), y.nr, i, y.ks[i], al.data() + (size_t)i * kMaxKv);
      HCK(x0, hipMemcpyAsync(y.alpha, al.data(), al.size() * sizeof(double2), hipMemcpyHostToDevice, st));
      // the staged copy must not be overwritten before it has been taken
      HCK(x0, hipStreamSynchronize(st));
    }
    HCK(x0, ev.mark(3, st));
    if (S[live[0]].phi32) {
      std::vector<AxpyArgs<float2>> ax;
      for (int s : live) {
        const Sys& y = S[s];
        ax.push_back(AxpyArgs<float2>{y.psi, y.n, (const float2*)y.phi, y.lstride, y.n, y.kk, y.alpha, kMaxKv, 1.0,
                                      y.n, nullptr, y.nr});
      }
      HCK(x0, launch_axpy_multi_grp<float2>(ax.data(), (int)ax.size(), st));
    } else {
      std::vector<AxpyArgs<double2>> ax;
      for (int s : live) {
        const Sys& y = S[s];
        ax.push_back(AxpyArgs<double2>{y.psi, y.n, (const double2*)y.phi, y.lstride, y.n, y.kk, y.alpha, kMaxKv, 1.0,
                                       y.n, nullptr, y.nr});
      }
      HCK(x0, launch_axpy_multi_grp<double2>(ax.data(), (int)ax.size(), st));
    }
    qdd_status q = apply_d(live, &Sys::psi, &Sys::t);
    if (q != QDD_OK) return q;
    {
      std::vector<SubArgs> sb;
      for (int s : live) {
        const Sys& y = S[s];
        sb.push_back(SubArgs{y.r, y.eta, y.t, y.n, y.n, y.nr});
      }
      HCK(x0, launch_sub_grp(sb.data(), (int)sb.size(), st));
    }
    q = r_sqnorm(live);
    if (q != QDD_OK) return q;
    HCK(x0, ev.mark(4, st));
    q = fetch_rn2(live);
    if (q != QDD_OK) return q;
    HCK(x0, ev.add(3, 4));
    tstage[7] += since(ta);
    for (int s : live) {
      Sys& y = S[s];
      for (int i = 0; i < y.nr; ++i) {
        if (y.conv[i]) continue;
        y.rn[i] = std::sqrt(std::fabs(y.h2[i].x));
        if (!std::isfinite(y.h2[i].x)) {
          y.nonfinite = true;
          y.act[i] = 0;
        } else if (y.rn[i] <= y.x->cfg.tol * y.etan[i]) {
          y.conv[i] = 1;
          y.act[i] = 0;
        } else {
          y.act[i] = 1;
          y.restarts[i]++;
        }
      }
      if (y.nonfinite) y.done = true;
    }
  }
  // solutions out, per-rhs records
  const double tot = since(t0);
  qdd_status status = QDD_OK;
  for (int s = 0; s < nsys; ++s) {
    Sys& y = S[s];
    PackedView pp = y.x->packed(QDD_F64, y.nr, 0, y.psi);
    HCK(x0, launch_unpack_spinor<double>(y.x->G, pp.f64, psi_c[s], y.nr, 0, pp.poff, pp.spoff, st));
    bool ok = true;
    for (int i = 0; i < y.nr; ++i) {
      ok = ok && y.conv[i];
      if (info && info[s]) {
        qdd_solve_info& f = info[s][i];
        f = qdd_solve_info{};
        f.iters = y.iters[i];
        f.restarts = y.conv[i] ? y.restarts[i] : std::max(0, y.restarts[i] - 1);
        f.converged = y.conv[i];
        f.fallbacks = 0;
        f.true_res = y.etan[i] > 0 ? y.rn[i] / y.etan[i] : 0.0;
        for (int j = 1; j < 8; ++j) f.t_ms[j] = tstage[j];
        f.t_ms[0] = tot;
        for (int j = 0; j < 4; ++j) f.gpu_ms[j] = ev.gpu_ms[j];
      }
    }
    if (!ok) {
      y.x->fail(y.nonfinite ? "non-finite residual" : "no convergence within nmx iterations");
      if (status == QDD_OK) status = QDD_ENOCONV;
    }
  }
  HCK(x0, hipStreamSynchronize(st));
  return status;
}
