// Oracle: link derivatives of the two-flavour effective action of Eq. 4 (the
// forces of the molecular-dynamics evolution in Sect. 2).
// TEST INFRASTRUCTURE ONLY (see orc_core.h).
//
// A link is varied as U_mu(x) -> exp(eps w) U_mu(x) with w traceless
// anti-Hermitian.  Each routine here adds, for every link, a complex 3x3 matrix
// M to an accumulator such that the first-order change of its quantity is
// eps Re tr(w M).  The force component along the generator T^a = i lambda^a / 2
// (Gell-Mann lambda^a) is then f^a = Re tr(T^a M).
#include "orc_core.h"

namespace orc {

static const cplx I(0.0, 1.0);

static void mm(const cplx* a, const cplx* b, cplx* c) { mat_mul(a, b, c); }

// product of a list of 3x3 matrices (identity for an empty list)
static void prod(const cplx* const* f, int n, cplx* out) {
  cplx acc[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, t[9];
  for (int k = 0; k < n; ++k) {
    mm(acc, f[k], t);
    for (int i = 0; i < 9; ++i) acc[i] = t[i];
  }
  for (int i = 0; i < 9; ++i) out[i] = acc[i];
}

// Clover part.  Quantity: sum_x Re tr(K(x) A(x)), with K(x) a 12x12 weight per
// site (row-major, index s*3+c) and A the clover field of clover_build, which is
// linear in the field strengths F_{mu nu}(x) of all ordered pairs mu != nu:
//   A = (4+m0) + c_sw sum_{mu != nu} (i/4) sigma_{mu nu} (x) F_{mu nu}.
// So the quantity changes by sum Re tr_colour(Lambda_{mu nu}(x) dF_{mu nu}(x)) with
//   Lambda_ab = c_sw (i/4) sum_{s,s'} K_{(s a),(s' b)} sigma_{mu nu}[s'][s],
// and with dF = (dQ - dQ^dag)/8, Re tr(Lambda dF) = Re tr(Lt dQ), Lt = (Lambda - Lambda^dag)/8,
// where Q_{mu nu}(x) is the sum of the four leaves of field_strength().
void clover_force(const Geom& g, const cplx* U, double csw, const cplx* K, cplx* M) {
  const Gamma& G = gammas();
  for (int64_t x = 0; x < g.V; ++x) {
    const cplx* k = K + x * 144;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = 0; nu < 4; ++nu) {
        if (mu == nu) continue;
        cplx lam[9], lt[9];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            cplx acc = 0;
            for (int s = 0; s < 4; ++s)
              for (int sp = 0; sp < 4; ++sp) acc += k[(s * 3 + a) * 12 + sp * 3 + b] * G.sigma[mu][nu][sp][s];
            lam[a * 3 + b] = csw * 0.25 * I * acc;
          }
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) lt[a * 3 + b] = (lam[a * 3 + b] - std::conj(lam[b * 3 + a])) / 8.0;
        // the leaves of field_strength(x, mu, nu), each as four (site, direction, adjoint) factors
        const int64_t xpm = g.up(x, mu), xpn = g.up(x, nu), xmm = g.dn(x, mu), xmn = g.dn(x, nu);
        const int64_t xmm_pn = g.up(xmm, nu), xmm_mn = g.dn(xmm, nu), xmn_pm = g.up(xmn, mu);
        struct Fac { int64_t site; int dir; bool dag; };
        const Fac leaves[4][4] = {
            {{x, mu, false}, {xpm, nu, false}, {xpn, mu, true}, {x, nu, true}},
            {{x, nu, false}, {xmm_pn, mu, true}, {xmm, nu, true}, {xmm, mu, false}},
            {{xmm, mu, true}, {xmm_mn, nu, true}, {xmm_mn, mu, false}, {xmn, nu, false}},
            {{xmn, nu, true}, {xmn, mu, false}, {xmn_pm, nu, false}, {x, mu, true}}};
        for (const auto& leaf : leaves) {
          cplx m[4][9];
          const cplx* f[4];
          for (int q = 0; q < 4; ++q) {
            const cplx* u = link(U, leaf[q].site, leaf[q].dir);
            if (leaf[q].dag) mat_dag(u, m[q]);
            else for (int i = 0; i < 9; ++i) m[q][i] = u[i];
            f[q] = m[q];
          }
          for (int q = 0; q < 4; ++q) {
            // leaf = f0 f1 f2 f3, d(f_q) = w f_q (not adjoint) or -f_q w (adjoint):
            //   not adjoint: d Re tr(Lt leaf) = Re tr(w (f_q..f_3) Lt (f_0..f_{q-1}))
            //   adjoint:     d Re tr(Lt leaf) = -Re tr(w (f_{q+1}..f_3) Lt (f_0..f_q))
            cplx right[9], left[9], t[9], c[9];
            const bool dag = leaf[q].dag;
            prod(f + (dag ? q + 1 : q), dag ? 3 - q : 4 - q, right);
            prod(f, dag ? q + 1 : q, left);
            mm(right, lt, t);
            mm(t, left, c);
            cplx* out = M + (leaf[q].site * 4 + leaf[q].dir) * 9;
            for (int i = 0; i < 9; ++i) out[i] += dag ? -c[i] : c[i];
          }
        }
      }
  }
}

// Hopping part.  Quantity: coef Re sum_x X(x)^dag (H Y)(x), with
//   (H Y)(x) = sum_mu [ s (1-g_mu) U_mu(x) Y(x+mu) + s (1+g_mu) U_mu(x-mu)^dag Y(x-mu) ]
// (s the fermion boundary sign of the hop, as in hop_site).  X and Y are full
// fields; X is usually non-zero on one parity only.
void hop_force(const Geom& g, const cplx* U, const cplx* X, const cplx* Y, double coef, cplx* M) {
  const Gamma& G = gammas();
  for (int64_t x = 0; x < g.V; ++x) {
    const cplx* a = X + x * 12;
    bool zero = true;
    for (int i = 0; i < 12; ++i) zero = zero && a[i] == cplx(0);
    if (zero) continue;
    for (int mu = 0; mu < 4; ++mu)
      for (int dir = 0; dir < 2; ++dir) {
        // P = 1 - g_mu (forward) or 1 + g_mu (backward); Z = P^dag X(x) (g_mu Hermitian)
        const double pm = dir == 0 ? -1.0 : 1.0;
        cplx z[12];
        for (int sb = 0; sb < 4; ++sb)
          for (int i = 0; i < 3; ++i) {
            cplx acc = a[sb * 3 + i];
            for (int sa = 0; sa < 4; ++sa) acc += pm * std::conj(G.g[mu][sa][sb]) * a[sa * 3 + i];
            z[sb * 3 + i] = acc;
          }
        if (dir == 0) {
          // link (x, mu): d[X^dag P U Y(x+mu)] = tr(w N), N_ji = sum_s (U y_s)_j conj(z_{s i})
          const int64_t y = g.up(x, mu);
          const cplx* u = link(U, x, mu);
          const double s = g.sign_up(x, mu);
          cplx* out = M + (x * 4 + mu) * 9;
          for (int sb = 0; sb < 4; ++sb) {
            cplx uy[3];
            for (int j = 0; j < 3; ++j) {
              uy[j] = 0;
              for (int k = 0; k < 3; ++k) uy[j] += u[j * 3 + k] * Y[y * 12 + sb * 3 + k];
            }
            for (int j = 0; j < 3; ++j)
              for (int i = 0; i < 3; ++i) out[j * 3 + i] += coef * s * uy[j] * std::conj(z[sb * 3 + i]);
          }
        } else {
          // link (x-mu, mu): d[X^dag P U^dag Y(x-mu)] = -tr(w N'), N'_kj = sum_s y_{s k} conj(c_{s j}), c_s = U z_s
          const int64_t y = g.dn(x, mu);
          const cplx* u = link(U, y, mu);
          const double s = g.sign_up(y, mu);
          cplx* out = M + (y * 4 + mu) * 9;
          for (int sb = 0; sb < 4; ++sb) {
            cplx c[3];
            for (int j = 0; j < 3; ++j) {
              c[j] = 0;
              for (int i = 0; i < 3; ++i) c[j] += u[j * 3 + i] * z[sb * 3 + i];
            }
            for (int k = 0; k < 3; ++k)
              for (int j = 0; j < 3; ++j) out[k * 3 + j] -= coef * s * Y[y * 12 + sb * 3 + k] * std::conj(c[j]);
          }
        }
      }
  }
}

// (H^dag X)(y) = sum_x H(x,y)^dag X(x): the hop x -> x+mu = y contributes
// s (1-g_mu) U_mu(y-mu)^dag X(y-mu), the hop x -> x-mu = y contributes
// s (1+g_mu) U_mu(y) X(y+mu) (g_mu Hermitian, so (1 -/+ g_mu)^dag = 1 -/+ g_mu)
void hop_adj(const Geom& g, const cplx* U, const cplx* X, cplx* out) {
  const Gamma& G = gammas();
  for (int64_t y = 0; y < g.V; ++y) {
    cplx o[12] = {};
    for (int mu = 0; mu < 4; ++mu)
      for (int dir = 0; dir < 2; ++dir) {
        const int64_t x = dir == 0 ? g.dn(y, mu) : g.up(y, mu);
        const cplx* u = dir == 0 ? link(U, x, mu) : link(U, y, mu);
        const double s = dir == 0 ? g.sign_up(x, mu) : g.sign_up(y, mu);
        cplx t[12];
        for (int sp = 0; sp < 4; ++sp)
          for (int a = 0; a < 3; ++a) {
            cplx acc = 0;
            for (int b = 0; b < 3; ++b)
              acc += (dir == 0 ? std::conj(u[b * 3 + a]) : u[a * 3 + b]) * X[x * 12 + sp * 3 + b];
            t[sp * 3 + a] = acc;
          }
        const double pm = dir == 0 ? -1.0 : 1.0;
        for (int sa = 0; sa < 4; ++sa)
          for (int a = 0; a < 3; ++a) {
            cplx acc = t[sa * 3 + a];
            for (int sb = 0; sb < 4; ++sb) acc += pm * G.g[mu][sa][sb] * t[sb * 3 + a];
            o[sa * 3 + a] += s * acc;
          }
      }
    for (int i = 0; i < 12; ++i) out[y * 12 + i] = o[i];
  }
}

// f^a = Re tr(T^a M) for the eight generators T^a = i lambda^a / 2
void force_components(int64_t nlinks, const cplx* M, double* f) {
  for (int64_t l = 0; l < nlinks; ++l) {
    const cplx* m = M + l * 9;
    auto e = [&](int i, int j) { return m[i * 3 + j]; };
    // tr(lambda^a M) = sum_ij lambda^a_ij M_ji for the Gell-Mann matrices
    const cplx t[8] = {e(1, 0) + e(0, 1),
                       I * e(0, 1) - I * e(1, 0),
                       e(0, 0) - e(1, 1),
                       e(2, 0) + e(0, 2),
                       I * e(0, 2) - I * e(2, 0),
                       e(2, 1) + e(1, 2),
                       I * e(1, 2) - I * e(2, 1),
                       (e(0, 0) + e(1, 1) - 2.0 * e(2, 2)) / std::sqrt(3.0)};
    for (int a = 0; a < 8; ++a) f[l * 8 + a] = (0.5 * I * t[a]).real();
  }
}

}  // namespace orc
