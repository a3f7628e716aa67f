// Oracle: the O(a)-improved Wilson-Dirac operator of Eq. (1) and its even-odd
// Schur complement of Eq. (2).  TEST INFRASTRUCTURE ONLY (see orc_core.h).
#include "orc_core.h"
#include <cstring>
#include <algorithm>

namespace orc {

static const cplx I(0.0, 1.0);

Gamma::Gamma() {
  std::memset((void*)g, 0, sizeof(g));
  // Pauli matrices
  cplx s[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  // g0 = [[0,-1],[-1,0]] in 2x2 spin blocks
  for (int a = 0; a < 2; ++a) {
    g[0][a][2 + a] = -1.0;
    g[0][2 + a][a] = -1.0;
  }
  // gk = [[0, -i sk], [i sk, 0]]
  for (int k = 1; k <= 3; ++k)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        g[k][a][2 + b] = -I * s[k - 1][a][b];
        g[k][2 + a][b] = I * s[k - 1][a][b];
      }
  // g5 = g0 g1 g2 g3
  cplx t1[4][4], t2[4][4];
  auto mm = [](cplx a[4][4], cplx b[4][4], cplx c[4][4]) {
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        cplx acc = 0;
        for (int k = 0; k < 4; ++k) acc += a[i][k] * b[k][j];
        c[i][j] = acc;
      }
  };
  mm(g[0], g[1], t1);
  mm(t1, g[2], t2);
  mm(t2, g[3], g[4]);
  // sigma_{mu nu} = (i/2) [g_mu, g_nu]
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu) {
      cplx a[4][4], b[4][4];
      mm(g[mu], g[nu], a);
      mm(g[nu], g[mu], b);
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) sigma[mu][nu][i][j] = 0.5 * I * (a[i][j] - b[i][j]);
    }
}

const Gamma& gammas() {
  static Gamma G;
  return G;
}

void mat_mul(const cplx* a, const cplx* b, cplx* c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx acc = 0;
      for (int k = 0; k < 3; ++k) acc += a[i * 3 + k] * b[k * 3 + j];
      c[i * 3 + j] = acc;
    }
}

void mat_dag(const cplx* a, cplx* c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c[i * 3 + j] = std::conj(a[j * 3 + i]);
}

void mat_mul_dag_right(const cplx* a, const cplx* b, cplx* c) {
  cplx bd[9];
  mat_dag(b, bd);
  mat_mul(a, bd, c);
}

// Clover leaves: the four plaquettes of the (mu,nu) plane that start and end at
// x, all traversed in the same (mu then nu) orientation.  Their sum is Q_{mu nu};
// F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag) / 8.  (Eq. 1, the field strength of the
// clover term; reading: no traceless projection.)
void field_strength(const Geom& g, const cplx* U, int64_t x, int mu, int nu, cplx* F) {
  cplx Q[9] = {}, t1[9], t2[9], t3[9], d[9];
  auto add = [&](const cplx* m) { for (int i = 0; i < 9; ++i) Q[i] += m[i]; };
  int64_t xpm = g.up(x, mu), xpn = g.up(x, nu), xmm = g.dn(x, mu), xmn = g.dn(x, nu);
  int64_t xmm_pn = g.up(xmm, nu), xmm_mn = g.dn(xmm, nu), xmn_pm = g.up(xmn, mu);
  // leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
  mat_mul(link(U, x, mu), link(U, xpm, nu), t1);
  mat_mul_dag_right(t1, link(U, xpn, mu), t2);
  mat_mul_dag_right(t2, link(U, x, nu), t3);
  add(t3);
  // leaf 2: x -> x+nu -> x+nu-mu -> x-mu -> x
  mat_mul_dag_right(link(U, x, nu), link(U, xmm_pn, mu), t1);
  mat_mul_dag_right(t1, link(U, xmm, nu), t2);
  mat_mul(t2, link(U, xmm, mu), t3);
  add(t3);
  // leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
  mat_dag(link(U, xmm, mu), d);
  mat_mul_dag_right(d, link(U, xmm_mn, nu), t1);
  mat_mul(t1, link(U, xmm_mn, mu), t2);
  mat_mul(t2, link(U, xmn, nu), t3);
  add(t3);
  // leaf 4: x -> x-nu -> x-nu+mu -> x+mu -> x
  mat_dag(link(U, xmn, nu), d);
  mat_mul(d, link(U, xmn, mu), t1);
  mat_mul(t1, link(U, xmn_pm, nu), t2);
  mat_mul_dag_right(t2, link(U, x, mu), t3);
  add(t3);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F[i * 3 + j] = (Q[i * 3 + j] - std::conj(Q[j * 3 + i])) / 8.0;
}

// Gauss-Jordan inverse with partial pivoting of an n x n complex matrix.
static bool invert(const cplx* a, cplx* inv, int n) {
  std::vector<cplx> m(a, a + n * n);
  for (int i = 0; i < n * n; ++i) inv[i] = 0;
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    double best = std::abs(m[col * n + col]);
    for (int r = col + 1; r < n; ++r)
      if (std::abs(m[r * n + col]) > best) { best = std::abs(m[r * n + col]); piv = r; }
    if (!(best > 1e-300)) return false;
    if (piv != col)
      for (int k = 0; k < n; ++k) {
        std::swap(m[piv * n + k], m[col * n + k]);
        std::swap(inv[piv * n + k], inv[col * n + k]);
      }
    cplx p = 1.0 / m[col * n + col];
    for (int k = 0; k < n; ++k) { m[col * n + k] *= p; inv[col * n + k] *= p; }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      cplx f = m[r * n + col];
      if (f == cplx(0)) continue;
      for (int k = 0; k < n; ++k) {
        m[r * n + k] -= f * m[col * n + k];
        inv[r * n + k] -= f * inv[col * n + k];
      }
    }
  }
  return true;
}

// A(x) = (4 + m0) 1 + c_sw sum_{mu,nu} (i/4) sigma_{mu nu} (x) F_{mu nu}(x)   [Eq. 1]
// with m0 = 1/(2 kappa) - 4 (reading of the kappa <-> m relation); the sum runs
// over all ordered pairs.  A is stored as a dense 12x12 per site.
int64_t clover_build(const Geom& g, const cplx* U, double kappa, double csw, cplx* A, cplx* Ainv,
                     double*) {
  const Gamma& G = gammas();
  const double diag = 1.0 / (2.0 * kappa);
  int64_t nbad = 0;
#pragma omp parallel for reduction(+ : nbad) schedule(static)
  for (int64_t x = 0; x < g.V; ++x) {
    cplx* a = A + x * 144;
    for (int i = 0; i < 144; ++i) a[i] = 0;
    for (int i = 0; i < 12; ++i) a[i * 12 + i] = diag;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = 0; nu < 4; ++nu) {
        if (mu == nu) continue;
        cplx F[9];
        field_strength(g, U, x, mu, nu, F);
        for (int s = 0; s < 4; ++s)
          for (int sp = 0; sp < 4; ++sp) {
            cplx f = csw * 0.25 * I * G.sigma[mu][nu][s][sp];
            if (f == cplx(0)) continue;
            for (int c = 0; c < 3; ++c)
              for (int cp = 0; cp < 3; ++cp) a[(s * 3 + c) * 12 + sp * 3 + cp] += f * F[c * 3 + cp];
          }
      }
    if (Ainv && !invert(a, Ainv + x * 144, 12)) ++nbad;
  }
  return nbad;
}

void apply_clover_site(const cplx* A, const cplx* in, cplx* out) {
  for (int i = 0; i < 12; ++i) {
    cplx acc = 0;
    for (int j = 0; j < 12; ++j) acc += A[i * 12 + j] * in[j];
    out[i] = acc;
  }
}

// scale * sum_mu [ s (1 - g_mu) U_mu(x) psi(x+mu) + s (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
void hop_site(const Geom& g, const cplx* U, const cplx* psi, int64_t x, double scale, cplx* out,
              const uint8_t* mask) {
  const Gamma& G = gammas();
  for (int mu = 0; mu < 4; ++mu) {
    for (int dir = 0; dir < 2; ++dir) {
      int64_t y = dir == 0 ? g.up(x, mu) : g.dn(x, mu);
      if (mask && !mask[y]) continue;
      double s = dir == 0 ? g.sign_up(x, mu) : g.sign_up(y, mu);
      const cplx* u = dir == 0 ? link(U, x, mu) : link(U, y, mu);
      // colour transport of every spin component
      cplx t[12];
      for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) {
          cplx acc = 0;
          for (int b = 0; b < 3; ++b)
            acc += (dir == 0 ? u[a * 3 + b] : std::conj(u[b * 3 + a])) * psi[y * 12 + sp * 3 + b];
          t[sp * 3 + a] = acc;
        }
      // spin projector (1 -/+ g_mu)
      double pm = dir == 0 ? -1.0 : 1.0;
      for (int sa = 0; sa < 4; ++sa)
        for (int a = 0; a < 3; ++a) {
          cplx acc = t[sa * 3 + a];
          for (int sb = 0; sb < 4; ++sb) acc += pm * G.g[mu][sa][sb] * t[sb * 3 + a];
          out[sa * 3 + a] += scale * s * acc;
        }
    }
  }
}

// (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [...]   [Eq. 1; D_W in the standard
// nearest-neighbour form, mass term folded into A]
void apply_D(const Geom& g, const cplx* U, const cplx* A, const cplx* psi, cplx* out) {
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < g.V; ++x) {
    cplx o[12];
    apply_clover_site(A + x * 144, psi + x * 12, o);
    hop_site(g, U, psi, x, -0.5, o, nullptr);
    for (int i = 0; i < 12; ++i) out[x * 12 + i] = o[i];
  }
}

void lex_of_parity(const Geom& g, int p, std::vector<int64_t>& out) {
  out.clear();
  for (int64_t x = 0; x < g.V; ++x)
    if (g.parity(x) == p) out.push_back(x);
}

// Dhat = D_ee - D_eo D_oo^{-1} D_oe on even fields   [Eq. 2, Schur complement]
void apply_Dhat(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const cplx* pe, cplx* oe) {
  std::vector<int64_t> ev, od;
  lex_of_parity(g, 0, ev);
  lex_of_parity(g, 1, od);
  std::vector<cplx> f(g.V * 12, 0.0), t(g.V * 12, 0.0);
  for (size_t i = 0; i < ev.size(); ++i)
    for (int k = 0; k < 12; ++k) f[ev[i] * 12 + k] = pe[i * 12 + k];
  // t_o = D_oo^{-1} D_oe pe
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)od.size(); ++i) {
    int64_t x = od[i];
    cplx h[12] = {};
    hop_site(g, U, f.data(), x, -0.5, h, nullptr);
    apply_clover_site(Ainv + x * 144, h, &t[x * 12]);
  }
  // oe = D_ee pe - D_eo t_o
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)ev.size(); ++i) {
    int64_t x = ev[i];
    cplx o[12], h[12] = {};
    apply_clover_site(A + x * 144, f.data() + x * 12, o);
    hop_site(g, U, t.data(), x, -0.5, h, nullptr);
    for (int k = 0; k < 12; ++k) oe[i * 12 + k] = o[k] - h[k];
  }
}

// sum_i conj(a_i) b_i over 64 fixed index ranges, each summed in index order,
// then the range sums in range order: the rounding does not depend on the
// thread count or schedule, so equal inputs give equal results
cplx dot(const cplx* a, const cplx* b, int64_t n) {
  constexpr int64_t kParts = 64;
  double re[kParts], im[kParts];
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < kParts; ++c) {
    double sr = 0, si = 0;
    for (int64_t i = n * c / kParts; i < n * (c + 1) / kParts; ++i) {
      cplx p = std::conj(a[i]) * b[i];
      sr += p.real();
      si += p.imag();
    }
    re[c] = sr;
    im[c] = si;
  }
  double sr = 0, si = 0;
  for (int64_t c = 0; c < kParts; ++c) {
    sr += re[c];
    si += im[c];
  }
  return cplx(sr, si);
}

double norm2(const cplx* a, int64_t n) { return dot(a, a, n).real(); }

}  // namespace orc
