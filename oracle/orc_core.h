// Oracle core: plain FP64 CPU reference of the clover-Wilson operator and the
// deflated Schwarz-preconditioned GCR solver.
//
// TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously-correct checker
// for the HIP library; it shares no source with it and must never be linked
// into, or called from, the product path.
//
// Conventions (the paper fixes only Eq. 1-5; the rest is this oracle's stated
// reading):
//   * lattice L0 x L1 x L2 x L3, direction 0 = time; lex = ((x0*L1+x1)*L2+x2)*L3+x3
//   * parity p(x) = (x0+x1+x2+x3) mod 2; even-site fields are indexed by lex >> 1
//   * spinor psi(x) has 12 complex entries, index s*3 + c (spin s, colour c)
//   * gamma matrices: chiral Euclidean basis
//       g0 = [[0,-1],[-1,0]],  gk = [[0,-i sk],[i sk,0]],  g5 = diag(1,1,-1,-1)
//   * fermion boundary sign: bc (= -1 antiperiodic, +1 periodic) on hops that
//     cross the time boundary x0 = L0-1 <-> 0; the clover term uses bare links
#pragma once
#include <complex>
#include <vector>
#include <cstdint>
#include <cmath>

namespace orc {

typedef std::complex<double> cplx;

struct Geom {
  int L[4];
  int64_t V;
  int bc;  // time boundary sign
  Geom(const int* l, int bc_) : bc(bc_) {
    for (int i = 0; i < 4; ++i) L[i] = l[i];
    V = (int64_t)L[0] * L[1] * L[2] * L[3];
  }
  void coords(int64_t lex, int x[4]) const {
    x[3] = (int)(lex % L[3]); lex /= L[3];
    x[2] = (int)(lex % L[2]); lex /= L[2];
    x[1] = (int)(lex % L[1]); lex /= L[1];
    x[0] = (int)lex;
  }
  int64_t lex(const int x[4]) const {
    return ((((int64_t)x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3]) + x[3];
  }
  int parity(int64_t lex_) const {
    int x[4]; coords(lex_, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
  }
  int64_t up(int64_t lex_, int mu) const {
    int x[4]; coords(lex_, x);
    x[mu] = (x[mu] + 1) % L[mu];
    return lex(x);
  }
  int64_t dn(int64_t lex_, int mu) const {
    int x[4]; coords(lex_, x);
    x[mu] = (x[mu] + L[mu] - 1) % L[mu];
    return lex(x);
  }
  // sign of the hop x -> x+mu (and of its adjoint x+mu -> x)
  double sign_up(int64_t lex_, int mu) const {
    if (mu != 0) return 1.0;
    int x[4]; coords(lex_, x);
    return (x[0] == L[0] - 1) ? (double)bc : 1.0;
  }
};

// gamma_mu as 4x4 complex matrices, and sigma_{mu nu} = (i/2)[g_mu, g_nu]
struct Gamma {
  cplx g[5][4][4];
  cplx sigma[4][4][4][4];
  Gamma();
};
const Gamma& gammas();

// 3x3 helpers (row-major complex)
void mat_mul(const cplx* a, const cplx* b, cplx* c);           // c = a b
void mat_mul_dag_right(const cplx* a, const cplx* b, cplx* c); // c = a b^dag
void mat_dag(const cplx* a, cplx* c);

// fields are flat arrays of cplx: links U[(lex*4+mu)*9 + a*3+b],
// spinors psi[lex*12 + s*3+c], clover A[lex*144 + i*12+j]
inline const cplx* link(const cplx* U, int64_t lex, int mu) { return U + (lex * 4 + mu) * 9; }

// ---- operators (orc_dirac.cpp) ----
// Clover field A(x) = (4+m0) + c_sw sum_{mu,nu} (i/4) sigma_{mu nu} F_{mu nu}(x), and its inverse.
// Returns the number of sites whose 12x12 inverse failed (singular pivot).
int64_t clover_build(const Geom& g, const cplx* U, double kappa, double csw, cplx* A, cplx* Ainv,
                     double* min_abs_eig_bound);
// F_{mu nu}(x) (3x3, anti-Hermitian) from the four clover leaves
void field_strength(const Geom& g, const cplx* U, int64_t x, int mu, int nu, cplx* F);
// hopping sum H psi (x) = sum_mu [ s (1-g_mu) U_mu(x) psi(x+mu) + s (1+g_mu) U_mu(x-mu)^dag psi(x-mu) ]
// evaluated at one site, accumulating `scale * H psi(x)` into out12.
void hop_site(const Geom& g, const cplx* U, const cplx* psi, int64_t x, double scale, cplx* out12,
              const uint8_t* mask /* optional: only neighbours with mask[y]!=0 contribute */);
void apply_D(const Geom& g, const cplx* U, const cplx* A, const cplx* psi, cplx* out);
void apply_clover_site(const cplx* A12x12, const cplx* in12, cplx* out12);
// even-odd pieces on even/odd-indexed fields (index lex >> 1)
void apply_Dhat(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const cplx* pe, cplx* oe);
void lex_of_parity(const Geom& g, int p, std::vector<int64_t>& out);

// ---- link derivatives (orc_force.cpp) ----
// Each adds to M (per link, [(lex*4+mu)*9]) the 3x3 matrix whose Re tr(w M) is
// the first-order change of its quantity under U_mu(x) -> exp(eps w) U_mu(x).
// clover_force: quantity sum_x Re tr(K(x) A(x)), K a 12x12 weight per site.
void clover_force(const Geom& g, const cplx* U, double csw, const cplx* K, cplx* M);
// hop_force: quantity coef Re sum_x X(x)^dag (H Y)(x) (H the hopping sum of hop_site).
void hop_force(const Geom& g, const cplx* U, const cplx* X, const cplx* Y, double coef, cplx* M);
// out = H^dag X (full fields)
void hop_adj(const Geom& g, const cplx* U, const cplx* X, cplx* out);
// f[l*8+a] = Re tr(T^a M_l), T^a = i lambda^a / 2
void force_components(int64_t nlinks, const cplx* M, double* f);

// ---- vector helpers ----
cplx dot(const cplx* a, const cplx* b, int64_t n);  // sum conj(a) b
double norm2(const cplx* a, int64_t n);

}  // namespace orc
