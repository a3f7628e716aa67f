// Oracle C entry points (host pointers; complex128 arrays passed as double*).
// TEST INFRASTRUCTURE ONLY: called from the test-suite, the smoke check and the
// CPU-baseline timing, never from the HIP library.
#include <functional>
#include <cstring>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "orc_dfl.h"

using namespace orc;
#define C(p) reinterpret_cast<cplx*>(p)
#define CC(p) reinterpret_cast<const cplx*>(p)

extern "C" {

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int64_t orc_clover(const int* L, int bc, const double* U, double kappa, double csw, double* A, double* Ainv) {
  Geom g(L, bc);
  return clover_build(g, CC(U), kappa, csw, C(A), Ainv ? C(Ainv) : nullptr, nullptr);
}

void orc_field_strength(const int* L, int bc, const double* U, int64_t x, int mu, int nu, double* F) {
  Geom g(L, bc);
  field_strength(g, CC(U), x, mu, nu, C(F));
}

void orc_block_bicgstab(const int* L, int bc, const double* U, const double* A, const double* Ainv, const int* bs,
                        const int64_t* blks, int64_t nlist, const double* eta, double* psi, double tol, int maxit,
                        int* iters, double* res) {
  Geom g(L, bc);
  block_bicgstab(g, CC(U), CC(A), CC(Ainv), bs, blks, nlist, CC(eta), C(psi), tol, maxit, iters, res);
}

void orc_clover_force(const int* L, int bc, const double* U, double csw, const double* K, double* M) {
  Geom g(L, bc);
  clover_force(g, CC(U), csw, CC(K), C(M));
}

void orc_hop_force(const int* L, int bc, const double* U, const double* X, const double* Y, double coef, double* M) {
  Geom g(L, bc);
  hop_force(g, CC(U), CC(X), CC(Y), coef, C(M));
}

void orc_hop_adj(const int* L, int bc, const double* U, const double* X, double* out) {
  Geom g(L, bc);
  hop_adj(g, CC(U), CC(X), C(out));
}

void orc_force_components(int64_t nlinks, const double* M, double* f) { force_components(nlinks, CC(M), f); }

void orc_gamma(double* out /* 5 x 4 x 4 complex */) {
  const Gamma& G = gammas();
  std::memcpy(out, G.g, sizeof(G.g));
}

void orc_apply_D(const int* L, int bc, const double* U, const double* A, const double* psi, double* out) {
  Geom g(L, bc);
  apply_D(g, CC(U), CC(A), CC(psi), C(out));
}

void orc_apply_Dhat(const int* L, int bc, const double* U, const double* A, const double* Ainv, const double* pe,
                    double* oe) {
  Geom g(L, bc);
  apply_Dhat(g, CC(U), CC(A), CC(Ainv), CC(pe), C(oe));
}

void orc_sap(const int* L, int bc, const double* U, const double* A, const double* Ainv, const int* bs, int ncy,
             int nmr, const double* eta, double* psi) {
  Geom g(L, bc);
  sap(g, CC(U), CC(A), CC(Ainv), bs, ncy, nmr, CC(eta), C(psi));
}

void orc_sap_half_sweep(const int* L, int bc, const double* U, const double* A, const double* Ainv, const int* bs,
                        int nmr, int col, const double* eta, double* psi, double* rho) {
  Geom g(L, bc);
  sap_half_sweep(g, CC(U), CC(A), CC(Ainv), bs, nmr, col, CC(eta), C(psi), C(rho));
}

// psi = the first Schwarz cycle (ncy = 1) on the listed colour-1 blocks and their
// face neighbours (see sap_one_cycle_on_blocks); returns -1 on a bad block list
int orc_sap_one_cycle_on_blocks(const int* L, int bc, const double* U, const double* A, const double* Ainv,
                                const int* bs, int nmr, const double* eta, const int64_t* blocks, int nblocks,
                                double* psi) {
  Geom g(L, bc);
  return sap_one_cycle_on_blocks(g, CC(U), CC(A), CC(Ainv), bs, nmr, CC(eta), blocks, nblocks, C(psi));
}

// ---- deflation handle ----
void* orc_dfl_new(const int* L, int bc, const int* bs, int Ns) {
  Geom* g = new Geom(L, bc);
  return new DflHandle(g, bs, Ns);
}
void orc_dfl_free(void* h) {
  DflHandle* d = (DflHandle*)h;
  delete d;
}
int64_t orc_dfl_nblocks(void* h) { return ((DflHandle*)h)->d->B.nblk; }
void orc_dfl_build(void* h, const double* U, const double* A, const double* Ainv, const int* sap_bs, int ncy,
                   int nmr, int nit, const double* init) {
  DflHandle* d = (DflHandle*)h;
  dfl_build(*d->d, CC(U), CC(A), CC(Ainv), sap_bs, ncy, nmr, nit, CC(init));
}
// install a given basis (Ns full fields) without SAP iterations, then orthonormalise + little op
void orc_dfl_set_fields(void* h, const double* U, const double* A, const double* fields) {
  DflHandle* d = (DflHandle*)h;
  dfl_set_fields(*d->d, CC(U), CC(A), CC(fields));
}
void orc_dfl_set_fields_on_blocks(void* h, const double* U, const double* A, const double* fields,
                                  const int64_t* blocks, int nblocks) {
  DflHandle* d = (DflHandle*)h;
  dfl_set_fields_on_blocks(*d->d, CC(U), CC(A), CC(fields), blocks, nblocks);
}
void orc_dfl_get_basis(void* h, double* out) {
  DflHandle* d = (DflHandle*)h;
  std::memcpy(out, d->d->W.data(), sizeof(cplx) * d->d->W.size());
}
void orc_dfl_get_little(void* h, double* out) {
  DflHandle* d = (DflHandle*)h;
  std::memcpy(out, d->d->little.data(), sizeof(cplx) * d->d->little.size());
}
void orc_dfl_restrict(void* h, const double* r, double* c) { dfl_restrict(*((DflHandle*)h)->d, CC(r), C(c)); }
void orc_dfl_prolong(void* h, const double* c, double* out) { dfl_prolong(*((DflHandle*)h)->d, CC(c), C(out)); }
void orc_dfl_coarse_apply(void* h, const double* c, double* out) {
  coarse_apply(*((DflHandle*)h)->d, CC(c), C(out));
}
int orc_dfl_coarse_solve(void* h, const double* f, double* c, double tol) {
  FgcrResult r = coarse_solve(*((DflHandle*)h)->d, CC(f), C(c), tol, 32, 100000);
  return r.converged ? r.iters : -1;
}
void orc_dfl_precond(void* h, const double* U, const double* A, const double* Ainv, const int* sap_bs, int ncy,
                     int nmr, double coarse_tol, const double* r, double* out) {
  dfl_precond(*((DflHandle*)h)->d, CC(U), CC(A), CC(Ainv), sap_bs, ncy, nmr, coarse_tol, CC(r), C(out));
}

// Two-level preconditioner with the network stage: out = C r + N(r1) + M_sap(r2),
// r1 = r - D C r, r2 = r1 - D N(r1); N dropped (fallback) if |r2| > |r1|.
// Returns 1 on fallback, else 0.
int orc_dfl_net_precond(void* h, const double* U, const double* A, const double* Ainv, const int* sap_bs, int ncy,
                        int nmr, double coarse_tol, int nl, const int* ch, const double* W, const double* r,
                        double* out) {
  return dfl_net_precond(*((DflHandle*)h)->d, CC(U), CC(A), CC(Ainv), sap_bs, ncy, nmr, coarse_tol, nl, ch, CC(W),
                         CC(r), C(out));
}

// ---- solver ----
// op: 0 = full D, 1 = Dhat (even sites).  prec: 0 none, 1 SAP, 2 deflated SAP,
// 3 deflated SAP with the network stage (weights `net_w`, channels `ch`, nl layers).
// info[0] = iterations, info[1] = restarts, info[2] = converged; *relres = true
// relative residual at exit.  Returns 0 on convergence, -4 otherwise.
int orc_fgcr(const int* L, int bc, const double* U, const double* A, const double* Ainv, int op, int prec,
             const int* sap_bs, int ncy, int nmr, void* dfl, double coarse_tol, int nl, const int* ch,
             const double* net_w, const double* eta, double* psi, int nkv, int nmx, double tol, int* info,
             double* relres, double* history, int nhist, int* fallbacks) {
  Geom g(L, bc);
  const cplx *u = CC(U), *a = CC(A), *ai = CC(Ainv);
  int64_t n = (op == 1 ? g.V / 2 : g.V) * 12;
  LinOp lop;
  if (op == 1) lop = [&](const cplx* in, cplx* out) { apply_Dhat(g, u, a, ai, in, out); };
  else lop = [&](const cplx* in, cplx* out) { apply_D(g, u, a, in, out); };
  int nfb = 0;
  LinOp pre;
  const LinOp* pp = nullptr;
  if (prec == 1) {
    pre = [&](const cplx* in, cplx* out) { sap(g, u, a, ai, sap_bs, ncy, nmr, in, out); };
    pp = &pre;
  } else if (prec == 2) {
    Deflation* d = ((DflHandle*)dfl)->d;
    pre = [&, d](const cplx* in, cplx* out) { dfl_precond(*d, u, a, ai, sap_bs, ncy, nmr, coarse_tol, in, out); };
    pp = &pre;
  } else if (prec == 3) {
    Deflation* d = ((DflHandle*)dfl)->d;
    pre = [&, d](const cplx* in, cplx* out) {
      nfb += dfl_net_precond(*d, u, a, ai, sap_bs, ncy, nmr, coarse_tol, nl, ch, CC(net_w), in, out);
    };
    pp = &pre;
  }
  FgcrResult r = fgcr(n, lop, pp, CC(eta), C(psi), nkv, nmx, tol, history, nhist);
  if (info) { info[0] = r.iters; info[1] = r.restarts; info[2] = r.converged; }
  if (relres) *relres = r.relres;
  if (fallbacks) *fallbacks = nfb;
  return r.converged ? 0 : -4;
}

// ---- network ----
void orc_net_layer_forward(const int* L, int bc, const double* U, int cin, int cout, const double* W,
                           const double* in, double* out) {
  Geom g(L, bc);
  net_layer_forward(g, CC(U), cin, cout, CC(W), CC(in), C(out));
}
void orc_net_layer_backward(const int* L, int bc, const double* U, int cin, int cout, const double* W,
                            const double* in, const double* gy, double* gx, double* gW) {
  Geom g(L, bc);
  net_layer_backward(g, CC(U), cin, cout, CC(W), CC(in), CC(gy), C(gx), C(gW));
}
void orc_net_forward(const int* L, int bc, const double* U, int nl, const int* ch, const double* W,
                     const double* in, double* out) {
  Geom g(L, bc);
  net_forward(g, CC(U), nl, ch, CC(W), CC(in), C(out));
}
void orc_net_forward_on_sites(const int* L, int bc, const double* U, int nl, const int* ch, const double* W,
                              const double* in, const int64_t* sites, int nsites, double* out) {
  Geom g(L, bc);
  net_forward_on_sites(g, CC(U), nl, ch, CC(W), CC(in), sites, nsites, C(out));
}
double orc_net_loss_grad(const int* L, int bc, const double* U, int nl, const int* ch, const double* W, int nb,
                         const double* r, const double* e, double* grad) {
  Geom g(L, bc);
  return net_loss_grad(g, CC(U), nl, ch, CC(W), nb, CC(r), CC(e), grad ? C(grad) : nullptr);
}

}  // extern "C"
