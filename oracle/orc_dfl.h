// Oracle: block decomposition, solver and deflation declarations.
// TEST INFRASTRUCTURE ONLY (see orc_core.h).
#pragma once
#include "orc_core.h"
#include <functional>

namespace orc {

// Block decomposition of the lattice into bs[0] x .. x bs[3] blocks.
struct Blocks {
  const Geom& g;
  int bs[4], nb[4];
  int64_t nblk;
  std::vector<std::vector<int64_t>> sites;  // lex sites of every block (lex order)
  std::vector<int> colour;                  // (sum of block coordinates) mod 2
  Blocks(const Geom& g_, const int* b) : g(g_) {
    nblk = 1;
    for (int i = 0; i < 4; ++i) { bs[i] = b[i]; nb[i] = g.L[i] / b[i]; nblk *= nb[i]; }
    sites.assign(nblk, {});
    colour.assign(nblk, 0);
    for (int64_t x = 0; x < g.V; ++x) sites[block_of(x)].push_back(x);
    for (int64_t b2 = 0; b2 < nblk; ++b2) {
      int c[4]; bcoords(b2, c);
      colour[b2] = (c[0] + c[1] + c[2] + c[3]) & 1;
    }
  }
  void bcoords(int64_t b, int c[4]) const {
    c[3] = (int)(b % nb[3]); b /= nb[3];
    c[2] = (int)(b % nb[2]); b /= nb[2];
    c[1] = (int)(b % nb[1]); b /= nb[1];
    c[0] = (int)b;
  }
  int64_t block_of(int64_t x) const {
    int c[4]; g.coords(x, c);
    return (((int64_t)(c[0] / bs[0]) * nb[1] + c[1] / bs[1]) * nb[2] + c[2] / bs[2]) * nb[3] + c[3] / bs[3];
  }
  // neighbouring block across face d: d = 1+2mu (up), 2+2mu (down)
  int64_t nbr(int64_t b, int d) const {
    int c[4]; bcoords(b, c);
    int mu = (d - 1) / 2;
    c[mu] = (d & 1) ? (c[mu] + 1) % nb[mu] : (c[mu] + nb[mu] - 1) % nb[mu];
    return (((int64_t)c[0] * nb[1] + c[1]) * nb[2] + c[2]) * nb[3] + c[3];
  }
  // is the hop x -> x +/- mu internal to x's block (does not cross a block face)?
  bool internal(int64_t x, int mu, int dir) const {
    int c[4]; g.coords(x, c);
    int p = c[mu] % bs[mu];
    return dir == 0 ? (p != bs[mu] - 1) : (p != 0);
  }
};

struct FgcrResult { int iters, restarts; double relres; int converged; };

typedef std::function<void(const cplx*, cplx*)> LinOp;

struct Deflation {
  Blocks B;
  int Ns;
  std::vector<cplx> W;      // Ns full fields, W[l*V*12 + x*12 + k]
  std::vector<cplx> little; // [nblk][9][Ns][Ns]
  Deflation(const Geom& g, const int* bs, int ns) : B(g, bs), Ns(ns) {}
};


// Dirichlet block solves by BiCGstab on a list of blocks (orc_solve.cpp)
void block_bicgstab(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const int* bs,
                    const int64_t* blks, int64_t nlist, const cplx* eta, cplx* psi, double tol, int maxit, int* iters,
                    double* res);
FgcrResult fgcr(int64_t n, const LinOp& op, const LinOp* prec, const cplx* eta, cplx* psi, int nkv, int nmx,
                double tol, double* history, int nhist);
void sap(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const int* bs, int ncy, int nmr,
         const cplx* eta, cplx* psi);
void sap_half_sweep(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const int* bs, int nmr,
                    int col, const cplx* eta, cplx* psi, cplx* rho);
void coarse_apply(const Deflation& d, const cplx* c, cplx* out);
void dfl_restrict(const Deflation& d, const cplx* r, cplx* c);
void dfl_prolong(const Deflation& d, const cplx* c, cplx* out);
FgcrResult coarse_solve(const Deflation& d, const cplx* f, cplx* c, double coarse_tol, int nkv, int nmx);
void dfl_build(Deflation& d, const cplx* U, const cplx* A, const cplx* Ainv, const int* sap_bs, int ncy,
               int nmr, int nit, const cplx* init);
void dfl_set_fields(Deflation& d, const cplx* U, const cplx* A, const cplx* fields);
void dfl_set_fields_on_blocks(Deflation& d, const cplx* U, const cplx* A, const cplx* fields,
                              const int64_t* blocks, int nblocks);
int sap_one_cycle_on_blocks(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const int* bs, int nmr,
                            const cplx* eta, const int64_t* blocks, int nblocks, cplx* psi);
void net_forward_on_sites(const Geom& g, const cplx* U, int nl, const int* ch, const cplx* W, const cplx* in,
                          const int64_t* sites, int nsites, cplx* out);
void dfl_precond(const Deflation& d, const cplx* U, const cplx* A, const cplx* Ainv, const int* sap_bs, int ncy,
                 int nmr, double coarse_tol, const cplx* r, cplx* out);
int dfl_net_precond(const Deflation& d, const cplx* U, const cplx* A, const cplx* Ainv, const int* sap_bs,
                    int ncy, int nmr, double coarse_tol, int nl, const int* ch, const cplx* W, const cplx* r,
                    cplx* out);

void net_layer_forward(const Geom& g, const cplx* U, int cin, int cout, const cplx* W, const cplx* in, cplx* out);
void net_layer_backward(const Geom& g, const cplx* U, int cin, int cout, const cplx* W, const cplx* in,
                        const cplx* gy, cplx* gx, cplx* gW);
void net_forward(const Geom& g, const cplx* U, int nl, const int* ch, const cplx* W, const cplx* in, cplx* out);
double net_loss_grad(const Geom& g, const cplx* U, int nl, const int* ch, const cplx* W, int nb, const cplx* r,
                     const cplx* e, cplx* grad);

// owning handle used by the C entry points
struct DflHandle {
  Geom* g;
  Deflation* d;
  DflHandle(Geom* g_, const int* bs, int Ns) : g(g_), d(new Deflation(*g_, bs, Ns)) {}
  ~DflHandle() { delete d; delete g; }
};

}  // namespace orc
