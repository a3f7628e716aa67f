// Oracle: Schwarz alternating procedure (SAP) with minimal-residual block
// solves, local deflation (little Dirac operator) and the flexible GCR outer
// solver -- the "locally deflated Schwarz-preconditioned GCR" the paper uses for
// its F2 inversions (Sect. 3 and Sect. 4, Table 1).  The paper names the method
// but does not restate its steps; the readings followed here are listed with
// each function.  TEST INFRASTRUCTURE ONLY (see orc_core.h).
#include "orc_dfl.h"
#include <functional>
#include <cstring>
#include <algorithm>

namespace orc {

// One term of the hopping sum: direction mu, dir 0 = forward (x+mu), 1 = backward.
// Accumulates scale * s (1 -/+ g_mu) U psi(y) into out12.
static void hop_term(const Geom& g, const cplx* U, const cplx* psi, int64_t x, int mu, int dir,
                     double scale, cplx* out) {
  const Gamma& G = gammas();
  int64_t y = dir == 0 ? g.up(x, mu) : g.dn(x, mu);
  double s = dir == 0 ? g.sign_up(x, mu) : g.sign_up(y, mu);
  const cplx* u = dir == 0 ? link(U, x, mu) : link(U, y, mu);
  cplx t[12];
  for (int sp = 0; sp < 4; ++sp)
    for (int a = 0; a < 3; ++a) {
      cplx acc = 0;
      for (int b = 0; b < 3; ++b)
        acc += (dir == 0 ? u[a * 3 + b] : std::conj(u[b * 3 + a])) * psi[y * 12 + sp * 3 + b];
      t[sp * 3 + a] = acc;
    }
  double pm = dir == 0 ? -1.0 : 1.0;
  for (int sa = 0; sa < 4; ++sa)
    for (int a = 0; a < 3; ++a) {
      cplx acc = t[sa * 3 + a];
      for (int sb = 0; sb < 4; ++sb) acc += pm * G.g[mu][sa][sb] * t[sb * 3 + a];
      out[sa * 3 + a] += scale * s * acc;
    }
}

// Dirichlet block operator applied at site x: hops that cross the block face are
// dropped.  Accumulates scale * H_Lambda psi(x).
static void hop_block(const Blocks& B, const cplx* U, const cplx* psi, int64_t x, double scale, cplx* out) {
  for (int mu = 0; mu < 4; ++mu)
    for (int dir = 0; dir < 2; ++dir)
      if (B.internal(x, mu, dir)) hop_term(B.g, U, psi, x, mu, dir, scale, out);
}

// Approximate block solve D_Lambda v = rho on one block (reading of the block
// solver, which the paper leaves to the cited SAP references): the source is
// reduced to the even sites of the block, nmr minimal-residual steps are taken on
// the block Schur complement Dhat_Lambda = A_e - D_eo,L A_o^{-1} D_oe,L starting
// from zero, and the odd sites are reconstructed.  rho, v: full-lattice fields;
// only the block's sites are read / written.
static void block_mr(const Blocks& B, int64_t blk, const cplx* U, const cplx* A, const cplx* Ainv,
                     const cplx* rho, cplx* v, int nmr, std::vector<cplx>& w1, std::vector<cplx>& w2,
                     std::vector<cplx>& w3, std::vector<cplx>& w4) {
  const Geom& g = B.g;
  const std::vector<int64_t>& st = B.sites[blk];
  std::vector<int64_t> ev, od;
  for (int64_t x : st) (g.parity(x) == 0 ? ev : od).push_back(x);
  // w1 = A_o^{-1} rho_o on odd sites of the block
  for (int64_t x : st) for (int k = 0; k < 12; ++k) w1[x * 12 + k] = 0;
  for (int64_t y : od) apply_clover_site(Ainv + y * 144, rho + y * 12, &w1[y * 12]);
  // b = rho_e - D_eo,L w1 = rho_e + 1/2 H_L w1  -> stored in w2 (r) ; x in w3
  for (int64_t x : ev) {
    cplx h[12] = {};
    hop_block(B, U, w1.data(), x, 0.5, h);
    for (int k = 0; k < 12; ++k) { w2[x * 12 + k] = rho[x * 12 + k] + h[k]; w3[x * 12 + k] = 0; }
  }
  for (int it = 0; it < nmr; ++it) {
    // p = Dhat_L r : w1_o = A_o^{-1}(-1/2 H_L r), p_e = A_e r + 1/2 H_L w1   (p -> w4)
    for (int64_t y : od) {
      cplx h[12] = {};
      hop_block(B, U, w2.data(), y, -0.5, h);
      apply_clover_site(Ainv + y * 144, h, &w1[y * 12]);
    }
    for (int64_t x : ev) {
      cplx o[12];
      apply_clover_site(A + x * 144, &w2[x * 12], o);
      hop_block(B, U, w1.data(), x, 0.5, o);
      for (int k = 0; k < 12; ++k) w4[x * 12 + k] = o[k];
    }
    // alpha = <p, r> / <p, p>
    cplx pr = 0;
    double pp = 0;
    for (int64_t x : ev)
      for (int k = 0; k < 12; ++k) {
        pr += std::conj(w4[x * 12 + k]) * w2[x * 12 + k];
        pp += std::norm(w4[x * 12 + k]);
      }
    cplx alpha = pp > 0 ? pr / pp : cplx(0);
    for (int64_t x : ev)
      for (int k = 0; k < 12; ++k) {
        w3[x * 12 + k] += alpha * w2[x * 12 + k];
        w2[x * 12 + k] -= alpha * w4[x * 12 + k];
      }
  }
  // v_e = x ; v_o = A_o^{-1} (rho_o - D_oe,L v_e) = A_o^{-1}(rho_o + 1/2 H_L v_e)
  for (int64_t x : ev) for (int k = 0; k < 12; ++k) v[x * 12 + k] = w3[x * 12 + k];
  for (int64_t y : od) {
    cplx h[12];
    for (int k = 0; k < 12; ++k) h[k] = rho[y * 12 + k];
    hop_block(B, U, w3.data(), y, 0.5, h);
    apply_clover_site(Ainv + y * 144, h, &v[y * 12]);
  }
}

// ---------------------------------------------------------------------------
// Dirichlet block solves D_Lambda psi = eta on a list of blocks: the block
// inversions of the DD-HMC forces, which the paper does with BiCGstab (Sect. 3).
// D_Lambda is D restricted to the block (hops that cross a block face dropped).
// The source is reduced to the block's even sites, b = eta_e - D_eo,L A_o^{-1} eta_o;
// BiCGstab (van der Vorst) on Dhat_Lambda = A_e - D_eo,L A_o^{-1} D_oe,L runs from
// zero until |r| <= tol |b| or maxit iterations; then
// psi_o = A_o^{-1}(eta_o - D_oe,L psi_e).  Fields are full-lattice; only the
// listed blocks' sites of psi are written.  iters[k] gets the iterations of the
// k-th listed block (-1 after a breakdown, a zero denominator), res[k] |r|/|b|.
namespace {
struct BlockLocal {
  const Blocks& B;
  int o[4];
  int64_t nsb;
  BlockLocal(const Blocks& B_, int64_t blk) : B(B_) {
    int c[4];
    B.bcoords(blk, c);
    nsb = 1;
    for (int i = 0; i < 4; ++i) { o[i] = c[i] * B.bs[i]; nsb *= B.bs[i]; }
  }
  int64_t local(int64_t x) const {  // block-local lexicographic index of site x
    int c[4];
    B.g.coords(x, c);
    return (((int64_t)(c[0] - o[0]) * B.bs[1] + (c[1] - o[1])) * B.bs[2] + (c[2] - o[2])) * B.bs[3] + (c[3] - o[3]);
  }
};

// out += scale * H_Lambda f at site x; f holds the block's sites by local index
void hop_local(const BlockLocal& L, const cplx* U, const cplx* f, int64_t x, double scale, cplx* out) {
  const Geom& g = L.B.g;
  const Gamma& G = gammas();
  for (int mu = 0; mu < 4; ++mu)
    for (int dir = 0; dir < 2; ++dir) {
      if (!L.B.internal(x, mu, dir)) continue;
      const int64_t y = dir == 0 ? g.up(x, mu) : g.dn(x, mu);
      const double s = dir == 0 ? g.sign_up(x, mu) : g.sign_up(y, mu);
      const cplx* u = dir == 0 ? link(U, x, mu) : link(U, y, mu);
      const cplx* v = f + L.local(y) * 12;
      cplx t[12];
      for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) {
          cplx acc = 0;
          for (int b = 0; b < 3; ++b) acc += (dir == 0 ? u[a * 3 + b] : std::conj(u[b * 3 + a])) * v[sp * 3 + b];
          t[sp * 3 + a] = acc;
        }
      const double pm = dir == 0 ? -1.0 : 1.0;
      for (int sa = 0; sa < 4; ++sa)
        for (int a = 0; a < 3; ++a) {
          cplx acc = t[sa * 3 + a];
          for (int sb = 0; sb < 4; ++sb) acc += pm * G.g[mu][sa][sb] * t[sb * 3 + a];
          out[sa * 3 + a] += scale * s * acc;
        }
    }
}
}  // namespace

void block_bicgstab(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const int* bs,
                    const int64_t* blks, int64_t nlist, const cplx* eta, cplx* psi, double tol, int maxit, int* iters,
                    double* res) {
  Blocks B(g, bs);
#pragma omp parallel for schedule(dynamic)
  for (int64_t k = 0; k < nlist; ++k) {
    const int64_t blk = blks[k];
    BlockLocal L(B, blk);
    const std::vector<int64_t>& st = B.sites[blk];
    std::vector<int64_t> ev, od;
    for (int64_t x : st) (g.parity(x) == 0 ? ev : od).push_back(x);
    const int64_t n = L.nsb * 12;
    // local vectors (even entries used for the Krylov vectors, odd for the intermediates)
    std::vector<cplx> w(n), b(n), x(n), r(n), rh(n), p(n), v(n), sv(n), t(n);
    auto local = [&](int64_t y) { return L.local(y) * 12; };
    // Dhat_Lambda in (even) -> out (even), with D_eo,L = -1/2 H_L:
    // w_o = A_o^{-1} D_oe,L in = A_o^{-1} (-1/2 H_L in), out_e = A_e in - D_eo,L w_o = A_e in + 1/2 H_L w_o
    auto dhat = [&](const std::vector<cplx>& in, std::vector<cplx>& out) {
      for (int64_t y : od) {
        cplx h[12] = {};
        hop_local(L, U, in.data(), y, -0.5, h);
        apply_clover_site(Ainv + y * 144, h, &w[local(y)]);
      }
      for (int64_t z : ev) {
        cplx o[12];
        apply_clover_site(A + z * 144, &in[local(z)], o);
        hop_local(L, U, w.data(), z, 0.5, o);
        for (int c = 0; c < 12; ++c) out[local(z) + c] = o[c];
      }
    };
    auto dotp = [&](const std::vector<cplx>& a, const std::vector<cplx>& c) {
      cplx acc = 0;
      for (int64_t z : ev)
        for (int q = 0; q < 12; ++q) acc += std::conj(a[local(z) + q]) * c[local(z) + q];
      return acc;
    };
    // b = eta_e - D_eo,L A_o^{-1} eta_o = eta_e + 1/2 H_L (A_o^{-1} eta_o)
    for (int64_t y : od) apply_clover_site(Ainv + y * 144, eta + y * 12, &w[local(y)]);
    for (int64_t z : ev) {
      cplx h[12] = {};
      hop_local(L, U, w.data(), z, 0.5, h);
      for (int c = 0; c < 12; ++c) b[local(z) + c] = eta[z * 12 + c] + h[c];
    }
    // BiCGstab from x = 0
    r = b;
    rh = b;
    const double bn = std::sqrt(dotp(b, b).real());
    cplx rho = 1, alpha = 1, omega = 1;
    int it = 0;
    double rn = bn;
    bool broke = false;
    while (rn > tol * bn && it < maxit) {
      const cplx rho_new = dotp(rh, r);
      const cplx beta = (rho_new / rho) * (alpha / omega);
      for (int64_t z : ev)
        for (int q = 0; q < 12; ++q) {
          const int64_t i = local(z) + q;
          p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
      dhat(p, v);
      const cplx rv = dotp(rh, v);
      if (rv == cplx(0)) { broke = true; break; }
      alpha = rho_new / rv;
      for (int64_t z : ev)
        for (int q = 0; q < 12; ++q) sv[local(z) + q] = r[local(z) + q] - alpha * v[local(z) + q];
      dhat(sv, t);
      const double tt = dotp(t, t).real();
      if (tt == 0) { broke = true; break; }
      omega = dotp(t, sv) / tt;
      for (int64_t z : ev)
        for (int q = 0; q < 12; ++q) {
          const int64_t i = local(z) + q;
          x[i] += alpha * p[i] + omega * sv[i];
          r[i] = sv[i] - omega * t[i];
        }
      rho = rho_new;
      rn = std::sqrt(dotp(r, r).real());
      ++it;
    }
    iters[k] = broke ? -1 : it;
    res[k] = bn > 0 ? rn / bn : 0.0;
    // psi_e = x, psi_o = A_o^{-1}(eta_o - D_oe,L psi_e) = A_o^{-1}(eta_o + 1/2 H_L psi_e)
    for (int64_t z : ev)
      for (int c = 0; c < 12; ++c) psi[z * 12 + c] = x[local(z) + c];
    for (int64_t y : od) {
      cplx h[12];
      for (int c = 0; c < 12; ++c) h[c] = eta[y * 12 + c];
      hop_local(L, U, x.data(), y, 0.5, h);
      apply_clover_site(Ainv + y * 144, h, &psi[y * 12]);
    }
  }
}

// Multiplicative two-colour Schwarz procedure (reading): psi = 0, rho = eta;
// ncy cycles, each over colour 0 then colour 1; all blocks of one colour are
// solved independently from the current residual, psi += v on those blocks,
// then the residual is recomputed as rho = eta - D psi.
void sap(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const int* bs, int ncy, int nmr,
         const cplx* eta, cplx* psi) {
  Blocks B(g, bs);
  int64_t n = g.V * 12;
  std::vector<cplx> rho(eta, eta + n), v(n, 0.0), Dpsi(n);
  for (int64_t i = 0; i < n; ++i) psi[i] = 0;
  for (int cy = 0; cy < ncy; ++cy)
    for (int col = 0; col < 2; ++col) {
#pragma omp parallel
      {
        std::vector<cplx> w1(n), w2(n), w3(n), w4(n);
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < B.nblk; ++b) {
          if (B.colour[b] != col) continue;
          block_mr(B, b, U, A, Ainv, rho.data(), v.data(), nmr, w1, w2, w3, w4);
          for (int64_t x : B.sites[b])
            for (int k = 0; k < 12; ++k) psi[x * 12 + k] += v[x * 12 + k];
        }
      }
      apply_D(g, U, A, psi, Dpsi.data());
      for (int64_t i = 0; i < n; ++i) rho[i] = eta[i] - Dpsi[i];
    }
}

// One colour half-sweep on given (psi, rho): exposes the block solves for tests.
// Blocks of colour `col` are solved from rho, psi += v; rho is then recomputed.
void sap_half_sweep(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const int* bs, int nmr,
                    int col, const cplx* eta, cplx* psi, cplx* rho) {
  Blocks B(g, bs);
  int64_t n = g.V * 12;
  std::vector<cplx> v(n, 0.0), Dpsi(n), w1(n), w2(n), w3(n), w4(n);
  for (int64_t b = 0; b < B.nblk; ++b) {
    if (B.colour[b] != col) continue;
    block_mr(B, b, U, A, Ainv, rho, v.data(), nmr, w1, w2, w3, w4);
    for (int64_t x : B.sites[b])
      for (int k = 0; k < 12; ++k) psi[x * 12 + k] += v[x * 12 + k];
  }
  apply_D(g, U, A, psi, Dpsi.data());
  for (int64_t i = 0; i < n; ++i) rho[i] = eta[i] - Dpsi[i];
}

// The first cycle of the Schwarz procedure (ncy = 1) evaluated only where a
// list of colour-1 blocks needs it, for checks at sizes where the full sweep is
// too slow: the face neighbours of the listed blocks (colour 0) are solved from
// rho = eta, the residual eta - D psi is formed on the listed blocks exactly as
// sap() forms it (per site, the clover term and then the hops), and the listed
// blocks are solved from it.  psi (full field, zeroed here) then holds the
// values sap(ncy = 1) gives on the listed blocks and on their face neighbours.
// Returns -1 (psi untouched) if a listed block is not of colour 1 or a face
// neighbour is not of colour 0, else 0.
int sap_one_cycle_on_blocks(const Geom& g, const cplx* U, const cplx* A, const cplx* Ainv, const int* bs, int nmr,
                            const cplx* eta, const int64_t* blocks, int nblocks, cplx* psi) {
  Blocks B(g, bs);
  int64_t n = g.V * 12;
  std::vector<int64_t> black;
  for (int i = 0; i < nblocks; ++i) {
    if (blocks[i] < 0 || blocks[i] >= B.nblk || B.colour[blocks[i]] != 1) return -1;
    for (int d = 1; d <= 8; ++d) {
      int64_t nb = B.nbr(blocks[i], d);
      if (B.colour[nb] != 0) return -1;
      if (std::find(black.begin(), black.end(), nb) == black.end()) black.push_back(nb);
    }
  }
  std::fill(psi, psi + n, cplx(0));
  std::vector<cplx> rho(eta, eta + n), v(n, 0.0), w1(n), w2(n), w3(n), w4(n);
  for (int64_t b : black) {
    block_mr(B, b, U, A, Ainv, rho.data(), v.data(), nmr, w1, w2, w3, w4);
    for (int64_t x : B.sites[b])
      for (int k = 0; k < 12; ++k) psi[x * 12 + k] += v[x * 12 + k];
  }
  for (int i = 0; i < nblocks; ++i)
    for (int64_t x : B.sites[blocks[i]]) {
      cplx o[12];
      apply_clover_site(A + x * 144, psi + x * 12, o);
      hop_site(g, U, psi, x, -0.5, o, nullptr);
      for (int k = 0; k < 12; ++k) rho[x * 12 + k] = eta[x * 12 + k] - o[k];
    }
  for (int i = 0; i < nblocks; ++i) {
    block_mr(B, blocks[i], U, A, Ainv, rho.data(), v.data(), nmr, w1, w2, w3, w4);
    for (int64_t x : B.sites[blocks[i]])
      for (int k = 0; k < 12; ++k) psi[x * 12 + k] += v[x * 12 + k];
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Flexible GCR (textbook restarted FGCR; reading of the paper's outer solver):
// phi_k = M(r_k), chi_k = A phi_k, classical Gram-Schmidt of chi_k against the
// earlier chi_l with one re-orthogonalisation pass, r_{k+1} = r_k - c_k chi_k;
// at the end of a cycle the triangular system is back-substituted, psi is
// updated and the residual is recomputed from the operator.
FgcrResult fgcr(int64_t n, const LinOp& op, const LinOp* prec, const cplx* eta, cplx* psi, int nkv, int nmx,
                double tol, double* history, int nhist) {
  FgcrResult res{0, 0, 0.0, 0};
  std::vector<std::vector<cplx>> phi(nkv, std::vector<cplx>(n)), chi(nkv, std::vector<cplx>(n));
  std::vector<cplx> r(n), tmp(n);
  std::vector<cplx> a(nkv * nkv), c(nkv), alpha(nkv);
  std::vector<double> b(nkv);
  double eta_norm = std::sqrt(norm2(eta, n));
  if (eta_norm == 0) {
    for (int64_t i = 0; i < n; ++i) psi[i] = 0;
    res.converged = 1;
    return res;
  }
  op(psi, tmp.data());
  for (int64_t i = 0; i < n; ++i) r[i] = eta[i] - tmp[i];
  double rn = std::sqrt(norm2(r.data(), n));
  if (history && nhist > 0) history[0] = rn / eta_norm;
  while (res.iters < nmx) {
    if (rn <= tol * eta_norm) { res.converged = 1; break; }
    int k = 0;
    for (; k < nkv && res.iters < nmx; ++k) {
      if (prec) (*prec)(r.data(), phi[k].data());
      else std::copy(r.begin(), r.end(), phi[k].begin());
      op(phi[k].data(), chi[k].data());
      for (int l = 0; l < k; ++l) a[l * nkv + k] = 0;
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<cplx> proj(k);
        for (int l = 0; l < k; ++l) proj[l] = dot(chi[l].data(), chi[k].data(), n);
        for (int l = 0; l < k; ++l) {
          a[l * nkv + k] += proj[l];
          for (int64_t i = 0; i < n; ++i) chi[k][i] -= proj[l] * chi[l][i];
        }
      }
      b[k] = std::sqrt(norm2(chi[k].data(), n));
      for (int64_t i = 0; i < n; ++i) chi[k][i] /= b[k];
      c[k] = dot(chi[k].data(), r.data(), n);
      for (int64_t i = 0; i < n; ++i) r[i] -= c[k] * chi[k][i];
      rn = std::sqrt(norm2(r.data(), n));
      res.iters++;
      if (history && res.iters < nhist) history[res.iters] = rn / eta_norm;
      if (rn <= tol * eta_norm) { ++k; break; }
    }
    // back substitution: b_j alpha_j + sum_{l>j} a_jl alpha_l = c_j
    for (int j = k - 1; j >= 0; --j) {
      cplx s = c[j];
      for (int l = j + 1; l < k; ++l) s -= a[j * nkv + l] * alpha[l];
      alpha[j] = s / b[j];
    }
    for (int j = 0; j < k; ++j)
      for (int64_t i = 0; i < n; ++i) psi[i] += alpha[j] * phi[j][i];
    op(psi, tmp.data());
    for (int64_t i = 0; i < n; ++i) r[i] = eta[i] - tmp[i];
    rn = std::sqrt(norm2(r.data(), n));
    if (!std::isfinite(rn)) break;
    if (rn <= tol * eta_norm) { res.converged = 1; break; }
    res.restarts++;
  }
  res.relres = rn / eta_norm;
  return res;
}

// ---------------------------------------------------------------------------
// Local deflation (reading of the deflation subspace construction the paper
// cites): Ns start fields (passed in, so that both implementations see the same
// random numbers) are improved by nit rounds of phi <- M_sap(phi), each followed
// by normalisation; then on every deflation block the block projections of the
// Ns fields are orthonormalised (Gram-Schmidt, ascending l, two passes).
// The little Dirac operator A_{bk, b'l} = <w_bk, D w_b'l> is stored per block as
// 9 Ns x Ns matrices: index 0 = the block with itself (hops inside the block),
// 1+2mu / 2+2mu = the coupling through the block's upper / lower face in mu.
static std::vector<int64_t> all_blocks(const Blocks& B) {
  std::vector<int64_t> b(B.nblk);
  for (int64_t i = 0; i < B.nblk; ++i) b[i] = i;
  return b;
}

static void dfl_orthonormalise(Deflation& d, const std::vector<int64_t>& blocks) {
  const Geom& g = d.B.g;
  int64_t V12 = g.V * 12;
#pragma omp parallel for schedule(dynamic)
  for (int64_t bi = 0; bi < (int64_t)blocks.size(); ++bi) {
    const int64_t b = blocks[bi];
    const std::vector<int64_t>& st = d.B.sites[b];
    for (int l = 0; l < d.Ns; ++l) {
      cplx* wl = &d.W[l * V12];
      for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < l; ++k) {
          const cplx* wk = &d.W[k * V12];
          cplx p = 0;
          for (int64_t x : st) for (int i = 0; i < 12; ++i) p += std::conj(wk[x * 12 + i]) * wl[x * 12 + i];
          for (int64_t x : st) for (int i = 0; i < 12; ++i) wl[x * 12 + i] -= p * wk[x * 12 + i];
        }
      double nn = 0;
      for (int64_t x : st) for (int i = 0; i < 12; ++i) nn += std::norm(wl[x * 12 + i]);
      double s = 1.0 / std::sqrt(nn);
      for (int64_t x : st) for (int i = 0; i < 12; ++i) wl[x * 12 + i] *= s;
    }
  }
}

static void dfl_little(Deflation& d, const cplx* U, const cplx* A, const std::vector<int64_t>& blocks) {
  const Geom& g = d.B.g;
  const Blocks& B = d.B;
  int Ns = d.Ns;
  int64_t V12 = g.V * 12;
  d.little.assign(B.nblk * 9 * Ns * Ns, 0.0);
#pragma omp parallel for schedule(dynamic)
  for (int64_t bi = 0; bi < (int64_t)blocks.size(); ++bi) {
    const int64_t b = blocks[bi];
    const std::vector<int64_t>& st = B.sites[b];
    for (int l = 0; l < Ns; ++l) {
      const cplx* wl = &d.W[l * V12];
      // self: (A - 1/2 H_internal) w_bl, projected on w_bk
      std::vector<cplx> y(st.size() * 12);
      for (size_t i = 0; i < st.size(); ++i) {
        int64_t x = st[i];
        apply_clover_site(A + x * 144, wl + x * 12, &y[i * 12]);
        for (int mu = 0; mu < 4; ++mu)
          for (int dir = 0; dir < 2; ++dir)
            if (B.internal(x, mu, dir)) hop_term(g, U, wl, x, mu, dir, -0.5, &y[i * 12]);
      }
      for (int k = 0; k < Ns; ++k) {
        const cplx* wk = &d.W[k * V12];
        cplx s = 0;
        for (size_t i = 0; i < st.size(); ++i)
          for (int j = 0; j < 12; ++j) s += std::conj(wk[st[i] * 12 + j]) * y[i * 12 + j];
        d.little[((b * 9 + 0) * Ns + k) * Ns + l] = s;
      }
      // faces: -1/2 of the face hop from the neighbouring block's w_{b',l}
      for (int mu = 0; mu < 4; ++mu)
        for (int dir = 0; dir < 2; ++dir) {
          int di = 1 + 2 * mu + dir;
          std::fill(y.begin(), y.end(), cplx(0));
          for (size_t i = 0; i < st.size(); ++i) {
            int64_t x = st[i];
            if (!B.internal(x, mu, dir)) hop_term(g, U, wl, x, mu, dir, -0.5, &y[i * 12]);
          }
          for (int k = 0; k < Ns; ++k) {
            const cplx* wk = &d.W[k * V12];
            cplx s = 0;
            for (size_t i = 0; i < st.size(); ++i)
              for (int j = 0; j < 12; ++j) s += std::conj(wk[st[i] * 12 + j]) * y[i * 12 + j];
            d.little[((b * 9 + di) * Ns + k) * Ns + l] = s;
          }
        }
    }
  }
}

// face index d = 1 + 2 mu + dir, dir 0 = up; the neighbouring block across it
static int64_t face_nbr(const Blocks& B, int64_t b, int d) {
  int mu = (d - 1) / 2, dir = (d - 1) % 2;
  return B.nbr(b, dir == 0 ? 1 + 2 * mu : 2 + 2 * mu);
}

void coarse_apply(const Deflation& d, const cplx* c, cplx* out) {
  int Ns = d.Ns;
  const Blocks& B = d.B;
  for (int64_t b = 0; b < B.nblk; ++b)
    for (int k = 0; k < Ns; ++k) {
      cplx s = 0;
      for (int di = 0; di < 9; ++di) {
        int64_t bb = di == 0 ? b : face_nbr(B, b, di);
        const cplx* m = &d.little[((b * 9 + di) * Ns + k) * Ns];
        for (int l = 0; l < Ns; ++l) s += m[l] * c[bb * Ns + l];
      }
      out[b * Ns + k] = s;
    }
}

void dfl_restrict(const Deflation& d, const cplx* r, cplx* c) {
  int64_t V12 = d.B.g.V * 12;
  for (int64_t b = 0; b < d.B.nblk; ++b)
    for (int k = 0; k < d.Ns; ++k) {
      cplx s = 0;
      for (int64_t x : d.B.sites[b])
        for (int i = 0; i < 12; ++i) s += std::conj(d.W[k * V12 + x * 12 + i]) * r[x * 12 + i];
      c[b * d.Ns + k] = s;
    }
}

void dfl_prolong(const Deflation& d, const cplx* c, cplx* out) {
  int64_t V12 = d.B.g.V * 12;
  for (int64_t b = 0; b < d.B.nblk; ++b)
    for (int64_t x : d.B.sites[b])
      for (int i = 0; i < 12; ++i) {
        cplx s = 0;
        for (int k = 0; k < d.Ns; ++k) s += d.W[k * V12 + x * 12 + i] * c[b * d.Ns + k];
        out[x * 12 + i] = s;
      }
}

// coarse solve A c = f: unpreconditioned GCR on the little operator to coarse_tol
FgcrResult coarse_solve(const Deflation& d, const cplx* f, cplx* c, double coarse_tol, int nkv, int nmx) {
  int64_t n = d.B.nblk * d.Ns;
  for (int64_t i = 0; i < n; ++i) c[i] = 0;
  LinOp op = [&](const cplx* in, cplx* out) { coarse_apply(d, in, out); };
  return fgcr(n, op, nullptr, f, c, nkv, nmx, coarse_tol, nullptr, 0);
}

void dfl_build(Deflation& d, const cplx* U, const cplx* A, const cplx* Ainv, const int* sap_bs, int ncy,
               int nmr, int nit, const cplx* init) {
  const Geom& g = d.B.g;
  int64_t V12 = g.V * 12;
  d.W.assign(init, init + d.Ns * V12);
  std::vector<cplx> tmp(V12);
  for (int it = 0; it < nit; ++it)
    for (int l = 0; l < d.Ns; ++l) {
      sap(g, U, A, Ainv, sap_bs, ncy, nmr, &d.W[l * V12], tmp.data());
      double s = 1.0 / std::sqrt(norm2(tmp.data(), V12));
      for (int64_t i = 0; i < V12; ++i) d.W[l * V12 + i] = tmp[i] * s;
    }
  dfl_orthonormalise(d, all_blocks(d.B));
  dfl_little(d, U, A, all_blocks(d.B));
}

// Two-level preconditioner (reading: inexact deflation): M(r) = C r + M_sap(r - D C r),
// C = W A^{-1} W^dag with the coarse system solved to coarse_tol.
void dfl_precond(const Deflation& d, const cplx* U, const cplx* A, const cplx* Ainv, const int* sap_bs, int ncy,
                 int nmr, double coarse_tol, const cplx* r, cplx* out) {
  const Geom& g = d.B.g;
  int64_t V12 = g.V * 12, nc = d.B.nblk * d.Ns;
  std::vector<cplx> cr(nc), cc(nc), Cr(V12), DCr(V12), r1(V12), s(V12);
  dfl_restrict(d, r, cr.data());
  coarse_solve(d, cr.data(), cc.data(), coarse_tol, 32, 100000);
  dfl_prolong(d, cc.data(), Cr.data());
  apply_D(g, U, A, Cr.data(), DCr.data());
  for (int64_t i = 0; i < V12; ++i) r1[i] = r[i] - DCr[i];
  sap(g, U, A, Ainv, sap_bs, ncy, nmr, r1.data(), s.data());
  for (int64_t i = 0; i < V12; ++i) out[i] = Cr[i] + s[i];
}

// Install given fields as the (un-orthonormalised) subspace, skipping the SAP
// iterations: used by tests that pin the orthonormalisation and the little
// operator on known inputs.
void dfl_set_fields(Deflation& d, const cplx* U, const cplx* A, const cplx* fields) {
  int64_t V12 = d.B.g.V * 12;
  d.W.assign(fields, fields + d.Ns * V12);
  dfl_orthonormalise(d, all_blocks(d.B));
  dfl_little(d, U, A, all_blocks(d.B));
}

// The same restricted to a list of blocks, for checks at sizes where the full
// little operator is too slow: the listed blocks and their face neighbours are
// orthonormalised, and the little-operator rows of the listed blocks (self and
// the 8 face couplings) are computed; they equal those of dfl_set_fields.  Basis
// values on other blocks stay un-orthonormalised, other rows zero.
void dfl_set_fields_on_blocks(Deflation& d, const cplx* U, const cplx* A, const cplx* fields,
                              const int64_t* blocks, int nblocks) {
  int64_t V12 = d.B.g.V * 12;
  d.W.assign(fields, fields + d.Ns * V12);
  std::vector<int64_t> rows(blocks, blocks + nblocks), orth;
  for (int64_t b : rows) {
    orth.push_back(b);
    for (int f = 1; f <= 8; ++f) orth.push_back(d.B.nbr(b, f));
  }
  std::sort(orth.begin(), orth.end());
  orth.erase(std::unique(orth.begin(), orth.end()), orth.end());
  dfl_orthonormalise(d, orth);
  dfl_little(d, U, A, rows);
}

// Two-level preconditioner with the network stage (reading of the learned
// stage): r1 = r - D C r, v_n = N(r1), r2 = r1 - D v_n, and
// M(r) = C r + v_n + M_sap(r2).  If |r2| > |r1| or r2 is not finite the network
// output is dropped (fallback to plain M(r) = C r + M_sap(r1)).  Returns 1 on
// fallback, else 0.
int dfl_net_precond(const Deflation& d, const cplx* U, const cplx* A, const cplx* Ainv, const int* sap_bs,
                    int ncy, int nmr, double coarse_tol, int nl, const int* ch, const cplx* W, const cplx* r,
                    cplx* out) {
  const Geom& g = d.B.g;
  int64_t V12 = g.V * 12, nc = d.B.nblk * d.Ns;
  std::vector<cplx> cr(nc), cc(nc), Cr(V12), DCr(V12), r1(V12), vn(V12), Dvn(V12), r2(V12), s(V12);
  dfl_restrict(d, r, cr.data());
  coarse_solve(d, cr.data(), cc.data(), coarse_tol, 32, 100000);
  dfl_prolong(d, cc.data(), Cr.data());
  apply_D(g, U, A, Cr.data(), DCr.data());
  for (int64_t i = 0; i < V12; ++i) r1[i] = r[i] - DCr[i];
  net_forward(g, U, nl, ch, W, r1.data(), vn.data());
  apply_D(g, U, A, vn.data(), Dvn.data());
  for (int64_t i = 0; i < V12; ++i) r2[i] = r1[i] - Dvn[i];
  double n1 = norm2(r1.data(), V12), n2 = norm2(r2.data(), V12);
  int fb = !(std::isfinite(n2) && n2 <= n1);
  if (fb) {
    r2 = r1;
    std::fill(vn.begin(), vn.end(), cplx(0));
  }
  sap(g, U, A, Ainv, sap_bs, ncy, nmr, r2.data(), s.data());
  for (int64_t i = 0; i < V12; ++i) out[i] = Cr[i] + vn[i] + s[i];
  return fb;
}

}  // namespace orc
