// Link derivatives of the effective action of Eq. 4 (the molecular-dynamics
// forces of Sect. 2) on gfx950, in FP64.
//
// A link is varied as U_mu(x) -> exp(eps w) U_mu(x), w traceless anti-Hermitian.
// For every link the kernels form the 3x3 matrix M whose Re tr(w M) is the
// first-order change of S_eff, as M = U S_f - S_b U^dag with U the bare link,
// and store f^a = Re tr(T^a M) for the generators T^a = i lambda^a / 2.
//  * clover part: a site's 12x12 weight K (the log-det term gives -2 A^{-1}, a
//    pseudofermion term outer products of its fields) enters through
//    Re tr(K dA) = sum over the six planes of Re tr(Lambda dF_{mu nu}), and with
//    F = (Q - Q^dag)/8 as Re tr(Lt dQ), Lt = (Lambda - Lambda^dag)/8 (anti-
//    Hermitian, 9 reals per plane and site).  The four leaves of Q through a link
//    put Lt at the four corners of the staples on either side of it.
//  * hopping part: for a term with fields X, Y (full fields: X, Y on the even
//    sites, their odd-site images on the odd ones) and weight c,
//    S_f += c s sum_spin Y(x+mu) ((1 - g_mu) X(x))^dag and
//    S_b += c s sum_spin Y(x) ((1 + g_mu) X(x+mu))^dag, s the boundary sign.
#include "qdd_kernels.h"
#include "qdd_su3.h"

namespace qdd {

// (1 + SG g_MU) in, chiral basis: g0 = [[0,-1],[-1,0]], gk = [[0,-i sk],[i sk,0]]
// on (upper, lower) spin pairs; component index 3 * spin + colour
template <int MU, int SG>
__device__ inline void proj_full(const zd in[12], zd out[12]) {
  const double sg = SG;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const zd u0 = in[c], u1 = in[3 + c], l0 = in[6 + c], l1 = in[9 + c];
    zd gu0, gu1, gl0, gl1;  // g_MU in
    if constexpr (MU == 0) {
      gu0 = -1.0 * l0, gu1 = -1.0 * l1, gl0 = -1.0 * u0, gl1 = -1.0 * u1;
    } else if constexpr (MU == 1) {  // s1 (v0, v1) = (v1, v0)
      gu0 = tmi(l1), gu1 = tmi(l0), gl0 = ti(u1), gl1 = ti(u0);
    } else if constexpr (MU == 2) {  // s2 (v0, v1) = (-i v1, i v0)
      gu0 = -1.0 * l1, gu1 = l0, gl0 = u1, gl1 = -1.0 * u0;
    } else {  // s3 (v0, v1) = (v0, -v1)
      gu0 = tmi(l0), gu1 = ti(l1), gl0 = ti(u0), gl1 = tmi(u1);
    }
    out[c] = u0 + sg * gu0;
    out[3 + c] = u1 + sg * gu1;
    out[6 + c] = l0 + sg * gl0;
    out[9 + c] = l1 + sg * gl1;
  }
}

__device__ inline void ld_aos(const double2* f, int64_t site, zd s[12]) {
  const double2* b = f + site * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) s[k] = {b[k].x, b[k].y};
}
__device__ inline void st_aos(double2* f, int64_t site, const zd s[12]) {
  double2* b = f + site * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = make_double2(s[k].re, s[k].im);
}

// acc += H f (one site of parity p, f: the opposite parity, [Vh][12] complex)
template <int MU, int SG>
__device__ inline void hop_aos(const Geo& g, const LinkV<double>& U, const double2* f, int p, int i, const int x[4],
                               zd (&acc)[12]) {
  zd u[9], s[12], h[6], gg[6];
  const int j = nbr_idx(g, x, MU, SG);
  if (SG > 0) ld_link_u<double>(U, p, MU, i, u);
  else ld_link_u<double>(U, 1 - p, MU, j, u);
  ld_aos(f, j, s);
  project<double, MU, SG>(s, h);
  su3_mul_half<double, (SG < 0)>(u, h, gg);
  reconstruct_add<double, MU, SG>(gg, acc, 1.0);
}
__device__ inline void hop_all_aos(const Geo& g, const LinkV<double>& U, const double2* f, int p, int i,
                                   const int x[4], zd (&acc)[12]) {
  hop_aos<0, 1>(g, U, f, p, i, x, acc);
  hop_aos<0, -1>(g, U, f, p, i, x, acc);
  hop_aos<1, 1>(g, U, f, p, i, x, acc);
  hop_aos<1, -1>(g, U, f, p, i, x, acc);
  hop_aos<2, 1>(g, U, f, p, i, x, acc);
  hop_aos<2, -1>(g, U, f, p, i, x, acc);
  hop_aos<3, 1>(g, U, f, p, i, x, acc);
  hop_aos<3, -1>(g, U, f, p, i, x, acc);
}

// odd-site images of the nt terms' fields, fields [t][parity][Vh][12]:
//   Y_o = A_o^{-1} H_oe Y_e,   X_o = g5 A_o^{-1} H_oe Z_e   (Z_e = g5 X_e, the
// even part as the solve left it: X_o = A_o^{-1} H_eo^dag X_e by g5-hermiticity)
__global__ void __launch_bounds__(128) k_force_odd(Geo g, LinkV<double> U, CloverV<double> Ai, int nt, double2* X,
                                                   double2* Y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  int x[4];
  site_coords(g, 1, i, x);
  const int64_t tstride = (int64_t)2 * g.Vh * 12, odd = (int64_t)g.Vh * 12;
  for (int t = 0; t < nt; ++t) {
#pragma unroll 1
    for (int w = 0; w < 2; ++w) {
      double2* f = (w == 0 ? Y : X) + t * tstride;
      zd acc[12], o[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = {0.0, 0.0};
      hop_all_aos(g, U, f, 1, i, x, acc);
      clover_apply_u<double>(Ai, 1, i, acc, o);
      if (w == 1)
#pragma unroll
        for (int k = 6; k < 12; ++k) o[k] = -1.0 * o[k];
      st_aos(f + odd, i, o);
    }
  }
}

// X_e = g5 Z_e in place (the even part of every term's X field)
__global__ void k_force_g5(int64_t Vh, int nt, double2* X) {
  const int64_t n = (int64_t)nt * Vh * 6, e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t t = e / (Vh * 6), r = e - t * Vh * 6, site = r / 6, k = 6 + r % 6;
  double2* p = X + t * 2 * Vh * 12 + site * 12 + k;
  *p = make_double2(-p->x, -p->y);
}

// sources of the adjoint solves: u_t = A_e^{-1} g5 w_t with w_0 = psi, w_1 = phi2 + dm xi
__global__ void __launch_bounds__(128) k_force_src(Geo g, CloverV<double> Ai, const double2* psi, const double2* xi,
                                                   const double2* phi2, double dm, double2* src) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
#pragma unroll 1
  for (int t = 0; t < 2; ++t) {
    zd w[12], o[12];
    ld_aos(t == 0 ? psi : xi, i, w);
    if (t == 1) {
      zd p2[12];
      ld_aos(phi2, i, p2);
#pragma unroll
      for (int k = 0; k < 12; ++k) w[k] = p2[k] + dm * w[k];
    }
#pragma unroll
    for (int k = 6; k < 12; ++k) w[k] = -1.0 * w[k];
    clover_apply_u<double>(Ai, 0, i, w, o);
    st_aos(src + (int64_t)t * g.Vh * 12, i, o);
  }
}

// planes: 0 (0,1), 1 (0,2), 2 (0,3), 3 (1,2), 4 (1,3), 5 (2,3).  The clover block
// of chirality blk (sg = +1, -1) holds (i c_sw/2) sum_k sigma_k (x) (sg F_0k - B_k),
// B_1 = F_23, B_2 = -F_13, B_3 = F_12: plane -> (Pauli index, coefficient / (c_sw/2))
__device__ inline void plane_sigma(int pl, int blk, int& k, double& cf) {
  const double sg = blk == 0 ? 1.0 : -1.0;
  switch (pl) {
    case 0: k = 1, cf = sg; break;
    case 1: k = 2, cf = sg; break;
    case 2: k = 3, cf = sg; break;
    case 3: k = 3, cf = -1.0; break;
    case 4: k = 2, cf = 1.0; break;
    default: k = 1, cf = -1.0; break;
  }
}

// G_ab = sum_{s,s'} K_{(s a),(s' b)} sigma_k[s'][s] for K = y x^dag (6-vectors of
// one chirality block): G = sum_{s'} (sigma_k y)_{s'} x_{s'}^dag
__device__ inline void sigma_outer(int k, const zd y[6], const zd x[6], double c, zd G[9]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    zd sy0, sy1;  // (sigma_k y)_{s'=0,1}, colour a
    if (k == 1) sy0 = y[3 + a], sy1 = y[a];
    else if (k == 2) sy0 = tmi(y[3 + a]), sy1 = ti(y[a]);
    else sy0 = y[a], sy1 = -1.0 * y[3 + a];
#pragma unroll
    for (int b = 0; b < 3; ++b) G[a * 3 + b] = G[a * 3 + b] + c * (sy0 * conj(x[b]) + sy1 * conj(x[3 + b]));
  }
}

// the same for K = c times the Hermitian 6x6 block stored in 18 slots
__device__ inline void sigma_herm(int k, const CloverV<double>& A, int p, int blk, int i, double c, zd G[9]) {
  zd M[36];
  const double2* b = A.p + ((int64_t)p * 36 + blk * 18) * A.n + i;
  const double2 d0 = b[0], d1 = b[A.n], d2 = b[2 * (int64_t)A.n];
  const double dg[6] = {d0.x, d0.y, d1.x, d1.y, d2.x, d2.y};
  int s = 3;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    M[r * 7] = {dg[r], 0.0};
#pragma unroll
    for (int q = r + 1; q < 6; ++q) {
      const double2 v = b[(int64_t)s * A.n];
      M[r * 6 + q] = {v.x, v.y};
      M[q * 6 + r] = {v.x, -v.y};
      ++s;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      const zd k00 = M[a * 6 + bb], k01 = M[a * 6 + 3 + bb], k10 = M[(3 + a) * 6 + bb], k11 = M[(3 + a) * 6 + 3 + bb];
      zd v;
      if (k == 1) v = k01 + k10;
      else if (k == 2) v = ti(k01) + tmi(k10);
      else v = k00 - k11;
      G[a * 3 + bb] = G[a * 3 + bb] + c * v;
    }
}

// clover insertions Lt of every site and plane, stored [p][plane][9][Vh]:
// (Im d0, Im d1, Im d2, z01, z02, z12) of the anti-Hermitian Lt
__global__ void __launch_bounds__(128) k_force_lt(Geo g, CloverV<double> Ai, double det_w, double csw, FrcTerms T,
                                                  double* lt) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= g.V) return;
  const int p = tid >= g.Vh, i = tid - p * g.Vh;
  const double h = 0.5 * csw;
  const int64_t tstride = (int64_t)2 * g.Vh * 12;
#pragma unroll 1
  for (int pl = 0; pl < 6; ++pl) {
    zd Lam[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Lam[k] = {0.0, 0.0};
#pragma unroll 1
    for (int blk = 0; blk < 2; ++blk) {
      int k;
      double cf;
      plane_sigma(pl, blk, k, cf);
      zd G[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) G[q] = {0.0, 0.0};
      if (det_w != 0.0) sigma_herm(k, Ai, p, blk, i, det_w, G);
#pragma unroll 1
      for (int t = 0; t < T.nt; ++t) {
        zd y[6], xv[6];
        const double2* Xf = T.X[t] + p * (int64_t)g.Vh * 12 + (int64_t)i * 12 + 6 * blk;
        const double2* Yf = T.Y[t] + p * (int64_t)g.Vh * 12 + (int64_t)i * 12 + 6 * blk;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          xv[q] = {Xf[q].x, Xf[q].y};
          y[q] = {Yf[q].x, Yf[q].y};
        }
        double c;
        if (p == 0) {  // (1 + s) Y - phi with weight -2c
          const double2* ph = T.phi[t] + (int64_t)i * 12 + 6 * blk;
#pragma unroll
          for (int q = 0; q < 6; ++q) y[q] = (1.0 + T.s[t]) * y[q] - zd{ph[q].x, ph[q].y};
          c = -2.0 * T.c[t];
        } else {  // odd images with weight -c/2
          c = -0.5 * T.c[t];
        }
        sigma_outer(k, y, xv, c, G);
      }
      // Lambda += cf h i G
#pragma unroll
      for (int q = 0; q < 9; ++q) Lam[q] = Lam[q] + (cf * h) * ti(G[q]);
    }
    double* o = lt + ((int64_t)(p * 6 + pl) * 9) * g.Vh + i;
    const int64_t n = g.Vh;
    o[0] = 0.25 * Lam[0].im;  // (Lam - Lam^dag)/8 on the diagonal: i Im(Lam_aa) / 4
    o[n] = 0.25 * Lam[4].im;
    o[2 * n] = 0.25 * Lam[8].im;
    const int od[3][2] = {{0, 1}, {0, 2}, {1, 2}};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const zd ab = Lam[od[q][0] * 3 + od[q][1]], ba = Lam[od[q][1] * 3 + od[q][0]];
      o[(3 + 2 * q) * n] = 0.125 * (ab.re - ba.re);
      o[(4 + 2 * q) * n] = 0.125 * (ab.im + ba.im);
    }
  }
}

__device__ inline M3 ld_lt(const Geo& g, const double* lt, const int y[4], int pl) {
  const int lex = lex_of(g, y), p = (y[0] + y[1] + y[2] + y[3]) & 1;
  const int64_t n = g.Vh;
  const double* b = lt + ((int64_t)(p * 6 + pl) * 9) * n + (lex >> 1);
  M3 m;
  m.a[0] = {0.0, b[0]};
  m.a[4] = {0.0, b[n]};
  m.a[8] = {0.0, b[2 * n]};
  const zd z01{b[3 * n], b[4 * n]}, z02{b[5 * n], b[6 * n]}, z12{b[7 * n], b[8 * n]};
  m.a[1] = z01, m.a[3] = -1.0 * conj(z01);
  m.a[2] = z02, m.a[6] = -1.0 * conj(z02);
  m.a[5] = z12, m.a[7] = -1.0 * conj(z12);
  return m;
}

__device__ inline M3 add(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.a[k] = a.a[k] + b.a[k];
  return r;
}
__device__ inline M3 dag(const M3& a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[i * 3 + j] = conj(a.a[j * 3 + i]);
  return r;
}

// B1 B2 B3 with Lt inserted before B1 (lf), between B1 and B2 (lm), between B2
// and B3 (ll) and after B3 (le): ((lf B1 + B1 lm) B2 + B1 B2 ll) B3 + B1 B2 B3 le
__device__ inline M3 staple_after(const M3& B1, const M3& B2, const M3& B3, const M3& lf, const M3& lm, const M3& ll,
                                  const M3& le) {
  const M3 b12 = mul(B1, B2);
  const M3 t = add(mul(add(mul(lf, B1), mul(B1, lm)), B2), mul(b12, ll));
  return add(mul(t, B3), mul(mul(b12, B3), le));
}
// C1 C2 C3 with Lt between C1 and C2 (lf), between C2 and C3 (lm), after C3 (ll)
// and before C1 (ls): C1 ((lf C2 + C2 lm) C3 + C2 C3 ll) + ls C1 C2 C3
__device__ inline M3 staple_before(const M3& C1, const M3& C2, const M3& C3, const M3& lf, const M3& lm,
                                   const M3& ll, const M3& ls) {
  const M3 c23 = mul(C2, C3);
  const M3 t = add(mul(add(mul(lf, C2), mul(C2, lm)), C3), mul(c23, ll));
  return add(mul(C1, t), mul(ls, mul(C1, c23)));
}

__device__ inline int plane_of(int a, int b) {  // a < b
  return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

// S += w sum_spin b_s (P a)_s^dag with P = 1 + SG g_MU
template <int MU, int SG>
__device__ inline void outer_proj(const zd a[12], const zd b[12], double w, M3& S) {
  zd pa[12];
  proj_full<MU, SG>(a, pa);
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      zd s{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) s = s + b[q * 3 + j] * conj(pa[q * 3 + k]);
      S.a[j * 3 + k] = S.a[j * 3 + k] + w * s;
    }
}

// hopping part of the link (x, MU), x of parity p and index i:
//   Sf += c/2 s sum_spin Y(x+MU) ((1 - g_MU) X(x))^dag,  Sb += c/2 s sum_spin Y(x) ((1 + g_MU) X(x+MU))^dag
template <int MU>
__device__ inline void hop_force_part(const Geo& g, const int x[4], int p, int i, const FrcTerms& T, M3& Sf, M3& Sb) {
  const double sgn = (MU == 0 && x[0] == g.L[0] - 1) ? (double)g.bc : 1.0;
  int xp[4];
  shift(g, x, MU, 1, xp);
  const int64_t sx = (int64_t)p * g.Vh + i, sp = (int64_t)(1 - p) * g.Vh + (lex_of(g, xp) >> 1);
#pragma unroll 1
  for (int t = 0; t < T.nt; ++t) {
    const double w = 0.5 * T.c[t] * sgn;
    zd a[12], b[12];
    ld_aos(T.X[t], sx, a);
    ld_aos(T.Y[t], sp, b);
    outer_proj<MU, -1>(a, b, w, Sf);
    ld_aos(T.X[t], sp, a);
    ld_aos(T.Y[t], sx, b);
    outer_proj<MU, 1>(a, b, w, Sb);
  }
}

// one thread per link (mu, parity, site)
__global__ void __launch_bounds__(128) k_force_link(Geo g, const double2* U, const double* lt, int clov, FrcTerms T,
                                                    double* force) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)4 * g.V) return;
  const int mu = (int)(tid / g.V), r = (int)(tid - (int64_t)mu * g.V);
  const int p = r >= g.Vh, i = r - p * g.Vh;
  int x[4];
  site_coords(g, p, i, x);
  M3 Sf, Sb;
#pragma unroll
  for (int k = 0; k < 9; ++k) Sf.a[k] = Sb.a[k] = {0.0, 0.0};
  if (clov) {
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
      if (nu == mu) continue;
      const int a = mu < nu ? mu : nu, b = mu < nu ? nu : mu, pl = plane_of(a, b);
      int xa[4], xb[4], xab[4], xma[4], xmb[4], xamb[4], xmab[4];
      shift(g, x, a, 1, xa);
      shift(g, x, b, 1, xb);
      shift(g, xa, b, 1, xab);
      shift(g, x, a, -1, xma);
      shift(g, x, b, -1, xmb);
      shift(g, xa, b, -1, xamb);
      shift(g, xma, b, 1, xmab);
      const M3 L0 = ld_lt(g, lt, x, pl);
      if (mu == a) {
        Sf = add(Sf, staple_after(bare_link(g, U, xa, b), dag(bare_link(g, U, xb, a)), dag(bare_link(g, U, x, b)),
                                  ld_lt(g, lt, xa, pl), ld_lt(g, lt, xab, pl), ld_lt(g, lt, xb, pl), L0));
        Sb = add(Sb, staple_before(dag(bare_link(g, U, xmb, b)), bare_link(g, U, xmb, a), bare_link(g, U, xamb, b),
                                   ld_lt(g, lt, xmb, pl), ld_lt(g, lt, xamb, pl), ld_lt(g, lt, xa, pl), L0));
      } else {
        Sf = add(Sf, staple_after(dag(bare_link(g, U, xmab, a)), dag(bare_link(g, U, xma, b)), bare_link(g, U, xma, a),
                                  ld_lt(g, lt, xb, pl), ld_lt(g, lt, xmab, pl), ld_lt(g, lt, xma, pl), L0));
        Sb = add(Sb, staple_before(bare_link(g, U, x, a), bare_link(g, U, xa, b), dag(bare_link(g, U, xb, a)),
                                   ld_lt(g, lt, xa, pl), ld_lt(g, lt, xab, pl), ld_lt(g, lt, xb, pl), L0));
      }
    }
  }
  if (T.nt) {
    switch (mu) {
      case 0: hop_force_part<0>(g, x, p, i, T, Sf, Sb); break;
      case 1: hop_force_part<1>(g, x, p, i, T, Sf, Sb); break;
      case 2: hop_force_part<2>(g, x, p, i, T, Sf, Sb); break;
      default: hop_force_part<3>(g, x, p, i, T, Sf, Sb); break;
    }
  }
  // M = Ul Sf - Sb Ul^dag
  const M3 Ul = bare_link(g, U, x, mu), m1 = mul(Ul, Sf), m2 = mul_nd(Sb, Ul);
  M3 Mt;
#pragma unroll
  for (int k = 0; k < 9; ++k) Mt.a[k] = m1.a[k] - m2.a[k];
  // f^a = Re tr(i lambda^a M / 2) = -Im tr(lambda^a M) / 2
  auto e = [&](int r, int c) { return Mt.a[r * 3 + c]; };
  const zd tr[8] = {e(1, 0) + e(0, 1),
                    ti(e(0, 1)) + tmi(e(1, 0)),
                    e(0, 0) - e(1, 1),
                    e(2, 0) + e(0, 2),
                    ti(e(0, 2)) + tmi(e(2, 0)),
                    e(2, 1) + e(1, 2),
                    ti(e(1, 2)) + tmi(e(2, 1)),
                    (1.0 / sqrt(3.0)) * (e(0, 0) + e(1, 1) - 2.0 * e(2, 2))};
  double* o = force + ((int64_t)lex_of(g, x) * 4 + mu) * 8;
#pragma unroll
  for (int q = 0; q < 8; ++q) o[q] = -0.5 * tr[q].im;
}

hipError_t launch_force_odd(const Geo& g, const DevOp<double>& op, int nt, double2* X, double2* Y, hipStream_t st) {
  hipLaunchKernelGGL(k_force_odd, dim3((g.Vh + 127) / 128), dim3(128), 0, st, g, op.U, op.Ainv, nt, X, Y);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  const int64_t n = (int64_t)nt * g.Vh * 6;
  hipLaunchKernelGGL(k_force_g5, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (int64_t)g.Vh, nt, X);
  return hipGetLastError();
}

hipError_t launch_force_src(const Geo& g, const DevOp<double>& op, const double2* psi, const double2* xi,
                            const double2* phi2, double dm, double2* src, hipStream_t st) {
  hipLaunchKernelGGL(k_force_src, dim3((g.Vh + 127) / 128), dim3(128), 0, st, g, op.Ainv, psi, xi, phi2, dm, src);
  return hipGetLastError();
}

hipError_t launch_force(const Geo& g, const DevOp<double>& op, const double2* U, double det_w, double csw,
                        const FrcTerms& T, double* lt, double* force, hipStream_t st) {
  const bool clov = det_w != 0.0 || T.nt > 0;
  if (clov) {
    hipLaunchKernelGGL(k_force_lt, dim3((g.V + 127) / 128), dim3(128), 0, st, g, op.Ainv, det_w, csw, T, lt);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  }
  const int64_t n = (int64_t)4 * g.V;
  hipLaunchKernelGGL(k_force_link, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, g, U, lt, clov ? 1 : 0, T,
                     force);
  return hipGetLastError();
}

}  // namespace qdd
