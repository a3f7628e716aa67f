// Clover term of Eq. (1): A(x) = (4+m0) + c_sw sum_{mu,nu} (i/4) sigma_{mu nu} F_{mu nu}(x),
// with F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag)/8 and Q the sum of the four
// plaquette leaves at x.  In the chiral basis the 12x12 matrix splits into two
// Hermitian 6x6 blocks (spin pairs (0,1) and (2,3)):
//   A_+/- = (4+m0) + (i c_sw / 2) sum_k sigma_k (x) ( +/-F_{0k} - B_k ),
//   B_1 = F_23, B_2 = F_31, B_3 = F_12.
// Each block and its inverse (Cholesky, FP64) are stored as 18 slots.
#include "qdd_kernels.h"
#include "qdd_su3.h"

namespace qdd {

// F_{mu nu}(x) from the four leaves (same orientation, all starting at x)
__device__ M3 field_strength(const Geo& g, const double2* U, const int x[4], int mu, int nu) {
  int xpm[4], xpn[4], xmm[4], xmn[4], xmmpn[4], xmmmn[4], xmnpm[4];
  shift(g, x, mu, 1, xpm);
  shift(g, x, nu, 1, xpn);
  shift(g, x, mu, -1, xmm);
  shift(g, x, nu, -1, xmn);
  shift(g, xmm, nu, 1, xmmpn);
  shift(g, xmm, nu, -1, xmmmn);
  shift(g, xmn, mu, 1, xmnpm);
  M3 Umu_x = bare_link(g, U, x, mu), Unu_x = bare_link(g, U, x, nu);
  M3 Umu_xmm = bare_link(g, U, xmm, mu), Unu_xmn = bare_link(g, U, xmn, nu);
  // x -> x+mu -> x+mu+nu -> x+nu -> x
  M3 Q = mul_nd(mul_nd(mul(Umu_x, bare_link(g, U, xpm, nu)), bare_link(g, U, xpn, mu)), Unu_x);
  // x -> x+nu -> x+nu-mu -> x-mu -> x
  M3 l = mul(mul_nd(mul_nd(Unu_x, bare_link(g, U, xmmpn, mu)), bare_link(g, U, xmm, nu)), Umu_xmm);
#pragma unroll
  for (int k = 0; k < 9; ++k) Q.a[k] = Q.a[k] + l.a[k];
  // x -> x-mu -> x-mu-nu -> x-nu -> x
  l = mul_dn(Umu_xmm, mul(mul_dn(bare_link(g, U, xmmmn, nu), bare_link(g, U, xmmmn, mu)), Unu_xmn));
#pragma unroll
  for (int k = 0; k < 9; ++k) Q.a[k] = Q.a[k] + l.a[k];
  // x -> x-nu -> x-nu+mu -> x+mu -> x
  l = mul_nd(mul(mul_dn(Unu_xmn, bare_link(g, U, xmn, mu)), bare_link(g, U, xmnpm, nu)), Umu_x);
#pragma unroll
  for (int k = 0; k < 9; ++k) Q.a[k] = Q.a[k] + l.a[k];
  M3 F;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      zd a = Q.a[i * 3 + j], b = Q.a[j * 3 + i];
      F.a[i * 3 + j] = {(a.re - b.re) * 0.125, (a.im + b.im) * 0.125};
    }
  return F;
}

// M += coef * (i c/2) sigma_k (x) F, M a 6x6 with index 3*s + c (s = 0,1)
__device__ inline void add_sigma(zd M[36], int k, double coef, const M3& F) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      zd f = coef * ti(F.a[a * 3 + b]);  // coef * i * F
      if (k == 1) {         // sigma_1 = [[0,1],[1,0]]
        M[a * 6 + 3 + b] = M[a * 6 + 3 + b] + f;
        M[(3 + a) * 6 + b] = M[(3 + a) * 6 + b] + f;
      } else if (k == 2) {  // sigma_2 = [[0,-i],[i,0]]
        M[a * 6 + 3 + b] = M[a * 6 + 3 + b] + tmi(f);
        M[(3 + a) * 6 + b] = M[(3 + a) * 6 + b] + ti(f);
      } else {              // sigma_3 = diag(1,-1)
        M[a * 6 + b] = M[a * 6 + b] + f;
        M[(3 + a) * 6 + 3 + b] = M[(3 + a) * 6 + 3 + b] - f;
      }
    }
}

__device__ inline void store_herm6(const zd M[36], double2* base, int64_t stride) {
  base[0] = make_double2(M[0].re, M[7].re);
  base[stride] = make_double2(M[14].re, M[21].re);
  base[2 * stride] = make_double2(M[28].re, M[35].re);
  int s = 3;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r + 1; c < 6; ++c) {
      base[(int64_t)s * stride] = make_double2(M[r * 6 + c].re, M[r * 6 + c].im);
      ++s;
    }
}

// Hermitian positive-definite 6x6 inverse via Cholesky; returns false if a pivot
// is not positive (block singular or indefinite)
__device__ inline bool herm6_inverse(const zd M[36], zd Minv[36]) {
  zd Lm[36];
  double dinv[6];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double d = M[j * 6 + j].re;
#pragma unroll
    for (int k = 0; k < j; ++k) d -= Lm[j * 6 + k].re * Lm[j * 6 + k].re + Lm[j * 6 + k].im * Lm[j * 6 + k].im;
    ok = ok && (d > 1e-300) && isfinite(d);
    double ljj = sqrt(d > 0 ? d : 1.0);
    dinv[j] = 1.0 / ljj;
    Lm[j * 6 + j] = {ljj, 0.0};
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      zd s = M[i * 6 + j];
#pragma unroll
      for (int k = 0; k < j; ++k) s = s - Lm[i * 6 + k] * conj(Lm[j * 6 + k]);
      Lm[i * 6 + j] = dinv[j] * s;
    }
  }
  // Li = L^{-1} (lower triangular)
  zd Li[36];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = 0; j < 6; ++j) Li[i * 6 + j] = {0.0, 0.0};
    Li[i * 6 + i] = {dinv[i], 0.0};
#pragma unroll
    for (int j = 0; j < i; ++j) {
      zd s{0.0, 0.0};
#pragma unroll
      for (int k = j; k < i; ++k) s = fma_c(Lm[i * 6 + k], Li[k * 6 + j], s);
      Li[i * 6 + j] = (-dinv[i]) * s;
    }
  }
  // M^{-1} = Li^dag Li
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      zd s{0.0, 0.0};
      int k0 = i > j ? i : j;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (k >= k0) s = fmac_c(Li[k * 6 + i], Li[k * 6 + j], s);
      Minv[i * 6 + j] = s;
    }
  return ok;
}

// one thread per site (lex order)
__global__ void __launch_bounds__(128) k_clover(Geo g, const double2* U, double diag, double csw, double2* A,
                                                double2* Ai, int* bad) {
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= g.V) return;
  int x[4];
  x[3] = lex % g.L[3];
  int r = lex / g.L[3];
  x[2] = r % g.L[2];
  r /= g.L[2];
  x[1] = r % g.L[1];
  x[0] = r / g.L[1];
  int p = (x[0] + x[1] + x[2] + x[3]) & 1, i = lex >> 1;
  double h = 0.5 * csw;
  int nbad = 0;
#pragma unroll 1
  for (int blk = 0; blk < 2; ++blk) {
    double sg = blk == 0 ? 1.0 : -1.0;
    zd M[36];
#pragma unroll
    for (int k = 0; k < 36; ++k) M[k] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 6; ++k) M[k * 7] = {diag, 0.0};
    if (csw != 0.0) {
      // +/- F_0k
      for (int k = 1; k <= 3; ++k) add_sigma(M, k, sg * h, field_strength(g, U, x, 0, k));
      // - B_k : B_1 = F_23, B_2 = F_31 = -F_13, B_3 = F_12
      add_sigma(M, 1, -h, field_strength(g, U, x, 2, 3));
      add_sigma(M, 2, h, field_strength(g, U, x, 1, 3));
      add_sigma(M, 3, -h, field_strength(g, U, x, 1, 2));
    }
    int64_t n = g.Vh;
    store_herm6(M, A + ((int64_t)p * 36 + blk * 18) * n + i, n);
    zd Mi[36];
    if (!herm6_inverse(M, Mi)) ++nbad;
    store_herm6(Mi, Ai + ((int64_t)p * 36 + blk * 18) * n + i, n);
  }
  if (nbad) atomicAdd(bad, nbad);
}

hipError_t launch_clover(const Geo& g, const double2* U, double diag, double csw, double2* A, double2* Ai, int* bad,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_clover, dim3((g.V + 127) / 128), dim3(128), 0, st, g, U, diag, csw, A, Ai, bad);
  return hipGetLastError();
}

}  // namespace qdd
