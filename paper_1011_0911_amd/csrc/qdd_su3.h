// FP64 SU(3) helpers shared by the clover construction and its derivative:
// 3x3 complex matrices, products with adjoints, the bare gauge link at
// lattice coordinates, and coordinate shifts.
#pragma once
#include "qdd_internal.h"

namespace qdd {

typedef cx<double> zd;

struct M3 {
  zd a[9];
};

__device__ inline M3 mul(const M3& x, const M3& y) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      zd s{0, 0};
#pragma unroll
      for (int k = 0; k < 3; ++k) s = fma_c(x.a[i * 3 + k], y.a[k * 3 + j], s);
      r.a[i * 3 + j] = s;
    }
  return r;
}
// x y^dag
__device__ inline M3 mul_nd(const M3& x, const M3& y) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      zd s{0, 0};
#pragma unroll
      for (int k = 0; k < 3; ++k) s = s + x.a[i * 3 + k] * conj(y.a[j * 3 + k]);
      r.a[i * 3 + j] = s;
    }
  return r;
}
// x^dag y
__device__ inline M3 mul_dn(const M3& x, const M3& y) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      zd s{0, 0};
#pragma unroll
      for (int k = 0; k < 3; ++k) s = fmac_c(x.a[k * 3 + i], y.a[k * 3 + j], s);
      r.a[i * 3 + j] = s;
    }
  return r;
}

// bare link U_mu(y) (boundary sign removed again) at coordinates y
__device__ inline M3 bare_link(const Geo& g, const double2* U, const int y[4], int mu) {
  int lex = lex_of(g, y);
  int p = (y[0] + y[1] + y[2] + y[3]) & 1;
  double s = (mu == 0 && y[0] == g.L[0] - 1) ? (double)g.bc : 1.0;
  const double2* b = U + (int64_t)(p * 4 + mu) * 9 * g.Vh + (lex >> 1);
  M3 m;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 v = b[(int64_t)k * g.Vh];
    m.a[k] = {s * v.x, s * v.y};
  }
  return m;
}

__device__ inline void shift(const Geo& g, const int x[4], int mu, int d, int y[4]) {
  for (int k = 0; k < 4; ++k) y[k] = x[k];
  y[mu] = (y[mu] + d + g.L[mu]) % g.L[mu];
}

}  // namespace qdd
