// Mass-preconditioning pieces of Eqs. 2-5 on the stored FP64 operator:
//  * log det Q_ee and log det Q_oo (Eq. 2).  Q_ee = gamma5 A_e is site-diagonal
//    and gamma5 has determinant 1 on a site's 12 components, so each is the sum
//    over one parity of log det A(x) = log det A_+(x) + log det A_-(x), from the
//    Cholesky factor of each Hermitian positive-definite 6x6 block
//    (log det = sum_j log d_j over its pivots d_j = L_jj^2).
//  * W(dm) = Q_S + dm (Eq. 3).  With Q = gamma5 D the gamma5 factors of
//    Q_ee^{-1} Q_eo Q_oo^{-1} Q_oe cancel pairwise, so Q_S = A_e^{-1} Dhat: the
//    FP64 Schur-complement apply followed by the even-site inverse clover block
//    and the shift.
#include "qdd_kernels.h"

namespace qdd {

constexpr int kLogdetThreads = 256;
constexpr int kLogdetMaxBlocks = 512;  // workgroups per parity (partial sums)

// log det of a Hermitian 6x6 block stored in 18 slots (diagonal as 3 complex
// words, then the strict upper triangle row by row); NaN if a pivot is not
// positive
__device__ inline double herm6_logdet(const cx<double> a[18]) {
  cx<double> M[36];
  const double dg[6] = {a[0].re, a[0].im, a[1].re, a[1].im, a[2].re, a[2].im};
  int s = 3;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    M[r * 6 + r] = {dg[r], 0.0};
#pragma unroll
    for (int c = r + 1; c < 6; ++c) {
      M[r * 6 + c] = a[s];
      M[c * 6 + r] = conj(a[s]);
      ++s;
    }
  }
  cx<double> Lm[36];
  double ld = 0.0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double d = M[j * 6 + j].re;
#pragma unroll
    for (int k = 0; k < j; ++k) d -= Lm[j * 6 + k].re * Lm[j * 6 + k].re + Lm[j * 6 + k].im * Lm[j * 6 + k].im;
    ok = ok && d > 0.0 && isfinite(d);
    const double ljj = sqrt(d > 0.0 ? d : 1.0);
    ld += log(d > 0.0 ? d : 1.0);
    const double inv = 1.0 / ljj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      cx<double> t = M[i * 6 + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t = t - Lm[i * 6 + k] * conj(Lm[j * 6 + k]);
      Lm[i * 6 + j] = inv * t;
    }
  }
  return ok ? ld : __builtin_nan("");
}

// part[p * gridDim.x + b]: sum of log det A(x) over the sites of parity p =
// blockIdx.y taken by workgroup b (grid-stride), tree-summed in a fixed order
__global__ void __launch_bounds__(kLogdetThreads) k_clover_logdet(CloverV<double> A, int Vh, double* part) {
  __shared__ double red[kLogdetThreads];
  const int p = blockIdx.y;
  double sum = 0.0;
  for (int i = blockIdx.x * kLogdetThreads + threadIdx.x; i < Vh; i += gridDim.x * kLogdetThreads) {
    const double2* b = A.p + (int64_t)p * 36 * A.n + i;
#pragma unroll 1
    for (int blk = 0; blk < 2; ++blk) {
      cx<double> a[18];
#pragma unroll
      for (int k = 0; k < 18; ++k) {
        const double2 w = b[(int64_t)(blk * 18 + k) * A.n];
        a[k] = {w.x, w.y};
      }
      sum += herm6_logdet(a);
    }
  }
  red[threadIdx.x] = sum;
  __syncthreads();
#pragma unroll
  for (int w = kLogdetThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)p * gridDim.x + blockIdx.x] = red[0];
}

int clover_logdet_blocks(int64_t Vh) {
  return (int)std::min<int64_t>(kLogdetMaxBlocks, std::max<int64_t>(1, (Vh + kLogdetThreads - 1) / kLogdetThreads));
}

hipError_t launch_clover_logdet(const Geo& g, const CloverV<double>& A, double* part, hipStream_t st) {
  const int nb = clover_logdet_blocks(g.Vh);
  hipLaunchKernelGGL(k_clover_logdet, dim3(nb, 2), dim3(kLogdetThreads), 0, st, A, g.Vh, part);
  return hipGetLastError();
}

// out = A_e^{-1} out + dm in on even sites (out holds Dhat in): one lane per
// (site, rhs), the right-hand side fastest
__global__ void __launch_bounds__(256) k_apply_w_finish(FieldV<double> in, FieldV<double> out, CloverV<double> Ai,
                                                        int nrhs, double dm, int Vh) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)Vh * nrhs) return;
  const int r = (int)(t % nrhs), i = (int)(t / nrhs);
  cx<double> v[12], w[12], y[12];
  ld_spinor<double>(out, r, i, v);
  clover_apply<double>(Ai, 0, i, v, y);
  ld_spinor<double>(in, r, i, w);
#pragma unroll
  for (int k = 0; k < 12; ++k) y[k] = y[k] + dm * w[k];
  st_spinor<double>(out, r, i, y);
}

hipError_t launch_apply_w_finish(const Geo& g, const FieldV<double>& in, const FieldV<double>& out,
                                 const CloverV<double>& Ai, int nrhs, double dm, hipStream_t st) {
  const int64_t n = (int64_t)g.Vh * nrhs;
  hipLaunchKernelGGL(k_apply_w_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, Ai, nrhs, dm,
                     g.Vh);
  return hipGetLastError();
}

// even part of the source of Eq. 5: eta_e = A_e phi (phi a canonical even field,
// [rhs][site][12] complex, its site index that of the packed even sites); one
// lane per (site, rhs).  The odd part of eta is zeroed by the caller.
__global__ void __launch_bounds__(256) k_qs_source(const double2* phi, FieldV<double> eta, CloverV<double> A,
                                                   int nrhs, int Vh) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)Vh * nrhs) return;
  const int r = (int)(t / Vh), i = (int)(t % Vh);
  const double2* src = phi + t * 12;
  cx<double> v[12], y[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = {src[k].x, src[k].y};
  clover_apply<double>(A, 0, i, v, y);
  st_spinor<double>(eta, r, i, y);
}

hipError_t launch_qs_source(const Geo& g, const double* phi_c, const FieldV<double>& eta, const CloverV<double>& A,
                            int nrhs, hipStream_t st) {
  const int64_t n = (int64_t)g.Vh * nrhs;
  hipLaunchKernelGGL(k_qs_source, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const double2*)phi_c, eta, A,
                     nrhs, g.Vh);
  return hipGetLastError();
}

}  // namespace qdd
