// Vector kernels of the outer flexible GCR (FP64 accumulation).  A "vector" is a
// contiguous array of n complex numbers (one right-hand side of an internal
// field); several right-hand sides sit at a fixed stride.  Reductions are
// two-pass and deterministic: per-block partial sums in a fixed order, then one
// wavefront per result sums the partials in a fixed order (no floating-point
// atomics), so repeated runs give bitwise identical results.
#include "qdd_kernels.h"
#include "qdd_blas.h"

namespace qdd {

template <class E>
__device__ inline cx<double> ldz(const E* p);
template <>
__device__ inline cx<double> ldz<double2>(const double2* p) {
  double2 v = *p;
  return {v.x, v.y};
}
template <>
__device__ inline cx<double> ldz<float2>(const float2* p) {
  float2 v = *p;
  return {(double)v.x, (double)v.y};
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// the workgroup's sums of the per-lane values acc[l] (l < m): wavefront sums,
// then the wavefronts in order, into part[(r*m + l) * nb + bid]
template <int MM>
__device__ __forceinline__ void block_partials(const cx<double> acc[MM], int m, double (*sh)[4][2], double2* part,
                                               int r, int bid, int nb) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int l = 0; l < MM; ++l) {
    if (l < m) {
      double re = wave_sum(acc[l].re), im = wave_sum(acc[l].im);
      if (lane == 0) {
        sh[l][w][0] = re;
        sh[l][w][1] = im;
      }
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < m) {
    int l = threadIdx.x;
    double re = 0, im = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      re += sh[l][k][0];
      im += sh[l][k][1];
    }
    part[((int64_t)r * m + l) * nb + bid] = make_double2(re, im);
  }
}

// partial sums: part[(r*m + l) * nb + b] = sum over block b of conj(x_l[r]) y[r]
template <class E, int MM>
__device__ __forceinline__ void dots_body(const E* x, int64_t lstride, int64_t xrs, int m, const double2* y,
                                          int64_t yrs, int64_t n, double2* part, int r, int bid, int nb) {
  __shared__ double sh[MM][4][2];
  const E* xr = x + r * xrs;
  const double2* yr = y + r * yrs;
  cx<double> acc[MM];
#pragma unroll
  for (int l = 0; l < MM; ++l) acc[l] = {0.0, 0.0};
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n; i += (int64_t)nb * blockDim.x) {
    double2 yv = yr[i];
    cx<double> yy{yv.x, yv.y};
#pragma unroll
    for (int l = 0; l < MM; ++l)
      if (l < m) acc[l] = fmac_c(ldz(xr + l * lstride + i), yy, acc[l]);
  }
  block_partials<MM>(acc, m, sh, part, r, bid, nb);
}
template <class E, int MM>
__global__ void __launch_bounds__(256) k_dots(const E* x, int64_t lstride, int64_t xrs, int m, const double2* y,
                                              int64_t yrs, int64_t n, double2* part) {
  dots_body<E, MM>(x, lstride, xrs, m, y, yrs, n, part, blockIdx.y, blockIdx.x, gridDim.x);
}
template <class E, int MM>
__global__ void __launch_bounds__(256) k_dots_grp(Grp<DotsArgs<E>> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  const DotsArgs<E>& a = G.a[s];
  if ((int)blockIdx.y >= a.nrhs) return;
  dots_body<E, MM>(a.x, a.lstride, a.xrs, a.m, a.y, a.yrs, a.n, a.part, blockIdx.y, blockIdx.x - G.start[s],
                   G.start[s + 1] - G.start[s]);
}

// one wavefront per result: lane j sums the partials j, j+64, ... in order, then a
// fixed shuffle tree adds the 64 lane sums (the same order on every run)
__device__ __forceinline__ void dots_final_body(const double2* part, int nb, int total, double2* out, int bid) {
  int t = bid * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t >= total) return;
  const double2* p = part + (int64_t)t * nb;
  double re = 0, im = 0;
  for (int b = lane; b < nb; b += 64) {
    double2 v = p[b];
    re += v.x;
    im += v.y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) out[t] = make_double2(re, im);
}
__global__ void __launch_bounds__(256) k_dots_final(const double2* part, int nb, int total, double2* out) {
  dots_final_body(part, nb, total, out, blockIdx.x);
}
template <class E>
__global__ void __launch_bounds__(256) k_dots_final_grp(Grp<DotsArgs<E>> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  const DotsArgs<E>& a = G.a[s];
  dots_final_body(a.part, a.nb, a.nrhs * a.m, a.out, blockIdx.x - G.start[s]);
}

static int dots_blocks(int64_t n) { return (int)std::min<int64_t>(kDotBlocks, (n + 255) / 256); }

// One sweep that updates y[r] and reduces over the updated values, in the
// element order and partial-sum blocking of k_dots (so that the sums equal those
// of the separate update and reduction bit for bit, and y is read once):
//   UPD 0: y <- y - sum_{l<m} c_l x_l   (as k_axpy_multi with sgn -1; not where
//          active[r] == 0), then MODE 0: part of conj(x_l) y for l < m (the next
//          Gram-Schmidt pass), MODE 1: part of conj(y) y (a norm);
//   UPD 1: y <- a[r] y (as k_axpby with b = 0), then part of conj(y) w[r].
template <int MM, int UPD, int MODE>
__device__ __forceinline__ void upd_dots_body(double2* y, int64_t yrs, const double2* x, int64_t lstride,
                                              int64_t xrs, int m, const double2* coef, int ldc, const int* active,
                                              const double* a, const double2* w, int64_t wrs, int64_t n,
                                              double2* part, int r, int bid, int nb) {
  __shared__ double sh[MM][4][2];
  __shared__ cx<double> c[MM];
  const bool upd = !(active && !active[r]);
  if constexpr (UPD == 0) {
    if ((int)threadIdx.x < m) {
      double2 v = coef[r * ldc + threadIdx.x];
      c[threadIdx.x] = {-1.0 * v.x, -1.0 * v.y};
    }
    __syncthreads();
  }
  double2* yr = y + r * yrs;
  const double2* xr = x + r * xrs;
  const double2* wr = w ? w + r * wrs : nullptr;
  const double av = (UPD == 1 && a) ? a[r] : 1.0;
  constexpr int NS = MODE == 0 ? MM : 1;
  const int ns = MODE == 0 ? m : 1;
  cx<double> acc[NS];
#pragma unroll
  for (int l = 0; l < NS; ++l) acc[l] = {0.0, 0.0};
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n; i += (int64_t)nb * blockDim.x) {
    const double2 yv = yr[i];
    cx<double> yy{yv.x, yv.y};
    if constexpr (UPD == 0) {
      cx<double> xv[MM];
#pragma unroll
      for (int l = 0; l < MM; ++l)
        if (l < m) xv[l] = ldz(xr + l * lstride + i);
      if (upd) {
#pragma unroll
        for (int l = 0; l < MM; ++l)
          if (l < m) yy = fma_c(c[l], xv[l], yy);
        yr[i] = make_double2(yy.re, yy.im);
      }
      if constexpr (MODE == 0) {
#pragma unroll
        for (int l = 0; l < MM; ++l)
          if (l < m) acc[l] = fmac_c(xv[l], yy, acc[l]);
      } else {
        acc[0] = fmac_c(yy, yy, acc[0]);
      }
    } else {
      yy = {av * yv.x + 0.0 * yv.x, av * yv.y + 0.0 * yv.y};
      yr[i] = make_double2(yy.re, yy.im);
      const double2 wv = wr[i];
      acc[0] = fmac_c(yy, cx<double>{wv.x, wv.y}, acc[0]);
    }
  }
  block_partials<NS>(acc, ns, sh, part, r, bid, nb);
}
template <int MM, int UPD, int MODE>
__global__ void __launch_bounds__(256) k_upd_dots(double2* y, int64_t yrs, const double2* x, int64_t lstride,
                                                  int64_t xrs, int m, const double2* coef, int ldc,
                                                  const int* active, const double* a, const double2* w, int64_t wrs,
                                                  int64_t n, double2* part) {
  upd_dots_body<MM, UPD, MODE>(y, yrs, x, lstride, xrs, m, coef, ldc, active, a, w, wrs, n, part, blockIdx.y,
                               blockIdx.x, gridDim.x);
}
template <int MM, int UPD, int MODE>
__global__ void __launch_bounds__(256) k_upd_dots_grp(Grp<UpdArgs> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  const UpdArgs& q = G.a[s];
  if ((int)blockIdx.y >= q.nrhs) return;
  upd_dots_body<MM, UPD, MODE>(q.y, q.yrs, q.x, q.lstride, q.xrs, q.m, q.coef, q.ldc, q.active, q.a, q.w, q.wrs, q.n,
                               q.part, blockIdx.y, blockIdx.x - G.start[s], G.start[s + 1] - G.start[s]);
}
__global__ void __launch_bounds__(256) k_upd_final_grp(Grp<UpdArgs> G, int mode) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  const UpdArgs& q = G.a[s];
  dots_final_body(q.part, q.nb, q.nrhs * (mode == 0 ? q.m : 1), q.out, blockIdx.x - G.start[s]);
}

// the same sweeps over several systems, one launch each (UpdArgs per system)
template <int UPD, int MODE>
static hipError_t launch_upd_dots_grp_m(const UpdArgs* a, int ns, hipStream_t st) {
  if (ns < 1 || ns > kGrpMax) return hipErrorInvalidValue;
  Grp<UpdArgs> G = grp_new<UpdArgs>(), F = grp_new<UpdArgs>();
  int mm = 1;
  for (int s = 0; s < ns; ++s) {
    if (a[s].m < 1) return hipErrorInvalidValue;
    UpdArgs b = a[s];
    b.nb = dots_blocks(b.n);
    grp_add(G, b, b.nb, b.nrhs);
    grp_add(F, b, (b.nrhs * (MODE == 0 ? b.m : 1) + 3) / 4);
    mm = std::max(mm, b.m);
  }
  const dim3 grid(G.start[ns], G.ny), blk(256);
#define UG(MM) hipLaunchKernelGGL((k_upd_dots_grp<MM, UPD, MODE>), grid, blk, 0, st, G)
  if (UPD == 1 || mm <= 1) UG(1);
  else if (mm <= 4) UG(4);
  else if (mm <= 8) UG(8);
  else if (mm <= 16) UG(16);
  else if (mm <= 32) UG(32);
  else return hipErrorInvalidValue;
#undef UG
  hipLaunchKernelGGL(k_upd_final_grp, dim3(F.start[ns]), blk, 0, st, F, MODE);
  return hipGetLastError();
}
hipError_t launch_sub_dots_grp(const UpdArgs* a, int ns, int mode, hipStream_t st) {
  return mode == 0 ? launch_upd_dots_grp_m<0, 0>(a, ns, st) : launch_upd_dots_grp_m<0, 1>(a, ns, st);
}
hipError_t launch_scale_dot_grp(const UpdArgs* a, int ns, hipStream_t st) { return launch_upd_dots_grp_m<1, 1>(a, ns, st); }

template <int UPD, int MODE>
static hipError_t launch_upd_dots_m(double2* y, int64_t yrs, const double2* x, int64_t lstride, int64_t xrs, int m,
                                    const double2* coef, int ldc, const int* active, const double* a,
                                    const double2* w, int64_t wrs, int64_t n, int nrhs, double2* part, double2* out,
                                    hipStream_t st) {
  const int nb = dots_blocks(n);
  const dim3 grid(nb, nrhs), blk(256);
#define UD(MM) hipLaunchKernelGGL((k_upd_dots<MM, UPD, MODE>), grid, blk, 0, st, y, yrs, x, lstride, xrs, m, coef, ldc, \
                                  active, a, w, wrs, n, part)
  if (UPD == 1 || m <= 1) UD(1);
  else if (m <= 4) UD(4);
  else if (m <= 8) UD(8);
  else if (m <= 16) UD(16);
  else if (m <= 32) UD(32);
  else return hipErrorInvalidValue;
#undef UD
  const int total = nrhs * (MODE == 0 ? m : 1);
  hipLaunchKernelGGL(k_dots_final, dim3((total + 3) / 4), blk, 0, st, part, nb, total, out);
  return hipGetLastError();
}

hipError_t launch_sub_dots(double2* y, int64_t yrs, const double2* x, int64_t lstride, int64_t xrs, int m,
                           const double2* coef, int ldc, const int* active, int mode, int64_t n, int nrhs,
                           double2* part, double2* out, hipStream_t st) {
  if (m < 1) return hipErrorInvalidValue;
  return mode == 0 ? launch_upd_dots_m<0, 0>(y, yrs, x, lstride, xrs, m, coef, ldc, active, nullptr, nullptr, 0, n,
                                             nrhs, part, out, st)
                   : launch_upd_dots_m<0, 1>(y, yrs, x, lstride, xrs, m, coef, ldc, active, nullptr, nullptr, 0, n,
                                             nrhs, part, out, st);
}
hipError_t launch_scale_dot(double2* y, int64_t yrs, const double* a, const double2* w, int64_t wrs, int64_t n,
                            int nrhs, double2* part, double2* out, hipStream_t st) {
  return launch_upd_dots_m<1, 1>(y, yrs, nullptr, 0, 0, 1, nullptr, 1, nullptr, a, w, wrs, n, nrhs, part, out, st);
}

template <class E>
hipError_t launch_dots(const E* x, int64_t lstride, int64_t xrs, int m, const double2* y, int64_t yrs, int64_t n,
                       int nrhs, double2* part, double2* out, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  int nb = dots_blocks(n);
  dim3 grid(nb, nrhs);
  if (m <= 1) hipLaunchKernelGGL((k_dots<E, 1>), grid, dim3(256), 0, st, x, lstride, xrs, m, y, yrs, n, part);
  else if (m <= 4) hipLaunchKernelGGL((k_dots<E, 4>), grid, dim3(256), 0, st, x, lstride, xrs, m, y, yrs, n, part);
  else if (m <= 8) hipLaunchKernelGGL((k_dots<E, 8>), grid, dim3(256), 0, st, x, lstride, xrs, m, y, yrs, n, part);
  else if (m <= 16) hipLaunchKernelGGL((k_dots<E, 16>), grid, dim3(256), 0, st, x, lstride, xrs, m, y, yrs, n, part);
  else if (m <= 32) hipLaunchKernelGGL((k_dots<E, 32>), grid, dim3(256), 0, st, x, lstride, xrs, m, y, yrs, n, part);
  else return hipErrorInvalidValue;
  int total = nrhs * m;
  hipLaunchKernelGGL(k_dots_final, dim3((total + 3) / 4), dim3(256), 0, st, part, nb, total, out);
  return hipGetLastError();
}

template <class E>
hipError_t launch_dots_grp(const DotsArgs<E>* a, int ns, hipStream_t st) {
  if (ns < 1 || ns > kGrpMax) return hipErrorInvalidValue;
  Grp<DotsArgs<E>> G = grp_new<DotsArgs<E>>(), F = grp_new<DotsArgs<E>>();
  int mm = 0;
  for (int s = 0; s < ns; ++s) {
    if (a[s].m < 1) return hipErrorInvalidValue;
    DotsArgs<E> b = a[s];
    b.nb = dots_blocks(b.n);
    grp_add(G, b, b.nb, b.nrhs);
    grp_add(F, b, (b.nrhs * b.m + 3) / 4);
    mm = std::max(mm, b.m);
  }
  const dim3 grid(G.start[ns], G.ny), blk(256);
  if (mm <= 1) hipLaunchKernelGGL((k_dots_grp<E, 1>), grid, blk, 0, st, G);
  else if (mm <= 4) hipLaunchKernelGGL((k_dots_grp<E, 4>), grid, blk, 0, st, G);
  else if (mm <= 8) hipLaunchKernelGGL((k_dots_grp<E, 8>), grid, blk, 0, st, G);
  else if (mm <= 16) hipLaunchKernelGGL((k_dots_grp<E, 16>), grid, blk, 0, st, G);
  else if (mm <= 32) hipLaunchKernelGGL((k_dots_grp<E, 32>), grid, blk, 0, st, G);
  else return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dots_final_grp<E>, dim3(F.start[ns]), blk, 0, st, F);
  return hipGetLastError();
}

// y[r] += sgn * sum_l coef[r*ldc + l] * x_l[r]    (active[r] == 0 skips rhs r)
template <class E, int MM>
__device__ __forceinline__ void axpy_multi_body(double2* y, int64_t yrs, const E* x, int64_t lstride, int64_t xrs,
                                                int m, const double2* coef, int ldc, double sgn, int64_t n,
                                                const int* active, int r, int bid, int nb) {
  if (active && !active[r]) return;
  __shared__ cx<double> c[MM];
  if ((int)threadIdx.x < m) {
    double2 v = coef[r * ldc + threadIdx.x];
    c[threadIdx.x] = {sgn * v.x, sgn * v.y};
  }
  __syncthreads();
  double2* yr = y + r * yrs;
  const E* xr = x + r * xrs;
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n; i += (int64_t)nb * blockDim.x) {
    double2 yv = yr[i];
    cx<double> acc{yv.x, yv.y};
#pragma unroll
    for (int l = 0; l < MM; ++l)
      if (l < m) acc = fma_c(c[l], ldz(xr + l * lstride + i), acc);
    yr[i] = make_double2(acc.re, acc.im);
  }
}
template <class E, int MM>
__global__ void __launch_bounds__(256) k_axpy_multi(double2* y, int64_t yrs, const E* x, int64_t lstride,
                                                    int64_t xrs, int m, const double2* coef, int ldc, double sgn,
                                                    int64_t n, const int* active) {
  axpy_multi_body<E, MM>(y, yrs, x, lstride, xrs, m, coef, ldc, sgn, n, active, blockIdx.y, blockIdx.x, gridDim.x);
}
template <class E, int MM>
__global__ void __launch_bounds__(256) k_axpy_multi_grp(Grp<AxpyArgs<E>> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  const AxpyArgs<E>& a = G.a[s];
  if ((int)blockIdx.y >= a.nrhs) return;
  axpy_multi_body<E, MM>(a.y, a.yrs, a.x, a.lstride, a.xrs, a.m, a.coef, a.ldc, a.sgn, a.n, a.active, blockIdx.y,
                         blockIdx.x - G.start[s], G.start[s + 1] - G.start[s]);
}
static int vec_blocks(int64_t n) { return (int)std::min<int64_t>(2048, (n + 255) / 256); }

template <class E>
hipError_t launch_axpy_multi(double2* y, int64_t yrs, const E* x, int64_t lstride, int64_t xrs, int m,
                             const double2* coef, int ldc, double sgn, int64_t n, int nrhs, const int* active,
                             hipStream_t st) {
  if (m <= 0) return hipSuccess;
  int nb = vec_blocks(n);
  dim3 grid(nb, nrhs);
  if (m <= 1) hipLaunchKernelGGL((k_axpy_multi<E, 1>), grid, dim3(256), 0, st, y, yrs, x, lstride, xrs, m, coef, ldc, sgn, n, active);
  else if (m <= 4) hipLaunchKernelGGL((k_axpy_multi<E, 4>), grid, dim3(256), 0, st, y, yrs, x, lstride, xrs, m, coef, ldc, sgn, n, active);
  else if (m <= 8) hipLaunchKernelGGL((k_axpy_multi<E, 8>), grid, dim3(256), 0, st, y, yrs, x, lstride, xrs, m, coef, ldc, sgn, n, active);
  else if (m <= 16) hipLaunchKernelGGL((k_axpy_multi<E, 16>), grid, dim3(256), 0, st, y, yrs, x, lstride, xrs, m, coef, ldc, sgn, n, active);
  else if (m <= 32) hipLaunchKernelGGL((k_axpy_multi<E, 32>), grid, dim3(256), 0, st, y, yrs, x, lstride, xrs, m, coef, ldc, sgn, n, active);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// systems with m = 0 take no part
template <class E>
hipError_t launch_axpy_multi_grp(const AxpyArgs<E>* a, int ns, hipStream_t st) {
  if (ns < 1 || ns > kGrpMax) return hipErrorInvalidValue;
  Grp<AxpyArgs<E>> G = grp_new<AxpyArgs<E>>();
  int mm = 0;
  for (int s = 0; s < ns; ++s) {
    if (a[s].m <= 0) continue;
    grp_add(G, a[s], vec_blocks(a[s].n), a[s].nrhs);
    mm = std::max(mm, a[s].m);
  }
  if (G.ns == 0) return hipSuccess;
  const dim3 grid(G.start[G.ns], G.ny), blk(256);
  if (mm <= 1) hipLaunchKernelGGL((k_axpy_multi_grp<E, 1>), grid, blk, 0, st, G);
  else if (mm <= 4) hipLaunchKernelGGL((k_axpy_multi_grp<E, 4>), grid, blk, 0, st, G);
  else if (mm <= 8) hipLaunchKernelGGL((k_axpy_multi_grp<E, 8>), grid, blk, 0, st, G);
  else if (mm <= 16) hipLaunchKernelGGL((k_axpy_multi_grp<E, 16>), grid, blk, 0, st, G);
  else if (mm <= 32) hipLaunchKernelGGL((k_axpy_multi_grp<E, 32>), grid, blk, 0, st, G);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// y[r] = a * x[r] + b * y[r] with per-rhs real scalars (device arrays, may be null = 1/0)
__device__ __forceinline__ void axpby_body(double2* y, int64_t yrs, const double2* x, int64_t xrs, const double* a,
                                           const double* b, int64_t n, const int* active, int r, int bid, int nb) {
  if (active && !active[r]) return;
  double av = a ? a[r] : 1.0, bv = b ? b[r] : 0.0;
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n; i += (int64_t)nb * blockDim.x) {
    double2 xv = x[r * xrs + i], yv = y[r * yrs + i];
    y[r * yrs + i] = make_double2(av * xv.x + bv * yv.x, av * xv.y + bv * yv.y);
  }
}
__global__ void k_axpby(double2* y, int64_t yrs, const double2* x, int64_t xrs, const double* a, const double* b,
                        int64_t n, const int* active) {
  axpby_body(y, yrs, x, xrs, a, b, n, active, blockIdx.y, blockIdx.x, gridDim.x);
}

hipError_t launch_axpby(double2* y, int64_t yrs, const double2* x, int64_t xrs, const double* a, const double* b,
                        int64_t n, int nrhs, const int* active, hipStream_t st) {
  int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_axpby, dim3(nb, nrhs), dim3(256), 0, st, y, yrs, x, xrs, a, b, n, active);
  return hipGetLastError();
}

// z[r] = x[r] - y[r]
__device__ __forceinline__ void sub_body(double2* z, const double2* x, const double2* y, int64_t rs, int64_t n, int r,
                                         int bid, int nb) {
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n; i += (int64_t)nb * blockDim.x) {
    double2 a = x[r * rs + i], b = y[r * rs + i];
    z[r * rs + i] = make_double2(a.x - b.x, a.y - b.y);
  }
}
__global__ void k_sub(double2* z, const double2* x, const double2* y, int64_t rs, int64_t n) {
  sub_body(z, x, y, rs, n, blockIdx.y, blockIdx.x, gridDim.x);
}
__global__ void k_sub_grp(Grp<SubArgs> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  const SubArgs& a = G.a[s];
  if ((int)blockIdx.y >= a.nrhs) return;
  sub_body(a.z, a.x, a.y, a.rs, a.n, blockIdx.y, blockIdx.x - G.start[s], G.start[s + 1] - G.start[s]);
}
hipError_t launch_sub(double2* z, const double2* x, const double2* y, int64_t rs, int64_t n, int nrhs,
                      hipStream_t st) {
  int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_sub, dim3(nb, nrhs), dim3(256), 0, st, z, x, y, rs, n);
  return hipGetLastError();
}
hipError_t launch_sub_grp(const SubArgs* a, int ns, hipStream_t st) {
  if (ns < 1 || ns > kGrpMax) return hipErrorInvalidValue;
  Grp<SubArgs> G = grp_new<SubArgs>();
  for (int s = 0; s < ns; ++s) grp_add(G, a[s], vec_blocks(a[s].n), a[s].nrhs);
  hipLaunchKernelGGL(k_sub_grp, dim3(G.start[ns], G.ny), dim3(256), 0, st, G);
  return hipGetLastError();
}

// Gram-Schmidt bookkeeping on device (one thread per rhs):
//  norm step: b = sqrt(|chi|^2), inv = 1/b (written as double2 for scaling)
__global__ void k_norm_finish(const double2* nrm2, double* b, double* binv, int nrhs) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double v = sqrt(fmax(nrm2[r].x, 0.0));
  b[r] = v;
  binv[r] = v > 0 ? 1.0 / v : 0.0;
}
hipError_t launch_norm_finish(const double2* nrm2, double* b, double* binv, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_norm_finish, dim3((nrhs + 63) / 64), dim3(64), 0, st, nrm2, b, binv, nrhs);
  return hipGetLastError();
}

// acc[r*lda + l] += src[r*m + l]   (accumulate Gram-Schmidt coefficients)
__global__ void k_acc_coef(double2* acc, int lda, const double2* src, int m, int nrhs) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * nrhs) return;
  int r = t / m, l = t % m;
  double2 a = acc[r * lda + l], s = src[t];
  acc[r * lda + l] = make_double2(a.x + s.x, a.y + s.y);
}
hipError_t launch_acc_coef(double2* acc, int lda, const double2* src, int m, int nrhs, hipStream_t st) {
  int t = m * nrhs;
  if (t == 0) return hipSuccess;
  hipLaunchKernelGGL(k_acc_coef, dim3((t + 63) / 64), dim3(64), 0, st, acc, lda, src, m, nrhs);
  return hipGetLastError();
}

// the per-rhs Gram-Schmidt bookkeeping of several systems, one workgroup each:
// op 0 zero acc[0 .. nrhs*lda), op 1 the norm step, op 2 the coefficient sum
__global__ void __launch_bounds__(256) k_coef_grp(Grp<CoefArgs> G, int op) {
  const CoefArgs& a = G.a[blockIdx.x];
  if (op == 0) {
    for (int t = threadIdx.x; t < a.nrhs * a.lda; t += blockDim.x) a.acc[t] = make_double2(0.0, 0.0);
  } else if (op == 1) {
    for (int r = threadIdx.x; r < a.nrhs; r += blockDim.x) {
      double v = sqrt(fmax(a.nrm2[r].x, 0.0));
      a.b[r] = v;
      a.binv[r] = v > 0 ? 1.0 / v : 0.0;
    }
  } else {
    for (int t = threadIdx.x; t < a.m * a.nrhs; t += blockDim.x) {
      int r = t / a.m, l = t % a.m;
      double2 x = a.acc[r * a.lda + l], y = a.src[t];
      a.acc[r * a.lda + l] = make_double2(x.x + y.x, x.y + y.y);
    }
  }
}
hipError_t launch_coef_grp(const CoefArgs* a, int ns, int op, hipStream_t st) {
  if (ns < 1 || ns > kGrpMax || op < 0 || op > 2) return hipErrorInvalidValue;
  Grp<CoefArgs> G = grp_new<CoefArgs>();
  for (int s = 0; s < ns; ++s) grp_add(G, a[s], 1);
  hipLaunchKernelGGL(k_coef_grp, dim3(ns), dim3(256), 0, st, G, op);
  return hipGetLastError();
}

template hipError_t launch_dots<double2>(const double2*, int64_t, int64_t, int, const double2*, int64_t, int64_t, int,
                                         double2*, double2*, hipStream_t);
template hipError_t launch_dots<float2>(const float2*, int64_t, int64_t, int, const double2*, int64_t, int64_t, int,
                                        double2*, double2*, hipStream_t);
template hipError_t launch_axpy_multi<double2>(double2*, int64_t, const double2*, int64_t, int64_t, int,
                                               const double2*, int, double, int64_t, int, const int*, hipStream_t);
template hipError_t launch_axpy_multi<float2>(double2*, int64_t, const float2*, int64_t, int64_t, int,
                                              const double2*, int, double, int64_t, int, const int*, hipStream_t);
template hipError_t launch_dots_grp<double2>(const DotsArgs<double2>*, int, hipStream_t);
template hipError_t launch_axpy_multi_grp<double2>(const AxpyArgs<double2>*, int, hipStream_t);
template hipError_t launch_axpy_multi_grp<float2>(const AxpyArgs<float2>*, int, hipStream_t);

}  // namespace qdd
