// Launchers of the local-deflation kernels (qdd_dfl.hip).
#pragma once
#include "qdd_kernels.h"
#include <type_traits>

namespace qdd {

struct DflGeo {
  int bs[4], nb[4];  // deflation block extents, blocks per direction
  int nblk;
};

__device__ __host__ inline cx<double> cvt_any(double2 v) { return {v.x, v.y}; }
__device__ __host__ inline cx<double> cvt_any(float2 v) { return {(double)v.x, (double)v.y}; }
template <class E>
__device__ inline E to_elem(cx<double> v);
template <>
__device__ inline double2 to_elem<double2>(cx<double> v) { return make_double2(v.re, v.im); }
template <>
__device__ inline float2 to_elem<float2>(cx<double> v) { return make_float2((float)v.re, (float)v.im); }

// block orthonormalisation of the Ns fields of W; work: 2 nblk Ns^2 complex
// (CholeskyQR on the matrix cores; Gram-Schmidt kernel where it does not apply)
hipError_t launch_block_orth(const Geo& g, const DflGeo& d, double2* W, int64_t vs, int Ns, double2* work,
                             hipStream_t st);
hipError_t launch_dfl_hops(const Geo& g, const DflGeo& d, const DevOp<double>& op, const double2* W, int64_t vs,
                           double2* F, int Ns, int mode, hipStream_t st);
// out[b*bso + kx*ldo + ky*kys] = sum over block b of conj(X_kx) Y_ky.  face =
// 1 + 2 mu + dir when Y vanishes off that face of every block (only the face's
// sites are then visited), else 0.
template <class EX, class EY>
hipError_t launch_block_dots(const Geo& g, const DflGeo& d, const EX* X, int64_t xvs, int nx, const EY* Y,
                             int64_t yvs, int ny, double2* out, int64_t bso, int64_t ldo, int64_t kys,
                             hipStream_t st, int face = 0);
// whether the matrix-core block product takes nx x ny (sym: Y is X)
bool block_mm_fits(int nx, int ny, int sym, const DflGeo& d);
// Block-major copy of Ns FP64 fields in FP32: block b, field v, x3 row q of the
// block, element (p * 12 + c) * bs3/2 + k at ((b * Ns + v) * rows + q) * 12 bs3 + ..
// (rows of even length only: block_major_ok)
bool block_major_ok(const DflGeo& d);
hipError_t launch_to_blocks(const Geo& g, const DflGeo& d, const double2* W, int64_t vs, int Ns, float2* out,
                            hipStream_t st);
// launch_block_dots with X block-major (Xb from launch_to_blocks)
hipError_t launch_block_dots_xb(const Geo& g, const DflGeo& d, const float2* Xb, int nx, const double2* Y,
                                int64_t yvs, int ny, double2* out, int64_t bso, int64_t ldo, int64_t kys,
                                hipStream_t st);
template <class EW, class EO>
hipError_t launch_prolong(const Geo& g, const DflGeo& d, const EW* W, int64_t wvs, int Ns, const double2* c,
                          int64_t nc, EO* out, int64_t ovs, int nrhs, hipStream_t st);
hipError_t launch_coarse_apply(const DflGeo& d, const double2* A, int Ns, const double2* in, double2* out,
                               int64_t nc, int nrhs, hipStream_t st);
// y[i] += a * x[i] over n complex elements (a real)
template <class E>
hipError_t launch_add(E* y, const E* x, double a, int64_t n, hipStream_t st);
}  // namespace qdd
