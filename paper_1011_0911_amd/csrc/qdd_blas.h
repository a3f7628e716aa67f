// Vector-kernel launchers of the outer FGCR (qdd_blas.hip).
#pragma once
#include "qdd_kernels.h"

namespace qdd {

constexpr int kDotBlocks = 512;  // partial sums per reduction (per rhs, per dot)

template <class E>
hipError_t launch_dots(const E* x, int64_t lstride, int64_t xrs, int m, const double2* y, int64_t yrs, int64_t n,
                       int nrhs, double2* part, double2* out, hipStream_t st);
template <class E>
hipError_t launch_axpy_multi(double2* y, int64_t yrs, const E* x, int64_t lstride, int64_t xrs, int m,
                             const double2* coef, int ldc, double sgn, int64_t n, int nrhs, const int* active,
                             hipStream_t st);
hipError_t launch_axpby(double2* y, int64_t yrs, const double2* x, int64_t xrs, const double* a, const double* b,
                        int64_t n, int nrhs, const int* active, hipStream_t st);
hipError_t launch_sub(double2* z, const double2* x, const double2* y, int64_t rs, int64_t n, int nrhs,
                      hipStream_t st);
hipError_t launch_norm_finish(const double2* nrm2, double* b, double* binv, int nrhs, hipStream_t st);
hipError_t launch_acc_coef(double2* acc, int lda, const double2* src, int m, int nrhs, hipStream_t st);
// fused update + reduction (one sweep, sums bit-identical to the separate
// launches): y[r] -= sum_{l<m} coef[r*ldc + l] x_l[r] (not where active[r] == 0),
// then out = (mode 0) the m sums <x_l[r], y[r]> ([r][l], for the next
// Gram-Schmidt pass) or (mode 1) <y[r], y[r]> ([r]); part: kDotBlocks * nrhs * m
hipError_t launch_sub_dots(double2* y, int64_t yrs, const double2* x, int64_t lstride, int64_t xrs, int m,
                           const double2* coef, int ldc, const int* active, int mode, int64_t n, int nrhs,
                           double2* part, double2* out, hipStream_t st);
// y[r] <- a[r] y[r], then out[r] = <y[r], w[r]>
hipError_t launch_scale_dot(double2* y, int64_t yrs, const double* a, const double2* w, int64_t wrs, int64_t n,
                            int nrhs, double2* part, double2* out, hipStream_t st);

// ---- the same for several systems in one launch (Grp, qdd_kernels.h): one
// argument record per system, each computing exactly what its own launch of the
// single-system kernel computes (the same partial-sum blocking)
template <class E>
struct DotsArgs {
  const E* x;
  int64_t lstride, xrs;
  int m;
  const double2* y;
  int64_t yrs, n;
  int nrhs;
  int nb;  // set by the launcher
  double2 *part, *out;
};
template <class E>
struct AxpyArgs {
  double2* y;
  int64_t yrs;
  const E* x;
  int64_t lstride, xrs;
  int m;
  const double2* coef;
  int ldc;
  double sgn;
  int64_t n;
  const int* active;
  int nrhs;
};
struct SubArgs {
  double2* z;
  const double2 *x, *y;
  int64_t rs, n;
  int nrhs;
};
struct CoefArgs {
  double2* acc;  // op 0, 2
  int lda;
  const double2* src;  // op 2: src[r*m + l]
  int m;
  const double2* nrm2;  // op 1
  double *b, *binv;
  int nrhs;
};
template <class E>
hipError_t launch_dots_grp(const DotsArgs<E>* a, int ns, hipStream_t st);
template <class E>
hipError_t launch_axpy_multi_grp(const AxpyArgs<E>* a, int ns, hipStream_t st);
hipError_t launch_sub_grp(const SubArgs* a, int ns, hipStream_t st);
// op 0: acc[0 .. nrhs*lda) = 0; op 1: b = |nrm2|^(1/2), binv = 1/b; op 2: acc[r*lda + l] += src[r*m + l]
hipError_t launch_coef_grp(const CoefArgs* a, int ns, int op, hipStream_t st);
// the fused sweeps (launch_sub_dots, launch_scale_dot) over several systems:
// y, x, coef, active as for launch_sub_dots (a, w for launch_scale_dot), out the sums
struct UpdArgs {
  double2* y;
  int64_t yrs;
  const double2* x;
  int64_t lstride, xrs;
  int m;
  const double2* coef;
  int ldc;
  const int* active;
  const double* a;
  const double2* w;
  int64_t wrs, n;
  int nrhs;
  int nb;  // set by the launcher
  double2 *part, *out;
};
hipError_t launch_sub_dots_grp(const UpdArgs* a, int ns, int mode, hipStream_t st);
hipError_t launch_scale_dot_grp(const UpdArgs* a, int ns, hipStream_t st);

}  // namespace qdd
