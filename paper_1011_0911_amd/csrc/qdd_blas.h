// Vector-kernel launchers of the outer FGCR (qdd_blas.hip).
#pragma once
#include "qdd_internal.h"

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

}  // namespace qdd
