// Internal interface between the outer FGCR and its operators / preconditioners.
#pragma once
#include "qdd_api_internal.h"
#include <functional>

struct FgcrOps {
  int64_t n = 0;      // complex numbers per right-hand side
  int nrhs = 1;
  bool phi32 = false;  // preconditioner output stored as float2 (else double2)
  bool sync_stages = false;
  std::function<qdd_status(const double2* in, double2* out)> op;  // FP64 operator, whole batch
  std::function<qdd_status(const double2* r, void* phi)> prec;    // phi = M(r), whole batch
  int* fallbacks = nullptr;  // per rhs (network stage)
  double* tstage = nullptr;  // preconditioner sub-stage times (ms), indices 4..6
};

qdd_status run_fgcr(qdd_ctx* x, FgcrOps& F, const double2* eta, double2* psi, qdd_solve_info* info);
// operator D (FP64) and the configured preconditioner for qdd_solve
qdd_status make_solver_ops(qdd_ctx* x, int nrhs, FgcrOps& F);
