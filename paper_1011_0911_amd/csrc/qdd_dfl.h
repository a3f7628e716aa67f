// Local deflation: subspace build, little Dirac operator, coarse solve and the
// two-level preconditioner (qdd_dfl.cpp / qdd_dfl.hip).
#pragma once
#include "qdd_solver.h"

qdd_status sap_apply(qdd_ctx* x, int nrhs, const double2* eta, void* psi);
qdd_status dfl_make_precond(qdd_ctx* x, int nrhs, FgcrOps& F);
qdd_status dfl_precond_apply(qdd_ctx* x, int nrhs, const double2* r, void* phi);
qdd_status net_stage(qdd_ctx* x, int nrhs, const double2* r1, float2* vn, double2* r2, float2* tbuf,
                     std::vector<int>& fb);
