// Preconditioners of the outer FGCR: identity, Schwarz (SAP) and the two-level
// deflated SAP, each applied to a whole right-hand-side batch.
#include "qdd_solver.h"

using namespace qdd;

qdd_status make_solver_ops(qdd_ctx* x, int nrhs, FgcrOps& F) {
  int64_t n = (int64_t)24 * x->G.Vh;
  F.n = n;
  F.nrhs = nrhs;
  F.op = [x, nrhs](const double2* in, double2* out) -> qdd_status {
    HCK(x, x->dw(QDD_F64, nrhs, (void*)in, out));
    return QDD_OK;
  };
  if (x->cfg.precond == QDD_PRECOND_NONE) {
    F.phi32 = false;
    F.prec = [x, nrhs, n](const double2* r, void* phi) -> qdd_status {
      HCK(x, hipMemcpyAsync(phi, r, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, x->st));
      return QDD_OK;
    };
    return QDD_OK;
  }
  x->fail("preconditioner not available");
  return QDD_EINVAL;
}

extern "C" qdd_status qdd_sap(qdd_ctx* x, int, const double*, double*) {
  if (x) x->fail("qdd_sap: not available");
  return QDD_EINVAL;
}
extern "C" qdd_status qdd_dfl_build(qdd_ctx* x, const double*) {
  if (x) x->fail("qdd_dfl_build: not available");
  return QDD_EINVAL;
}
