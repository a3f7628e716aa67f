// Local deflation (host side).
#include "qdd_dfl.h"

using namespace qdd;

qdd_status dfl_make_precond(qdd_ctx* x, int, FgcrOps&) {
  x->fail("deflation not available");
  return QDD_EINVAL;
}

extern "C" qdd_status qdd_dfl_build(qdd_ctx* x, const double*) {
  if (x) x->fail("qdd_dfl_build: not available");
  return QDD_EINVAL;
}
