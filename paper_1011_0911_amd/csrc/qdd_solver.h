// Internal interface between the outer FGCR and its operators / preconditioners.
#pragma once
#include "qdd_api_internal.h"
#include <functional>
#include <vector>

// optional capture of (residual, iterate) pairs at every iteration of every
// right-hand side; after the solve the iterates are turned into errors
// e_k = psi* - psi_k
struct Harvest {
  float2* r = nullptr;  // packed FP32 full fields, one per pair
  void* e = nullptr;    // FP64-sized slots during the solve; FP32 errors packed at the front afterwards
  int max = 0, n = 0;
  std::vector<int> rhs;  // right-hand side of each pair
};

struct FgcrOps {
  int64_t n = 0;      // complex numbers per right-hand side
  int nrhs = 1;
  bool phi32 = false;  // preconditioner output stored as float2 (else double2)
  bool sync_stages = false;
  bool warm = false;  // psi holds an initial guess (else the solve starts from 0)
  std::function<qdd_status(const double2* in, double2* out)> op;  // FP64 operator, whole batch
  std::function<qdd_status(const double2* r, void* phi)> prec;    // phi = M(r), whole batch
  int* fallbacks = nullptr;  // per rhs (network stage)
  double* tstage = nullptr;  // preconditioner sub-stage times (ms), indices 4..6
  Harvest* hv = nullptr;
};

qdd_status run_fgcr(qdd_ctx* x, FgcrOps& F, const double2* eta, double2* psi, qdd_solve_info* info);
// HIP events at stage boundaries on one stream; gpu_ms[k] accumulates the time
// between marks k and k + 1 once the stream has been waited for
struct StageEvents {
  hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double gpu_ms[4] = {0, 0, 0, 0};
  hipError_t init() {
    for (auto& v : e) {
      hipError_t r = hipEventCreate(&v);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  }
  hipError_t mark(int k, hipStream_t st) { return hipEventRecord(e[k], st); }
  // after a wait on the stream: stage k = [mark k, mark k + 1) for k in [k0, k1)
  hipError_t add(int k0, int k1) {
    for (int k = k0; k < k1; ++k) {
      float ms = 0;
      hipError_t r = hipEventElapsedTime(&ms, e[k], e[k + 1]);
      if (r != hipSuccess) return r;
      gpu_ms[k] += ms;
    }
    return hipSuccess;
  }
  ~StageEvents() {
    for (auto v : e)
      if (v) (void)hipEventDestroy(v);
  }
};

// alpha (al[0 .. m)) of right-hand side i from the host copies of the Gram-Schmidt
// coefficients (ah), the norms (bh) and the projections (chh) of m steps
void fgcr_backsub(const double2* ah, const double* bh, const double2* chh, int nr, int i, int m, double2* al);
// the Schwarz preconditioner of ns systems (FP32 storage), every stage one launch
// over all systems: psi[s] = M_sap eta[s] (st: the stream of the whole group)
qdd_status sap_apply_grp(qdd_ctx* const* xs, const int* nrhs, const double2* const* eta, void* const* psi, int ns,
                         hipStream_t st);
// operator D (FP64) and the configured preconditioner for qdd_solve
qdd_status make_solver_ops(qdd_ctx* x, int nrhs, FgcrOps& F);
