// Autotuner: for the stencil kernels times every candidate launch shape
// (threads per block, sites per block, right-hand sides per lane, XCD remap,
// streaming access for Dhat), for the Schwarz procedure every half-sweep kernel
// variant, with HIP events on the context's stream, and keeps the fastest one.
#include "qdd_api_internal.h"
#include "qdd_sap.h"

#include <vector>

using namespace qdd;

qdd_status sap_apply(qdd_ctx* x, int nrhs, const double2* eta, void* psi);

// Schwarz procedure: times each half-sweep kernel variant on whole preconditioner
// calls psi = M_sap eta (eta: packed FP64 full fields, psi: packed FP32 full fields)
static qdd_status tune_sap(qdd_ctx* x, qdd_prec prec, int nrhs, const void* in, void* out, int reps,
                           float* best_ms) {
  if (prec != x->cfg.sap_prec || prec == QDD_F64) {
    x->fail("qdd_autotune: the Schwarz kernel is tuned for the configured FP32 or FP16 SAP precision");
    return QDD_EINVAL;
  }
  std::string why;
  if (!valid_sap_blocks(&x->geom, &x->cfg, &why)) {
    x->fail("qdd_autotune: %s", why.c_str());
    return QDD_EINVAL;
  }
  hipEvent_t e0, e1;
  HCK(x, hipEventCreate(&e0));
  HCK(x, hipEventCreate(&e1));
  const int keep = x->sap_variant[prec];
  int best = keep;
  float tbest = 1e30f;
  qdd_status st = QDD_OK;
  hipError_t err = hipSuccess;
  for (int v = 1; v <= 4 && st == QDD_OK && err == hipSuccess; ++v) {
    if (!sap_variant_ok(prec, v)) continue;
    x->sap_variant[prec] = v;
    st = sap_apply(x, nrhs, (const double2*)in, out);  // warm-up
    if (st == QDD_OK) err = hipEventRecord(e0, x->st);
    for (int r = 0; r < reps && st == QDD_OK && err == hipSuccess; ++r) st = sap_apply(x, nrhs, (const double2*)in, out);
    if (st == QDD_OK && err == hipSuccess) err = hipEventRecord(e1, x->st);
    if (st == QDD_OK && err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0;
    if (st == QDD_OK && err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (st != QDD_OK || err != hipSuccess) break;
    ms /= reps;
    if (ms < tbest) {
      tbest = ms;
      best = v;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  x->sap_variant[prec] = (st == QDD_OK && err == hipSuccess) ? best : keep;
  if (st != QDD_OK) return st;
  HCK(x, err);
  if (best_ms) *best_ms = tbest;
  return QDD_OK;
}

extern "C" qdd_status qdd_autotune(qdd_ctx* x, int kernel, qdd_prec prec, int nrhs, const void* in, void* out,
                                   int reps, float* best_ms) {
  if (!x || !in || !out || kernel < 0 || kernel > 2 || prec < QDD_F64 || prec > QDD_F16 || nrhs < 1 ||
      nrhs > x->cfg.max_nrhs || reps < 1) {
    if (x) x->fail("qdd_autotune: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_autotune before qdd_set_params"); return QDD_ESTATE; }
  if (kernel == 2) return tune_sap(x, prec, nrhs, in, out, reps, best_ms);
  std::vector<LaunchCfg> cand;
  for (int block : {64, 128, 256})
    for (int sb : {16, 32, 64, 128, 256}) {
      if (sb > block || block % sb) continue;
      int lane_groups = block / sb;
      for (int nr : {1, 2, 4}) {
        if (lane_groups * nr > 2 * nrhs && !(lane_groups == 1 && nr == 1)) continue;  // mostly idle lanes
        if (nr > nrhs) continue;
        for (int xcd : {0, 1, 2, 3}) {
          cand.push_back(LaunchCfg{block, nr, xcd, sb == block ? 0 : sb});
          if (kernel == 0 && nr == 1)  // streaming access: links + clover (4), own spinor + output (8);
                                       // compressed links (16)
            for (int ntm : {4, 8, 12, 16, 20, 24, 28}) cand.push_back(LaunchCfg{block, nr, xcd | ntm, sb == block ? 0 : sb});
          if (kernel == 0 && nr > 1 && dhat_vec_ok(prec, nr) && nrhs % nr == 0)  // rhs-vector loads
            for (int ntm : {0, 8, 16, 24}) cand.push_back(LaunchCfg{block, nr, xcd | 32 | ntm, sb == block ? 0 : sb});
        }
      }
      // staged variant (Dhat): R = block / sb lanes per site loop over the right-hand sides
      if (kernel == 0 && lane_groups <= nrhs && staged_lds_bytes(prec, sb) <= kStagedLdsMax)
        for (int xcd : {0, 1, 2, 3}) cand.push_back(LaunchCfg{block, 0, xcd, sb == block ? 0 : sb});
    }
  if (kernel == 0) {  // the same shapes with pass B walking backwards
    const size_t n = cand.size();
    for (size_t k = 0; k < n; ++k)
      if (cand[k].nr != 0) cand.push_back(LaunchCfg{cand[k].block, cand[k].nr, cand[k].xcd | 64, cand[k].sb});
  }
  hipEvent_t e0, e1;
  HCK(x, hipEventCreate(&e0));
  HCK(x, hipEventCreate(&e1));
  LaunchCfg keep = x->launch[kernel][prec], best = keep;
  float tbest = 1e30f;
  hipError_t err = hipSuccess;
  for (const LaunchCfg& c : cand) {
    x->launch[kernel][prec] = c;
    auto run = [&]() { return kernel == 0 ? x->dhat(prec, nrhs, (void*)in, out) : x->dw(prec, nrhs, (void*)in, out); };
    err = run();  // warm-up
    if (err == hipSuccess) err = hipEventRecord(e0, x->st);
    for (int r = 0; r < reps && err == hipSuccess; ++r) err = run();
    if (err == hipSuccess) err = hipEventRecord(e1, x->st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err != hipSuccess) break;
    ms /= reps;
    if (ms < tbest) {
      tbest = ms;
      best = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  x->launch[kernel][prec] = err == hipSuccess ? best : keep;
  HCK(x, err);
  if (best_ms) *best_ms = tbest;
  return QDD_OK;
}
