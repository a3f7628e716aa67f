// Launch-shape autotuner for the stencil kernels: times every candidate
// (threads per block, sites per block, right-hand sides per lane, XCD remap,
// streaming access for Dhat) with
// HIP events on the context's stream and keeps the fastest one.
#include "qdd_api_internal.h"

#include <vector>

using namespace qdd;

extern "C" qdd_status qdd_autotune(qdd_ctx* x, int kernel, qdd_prec prec, int nrhs, const void* in, void* out,
                                   int reps, float* best_ms) {
  if (!x || !in || !out || kernel < 0 || kernel > 1 || prec < QDD_F64 || prec > QDD_F16 || nrhs < 1 ||
      nrhs > x->cfg.max_nrhs || reps < 1) {
    if (x) x->fail("qdd_autotune: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_autotune before qdd_set_params"); return QDD_ESTATE; }
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
        }
      }
      // staged variant (Dhat): R = block / sb lanes per site loop over the right-hand sides
      if (kernel == 0 && lane_groups <= nrhs && staged_lds_bytes(prec, sb) <= kStagedLdsMax)
        for (int xcd : {0, 1, 2, 3}) cand.push_back(LaunchCfg{block, 0, xcd, sb == block ? 0 : sb});
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
