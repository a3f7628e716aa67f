// C entry of the Dirichlet block solver (the BiCGstab block inversions of the
// DD-HMC forces, Sect. 3); the kernels are in qdd_block.hip.
#include <algorithm>
#include <vector>

#include "qdd_api_internal.h"
#include "qdd_kernels.h"

using namespace qdd;

extern "C" qdd_status qdd_block_solve(qdd_ctx* x, int nrhs, const double* eta, double* psi, double tol, int maxit,
                                      int* blk_iters, double* blk_res, qdd_block_info* info) {
  if (!x || !eta || !psi || nrhs < 1 || nrhs > x->cfg.max_nrhs || !(tol > 0) || maxit < 1 || !x->cfg.blk_bs[0]) {
    if (x) x->fail("qdd_block_solve: invalid arguments (needs config.blk_bs)");
    return QDD_EINVAL;
  }
  if (!x->have_clover) {
    x->fail("qdd_block_solve before qdd_set_params");
    return QDD_ESTATE;
  }
  const Geo& G = x->G;
  BlkGeo B;
  B.nblk = 1;
  for (int i = 0; i < 4; ++i) {
    B.bs[i] = x->cfg.blk_bs[i];
    B.nb[i] = G.L[i] / B.bs[i];
    B.nblk *= B.nb[i];
  }
  B.neb = G.Vh / B.nblk;
  hipStream_t st = x->st;
  double2 *BU = x->ptr<double2>(x->lo.blk_U), *BA = x->ptr<double2>(x->lo.blk_A), *BAi = x->ptr<double2>(x->lo.blk_Ai);
  if (!x->blk_ready) {
    HCK(x, launch_blk_gather(G, B, x->ptr<double2>(x->lo.U[0]), x->ptr<double2>(x->lo.A[0]),
                             x->ptr<double2>(x->lo.Ai[0]), BU, BA, BAi, st));
    x->blk_ready = true;
  }
  int* it_d = x->ptr<int>(x->lo.blk_it);
  double* res_d = x->ptr<double>(x->lo.blk_res);
  hipEvent_t e0, e1;
  HCK(x, hipEventCreate(&e0));
  HCK(x, hipEventCreate(&e1));
  hipError_t err = hipEventRecord(e0, st);
  if (err == hipSuccess)
    err = launch_blk_bicgstab(G, B, BU, BA, BAi, x->ptr<double2>(x->lo.blk_work), (const double2*)eta, (double2*)psi,
                              nrhs, tol, maxit, it_d, res_d, st);
  if (err == hipSuccess) err = hipEventRecord(e1, st);
  const size_t n = (size_t)nrhs * B.nblk;
  std::vector<int> it(n);
  std::vector<double> res(n);
  if (err == hipSuccess) err = hipMemcpyAsync(it.data(), it_d, n * sizeof(int), hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipMemcpyAsync(res.data(), res_d, n * sizeof(double), hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  float ms = 0;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HCK(x, err);
  qdd_block_info inf{};
  inf.nblk = (int)n;
  inf.t_ms = ms;
  for (size_t k = 0; k < n; ++k) {
    if (it[k] < 0) ++inf.breakdowns;
    else if (res[k] <= tol) ++inf.converged;
    inf.iters_max = std::max(inf.iters_max, it[k]);
    inf.res_max = std::max(inf.res_max, res[k]);
  }
  if (blk_iters) std::copy(it.begin(), it.end(), blk_iters);
  if (blk_res) std::copy(res.begin(), res.end(), blk_res);
  if (info) *info = inf;
  if (inf.converged != inf.nblk) {
    x->fail("qdd_block_solve: %d of %d blocks did not converge (%d breakdowns)", inf.nblk - inf.converged, inf.nblk,
            inf.breakdowns);
    return QDD_ENOCONV;
  }
  return QDD_OK;
}
