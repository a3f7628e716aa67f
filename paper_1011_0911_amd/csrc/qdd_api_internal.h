// Host-side context of the qdd library (not part of the public ABI).
#pragma once
#include "../../include/qdd.h"
#include "qdd_kernels.h"
#include "qdd_blas.h"

#include <algorithm>
#include <string>
#include <vector>

namespace qdd {
constexpr int kMaxKv = 32;         // outer Krylov vectors
constexpr int kSapMaxSites = 256;  // sites per Schwarz block (one workgroup)
constexpr int kMaxNs = 64;         // deflation vectors
constexpr int kMaxNetCh = 16;      // network channels
constexpr int kCoarseKv = 16;      // Krylov vectors of the little-operator GCR

// byte offsets of every buffer inside the caller's workspace
struct Layout {
  size_t U[3], A[3], Ai[3];
  size_t tmp_o, tmp_o_scale, flag, dw_shift, dw_ce;
  size_t eta, psi, res, t64, chi, phi;
  bool phi32;
  size_t s_rho, s_psi, s_v, s_eta, s_scale, s_tmp;
  int64_t nblk_dfl;
  size_t dfl_W, dfl_W32, dfl_W32b, dfl_A, dfl_Ainv, dfl_cvec, dfl_init, dfl_cr, dfl_t;
  size_t cpart, ccoef, crn2, calpha, cbinv, cactive;
  size_t net_nw, net_w, net_wb, net_wadj, net_wmx, net_wmxa, net_act, net_grad, net_adam, net_gpart, net_loss, net_tmp;
  size_t net_pairs, net_pairs_bytes, net_gpart_floats;
  size_t part, coef, ahist, bhist, binv, chist, rn2, alpha, active, scal, chrono;
  size_t frc_x, frc_y, frc_lt, frc_src;
  size_t blk_U, blk_A, blk_Ai, blk_work, blk_it, blk_res;
  size_t total;
};

struct PackedView {
  FieldV<double> f64;
  FieldV<float> f32;
  FieldV<__half> f16;
  int64_t poff, spoff;
};
}  // namespace qdd

void compute_layout(const qdd_geom* g, const qdd_config* c, qdd::Layout& Lo);
bool valid_sap_blocks(const qdd_geom* g, const qdd_config* c, std::string* why);

struct Harvest;
struct qdd_ctx {
  qdd_geom geom;
  qdd_config cfg;
  qdd::Geo G;
  qdd::Layout lo;
  char* ws = nullptr;
  hipStream_t st = nullptr;
  int device = 0;  // HIP device current at qdd_create
  bool have_gauge = false, have_clover = false, have_dfl = false, have_net = false;
  double kappa = 0, csw = 0;
  long coarse_iters = 0;  // little-operator GCR iterations since the last solve began
  int net_step = 0;       // Adam steps taken
  int net_calls = 0;      // network stage in the first net_calls preconditioner applications of a solve (0 = all)
  int net_calls_done = 0;  // network-stage applications in the current solve
  std::vector<int> fallbacks;  // network stage rejected, per rhs of the current solve
  std::vector<double> dw_shift_host;  // source of the per-rhs mass shifts copied to the device
  struct Harvest* harvest = nullptr;  // pair capture of the next solve (qdd_solve_harvest)
  qdd::LaunchCfg launch[2][3];
  int sap_variant[3] = {0, 0, 0};  // Schwarz kernel per storage precision (0 = default)
  std::vector<int> chrono_count, chrono_head;  // stored solutions per rhs slot, next slot to write
  int dfl_builds = 0, dfl_refreshes = 0;
  bool have_basis = false;  // the workspace holds a deflation basis (kept across set_gauge / set_params)
  bool blk_ready = false;   // block-major links and clover of the block solver are current
  std::string err;

  template <class T>
  T* ptr(size_t off) const { return (T*)(ws + off); }
  void fail(const char* fmt, ...);
  static std::string& last_global();

  template <class S>
  qdd::DevOp<S> op() const {
    int p = sizeof(S) == 8 ? 0 : (sizeof(S) == 4 ? 1 : 2);
    typedef typename qdd::St<S>::E E;
    return qdd::DevOp<S>{qdd::LinkV<S>{ptr<E>(lo.U[p]), G.Vh}, qdd::CloverV<S>{ptr<E>(lo.A[p]), G.Vh},
                         qdd::CloverV<S>{ptr<E>(lo.Ai[p]), G.Vh}};
  }
  qdd::PackedView packed(qdd_prec prec, int nrhs, int even_only, void* field) const;
  // tmp: device buffer of dhat_tmp_bytes() for the odd-site intermediate (nullptr:
  // the workspace's)
  hipError_t dhat(qdd_prec prec, int nrhs, void* in, void* out, hipEvent_t mid = nullptr, void* tmp = nullptr);
  size_t dhat_tmp_bytes(qdd_prec prec, int nrhs, size_t* scale_off = nullptr) const;
  // ce (device, nrhs doubles, optional): factor on the even sites' clover term per rhs
  hipError_t dw(qdd_prec prec, int nrhs, void* in, void* out, const double* ce = nullptr);
};

#define HCK(x, ...)                                                                   \
  do {                                                                                \
    hipError_t e_ = (__VA_ARGS__);                                                         \
    if (e_ != hipSuccess) {                                                           \
      (x)->fail("HIP error %s at %s:%d", hipGetErrorString(e_), __FILE__, __LINE__); \
      return QDD_EHIP;                                                                \
    }                                                                                 \
  } while (0)
