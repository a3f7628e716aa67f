// Host side of the qdd C ABI: context, workspace layout, set-up calls, the
// operator entry points and the FP64 flexible GCR driver.
#include "../../include/qdd.h"
#include "qdd_api_internal.h"
#include "qdd_net.h"
#include "qdd_sap.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

using namespace qdd;

// ------------------------------------------------------------------ helpers
void qdd_ctx::fail(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  char buf[512];
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  err = buf;
}

static bool valid_geom(const qdd_geom* g, std::string* why) {
  if (!g) { *why = "null geometry"; return false; }
  for (int i = 0; i < 4; ++i)
    if (g->L[i] < 2 || (g->L[i] & 1)) { *why = "every lattice extent must be even and >= 2"; return false; }
  if (g->bc_time != 1 && g->bc_time != -1) { *why = "bc_time must be +1 or -1"; return false; }
  int64_t V = (int64_t)g->L[0] * g->L[1] * g->L[2] * g->L[3];
  if (V > (int64_t)1 << 30) { *why = "lattice volume above 2^30 sites"; return false; }
  return true;
}

static bool valid_blocks(const qdd_geom* g, const int* bs, bool need_even_count, std::string* why,
                         const char* what) {
  for (int i = 0; i < 4; ++i) {
    if (bs[i] < 1 || g->L[i] % bs[i]) { *why = std::string(what) + " block extents must divide the lattice"; return false; }
    if (need_even_count && ((g->L[i] / bs[i]) & 1)) {
      *why = std::string(what) + ": the number of blocks in every direction must be even";
      return false;
    }
  }
  return true;
}

bool valid_sap_blocks(const qdd_geom* g, const qdd_config* c, std::string* why) {
  if (!valid_blocks(g, c->sap_bs, true, why, "SAP")) return false;
  int nsite = c->sap_bs[0] * c->sap_bs[1] * c->sap_bs[2] * c->sap_bs[3];
  for (int i = 0; i < 4; ++i)
    if (c->sap_bs[i] & 1) {
      *why = "SAP block extents must be even";
      return false;
    }
  if (nsite > kSapMaxSites) {
    *why = "SAP blocks may hold at most 256 sites";
    return false;
  }
  return true;
}

static bool valid_cfg(const qdd_geom* g, const qdd_config* c, std::string* why) {
  if (!c) { *why = "null configuration"; return false; }
  if (c->max_nrhs < 1 || c->max_nrhs > 64) { *why = "max_nrhs must be in 1..64"; return false; }
  if (c->nkv < 1 || c->nkv > kMaxKv) { *why = "nkv must be in 1..32"; return false; }
  if (c->nmx < 1) { *why = "nmx must be >= 1"; return false; }
  if (!(c->tol > 0)) { *why = "tol must be > 0"; return false; }
  if (c->sap_prec < QDD_F64 || c->sap_prec > QDD_F16) { *why = "invalid sap_prec"; return false; }
  if (c->precond < QDD_PRECOND_NONE || c->precond > QDD_PRECOND_DFL) { *why = "invalid precond"; return false; }
  if (c->ncy < 1 || c->nmr < 1) { *why = "ncy and nmr must be >= 1"; return false; }
  // the Schwarz blocks matter only where SAP runs (preconditioner, subspace build)
  if (c->precond != QDD_PRECOND_NONE || c->dfl_Ns > 0)
    if (!valid_sap_blocks(g, c, why)) return false;
  if (c->dfl_Ns < 0 || c->dfl_Ns > kMaxNs) { *why = "dfl_Ns must be in 0..64"; return false; }
  if (c->dfl_Ns > 0) {
    if (!valid_blocks(g, c->dfl_bs, false, why, "deflation")) return false;
    if (c->dfl_nit < 0 || !(c->dfl_coarse_tol > 0) || c->dfl_coarse_nmx < 1) {
      *why = "invalid deflation parameters";
      return false;
    }
  }
  if (c->precond == QDD_PRECOND_DFL && c->dfl_Ns == 0) { *why = "precond DFL needs dfl_Ns > 0"; return false; }
  if (c->chrono_nv < 0 || c->chrono_nv > 16 || c->chrono_nv > c->nkv * c->max_nrhs) {
    *why = "chrono_nv must be in 0..min(16, nkv * max_nrhs)";
    return false;
  }
  if (c->dfl_refresh_iters < 0 || c->dfl_refresh_nit < 0) { *why = "invalid refresh parameters"; return false; }
  if (c->force != 0 && c->force != 1) { *why = "force must be 0 or 1"; return false; }
  if (c->blk_bs[0] || c->blk_bs[1] || c->blk_bs[2] || c->blk_bs[3]) {
    if (!valid_blocks(g, c->blk_bs, false, why, "block-solver")) return false;
    for (int i = 0; i < 4; ++i)
      if (c->blk_bs[i] & 1) { *why = "block-solver block extents must be even"; return false; }
  }
  if (c->use_net) {
    if (c->net_nl < 1 || c->net_nl > 7 || c->net_ch[0] != 1 || c->net_ch[c->net_nl] != 1) {
      *why = "network: 1..7 layers, one input and one output channel";
      return false;
    }
    for (int l = 1; l < c->net_nl; ++l)
      if (c->net_ch[l] < 1 || c->net_ch[l] > kMaxNetCh) { *why = "network: channels must be in 1..16"; return false; }
    if (c->net_terms < 1 || c->net_terms > 3) { *why = "network: net_terms must be 1, 2 or 3"; return false; }
    if (c->dfl_Ns == 0) { *why = "network stage needs deflation (dfl_Ns > 0)"; return false; }
    if (c->sap_prec == QDD_F64) { *why = "network stage needs FP32 or FP16 SAP"; return false; }
  }
  return true;
}

// ------------------------------------------------------------------ layout
static size_t elem_bytes(qdd_prec p) { return p == QDD_F64 ? 16 : (p == QDD_F32 ? 8 : 4); }

void compute_layout(const qdd_geom* g, const qdd_config* c, Layout& Lo) {
  struct Bump {
    size_t off = 0;
    size_t take(size_t b) {
      off = (off + 255) & ~size_t(255);
      size_t o = off;
      off += b;
      return o;
    }
  } B;
  int64_t V = (int64_t)g->L[0] * g->L[1] * g->L[2] * g->L[3], Vh = V / 2;
  int nr = c->max_nrhs, nkv = c->nkv;
  int64_t links = 2 * 4 * 9 * Vh, clov = 2 * 36 * Vh;
  Lo.U[0] = B.take(links * 16);
  Lo.U[1] = B.take(links * 8);
  Lo.U[2] = B.take(links * 4);
  for (int p = 0; p < 3; ++p) {
    Lo.A[p] = B.take(clov * elem_bytes((qdd_prec)p));
    Lo.Ai[p] = B.take(clov * elem_bytes((qdd_prec)p));
  }
  Lo.tmp_o = B.take((size_t)nr * 12 * Vh * 16);
  Lo.tmp_o_scale = B.take((size_t)nr * Vh * 4);
  Lo.dw_shift = B.take((size_t)kMaxShift * 8);
  Lo.dw_ce = B.take((size_t)kMaxShift * 8);
  Lo.flag = B.take(256);
  // FP64 solver fields (full lattice, nr rhs)
  size_t f64 = (size_t)nr * 24 * Vh * 16;
  Lo.eta = B.take(f64);
  Lo.psi = B.take(f64);
  Lo.res = B.take(f64);
  Lo.t64 = B.take(f64);
  Lo.chi = B.take(f64 * nkv);
  bool phi32 = c->precond != QDD_PRECOND_NONE && c->sap_prec != QDD_F64;
  Lo.phi32 = phi32;
  Lo.phi = B.take((size_t)nr * 24 * Vh * (phi32 ? 8 : 16) * nkv);
  // SAP fields in the SAP precision: rho, psi, v (+ FP16 scales) and an FP64 staging copy
  size_t se = elem_bytes(c->sap_prec);
  Lo.s_rho = B.take((size_t)nr * 24 * Vh * se);
  Lo.s_psi = B.take((size_t)nr * 24 * Vh * se);
  Lo.s_v = B.take((size_t)nr * 24 * Vh * se);
  Lo.s_eta = B.take((size_t)nr * 24 * Vh * se);
  Lo.s_scale = B.take((size_t)4 * nr * 2 * Vh * 4);
  Lo.s_tmp = B.take(f64);
  // deflation
  Lo.nblk_dfl = 0;
  if (c->dfl_Ns > 0) {
    int64_t nb = 1;
    for (int i = 0; i < 4; ++i) nb *= g->L[i] / c->dfl_bs[i];
    Lo.nblk_dfl = nb;
    int Ns = c->dfl_Ns;
    Lo.dfl_W = B.take((size_t)Ns * 24 * Vh * 16);
    Lo.dfl_W32 = B.take((size_t)Ns * 24 * Vh * 8);
    Lo.dfl_W32b = B.take((size_t)Ns * 24 * Vh * 8);  // block-major copy for the restriction
    Lo.dfl_A = B.take((size_t)nb * 9 * Ns * Ns * 16);
    Lo.dfl_Ainv = B.take((size_t)nb * Ns * Ns * 16);
    size_t cv = (size_t)nr * nb * Ns * 16;
    Lo.dfl_cvec = B.take(cv * (2 * kCoarseKv + 8));
    // start fields / block-hop scratch of the build: shares the Krylov space when
    // that is large enough (the build and the solves never overlap)
    if ((int64_t)nkv * nr >= Ns) Lo.dfl_init = Lo.chi;
    else Lo.dfl_init = B.take((size_t)Ns * 24 * Vh * 16);
    Lo.dfl_cr = B.take((size_t)nr * 24 * Vh * 16);
    Lo.dfl_t = B.take((size_t)nr * 24 * Vh * 16);
    Lo.cpart = B.take((size_t)kDotBlocks * kCoarseKv * nr * 16 + 4096);
    Lo.ccoef = B.take((size_t)nr * kCoarseKv * 16);
    Lo.crn2 = B.take((size_t)nr * 16);
    Lo.calpha = B.take((size_t)nr * 16);
    Lo.cbinv = B.take((size_t)nr * 16);
    Lo.cactive = B.take((size_t)nr * 4);
  }
  // network weights, activations (levels 0..nl and two gradient buffers) and
  // the staging area for training pairs
  Lo.net_nw = 0;
  if (c->use_net) {
    size_t nw = 0, maxch = 1;
    for (int l = 0; l < c->net_nl; ++l) {
      size_t k = (size_t)9 * c->net_ch[l] * c->net_ch[l + 1] * 16;
      nw += k;
      maxch = std::max<size_t>(maxch, c->net_ch[l + 1]);
    }
    Lo.net_nw = nw;
    Lo.net_w = B.take(nw * 8);       // complex FP32 master weights
    Lo.net_wb = B.take(nw * 4);      // complex BF16 compute copy
    Lo.net_wadj = B.take(nw * 4);    // BF16 adjoint weights (backward pass)
    // matrix-core operand copies, forward (the two gradient levels, 2 maxch
    // channel fields, serve as scratch there) and backward (no scratch)
    size_t nmx = 0, nmxa = 0;
    for (int l = 0; l < c->net_nl; ++l) {
      nmx += net_wmx_elems(c->net_ch[l], c->net_ch[l + 1], (int)(2 * maxch));
      nmxa += net_wmx_elems(c->net_ch[l + 1], c->net_ch[l], 0);
    }
    Lo.net_wmx = B.take(nmx * 2);
    Lo.net_wmxa = B.take(nmxa * 2);
    Lo.net_act = B.take((size_t)(c->net_nl + 3) * maxch * 24 * Vh * 8);
    Lo.net_grad = B.take(nw * 8);
    Lo.net_adam = B.take(nw * 16);
    size_t gpart = 0;  // weight-gradient partial products (floats), the largest layer's need
    for (int l = 0; l < c->net_nl; ++l)
      gpart = std::max(gpart, net_wgrad_part_floats(V, c->net_ch[l], c->net_ch[l + 1]));
    Lo.net_gpart_floats = gpart;
    Lo.net_gpart = B.take(gpart * 4);
    Lo.net_loss = B.take(4096 * 8);
    Lo.net_tmp = B.take((size_t)nr * 24 * Vh * 8);
    Lo.net_pairs_bytes = (size_t)2 * 8 * 24 * Vh * 8;
    Lo.net_pairs = B.take(Lo.net_pairs_bytes);
  }
  // chronological inversion: the last chrono_nv solutions of every rhs slot (FP64 full fields)
  Lo.chrono = c->chrono_nv > 0 ? B.take((size_t)c->chrono_nv * nr * 24 * Vh * 16) : 0;
  // force buffers: X- and Y-type full fields of the two pseudofermion terms
  // ([term][parity][site][12] complex), the clover insertions ([parity][plane][9][site])
  // and two canonical even fields
  Lo.frc_x = Lo.frc_y = Lo.frc_lt = Lo.frc_src = 0;
  if (c->force) {
    Lo.frc_x = B.take((size_t)2 * 24 * Vh * 16);
    Lo.frc_y = B.take((size_t)2 * 24 * Vh * 16);
    Lo.frc_lt = B.take((size_t)2 * 6 * 9 * Vh * 8);
    Lo.frc_src = B.take((size_t)2 * 12 * Vh * 16);
  }
  // block solver: block-major links and clover blocks (both parities), eight
  // FP64 even-site vectors per rhs, per-block iteration counts and residuals
  Lo.blk_U = Lo.blk_A = Lo.blk_Ai = Lo.blk_work = Lo.blk_it = Lo.blk_res = 0;
  if (c->blk_bs[0]) {
    int64_t nblk = 1;
    for (int i = 0; i < 4; ++i) nblk *= g->L[i] / c->blk_bs[i];
    Lo.blk_U = B.take(links * 16);
    Lo.blk_A = B.take(clov * 16);
    Lo.blk_Ai = B.take(clov * 16);
    Lo.blk_work = B.take((size_t)nr * 8 * 12 * Vh * 16);
    Lo.blk_it = B.take((size_t)nr * nblk * 4);
    Lo.blk_res = B.take((size_t)nr * nblk * 8);
  }
  // reductions and small solver arrays
  Lo.part = B.take((size_t)kDotBlocks * kMaxKv * nr * 16 + 4096);
  Lo.coef = B.take((size_t)nr * kMaxKv * 16);
  Lo.ahist = B.take((size_t)kMaxKv * nr * kMaxKv * 16);
  Lo.bhist = B.take((size_t)kMaxKv * nr * 8);
  Lo.binv = B.take((size_t)nr * 8);
  Lo.chist = B.take((size_t)kMaxKv * nr * 16);
  Lo.rn2 = B.take((size_t)nr * 16 * 4);
  Lo.alpha = B.take((size_t)nr * kMaxKv * 16);
  Lo.active = B.take((size_t)nr * 4);
  Lo.scal = B.take((size_t)nr * 64 * 8);
  Lo.total = (B.off + 255) & ~size_t(255);
}

// ------------------------------------------------------------------ API
extern "C" {

void qdd_config_default(qdd_config* c) {
  std::memset(c, 0, sizeof(*c));
  c->max_nrhs = 1;
  for (int i = 0; i < 4; ++i) c->sap_bs[i] = c->dfl_bs[i] = 4;
  c->ncy = 5;
  c->nmr = 4;
  c->sap_prec = QDD_F32;
  c->dfl_Ns = 0;
  c->dfl_nit = 5;
  c->dfl_coarse_tol = 1e-6;
  c->dfl_coarse_nmx = 2000;
  c->nkv = 16;
  c->nmx = 2048;
  c->tol = 1e-10;
  c->precond = QDD_PRECOND_NONE;
  c->use_net = 0;
  c->net_nl = 3;
  c->net_ch[0] = 1;
  c->net_ch[1] = 12;
  c->net_ch[2] = 12;
  c->net_ch[3] = 1;
  c->net_terms = 3;
  c->chrono_nv = 0;
  c->dfl_refresh_iters = 0;
  c->dfl_refresh_nit = 2;
  c->force = 0;
  for (int i = 0; i < 4; ++i) c->blk_bs[i] = 0;
}

size_t qdd_workspace_bytes(const qdd_geom* g, const qdd_config* c) {
  std::string why;
  if (!valid_geom(g, &why) || !valid_cfg(g, c, &why)) return 0;
  Layout Lo;
  compute_layout(g, c, Lo);
  return Lo.total;
}

qdd_status qdd_create(const qdd_geom* g, const qdd_config* c, void* ws, size_t ws_bytes, void* stream,
                      qdd_ctx** out) {
  if (!out) return QDD_EINVAL;
  *out = nullptr;
  std::string why;
  if (!valid_geom(g, &why) || !valid_cfg(g, c, &why)) {
    qdd_ctx::last_global() = why;
    return QDD_EINVAL;
  }
  Layout Lo;
  compute_layout(g, c, Lo);
  if (!ws || ws_bytes < Lo.total) {
    qdd_ctx::last_global() = "workspace missing or smaller than qdd_workspace_bytes()";
    return QDD_ENOWS;
  }
  if (((uintptr_t)ws & 255) != 0) {
    qdd_ctx::last_global() = "workspace must be 256-byte aligned";
    return QDD_EINVAL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    qdd_ctx::last_global() = "hipGetDevice failed";
    return QDD_EHIP;
  }
  qdd_ctx* x = new qdd_ctx();
  x->device = dev;
  x->chrono_count.assign(c->max_nrhs, 0);
  x->chrono_head.assign(c->max_nrhs, 0);
  x->geom = *g;
  x->cfg = *c;
  x->lo = Lo;
  x->ws = (char*)ws;
  x->st = (hipStream_t)stream;
  Geo& G = x->G;
  for (int i = 0; i < 4; ++i) G.L[i] = g->L[i];
  G.V = g->L[0] * g->L[1] * g->L[2] * g->L[3];
  G.Vh = G.V / 2;
  G.Lh3 = g->L[3] / 2;
  G.bc = g->bc_time;
  for (int k = 0; k < 2; ++k)
    for (int p = 0; p < 3; ++p) x->launch[k][p] = LaunchCfg();
  // Dhat: streaming access to the own spinor and the output (the better or equal
  // choice for every precision and batch size measured at 32^3x64)
  for (int p = 0; p < 3; ++p) x->launch[0][p].xcd = 2 | 8;
  *out = x;
  return QDD_OK;
}

void qdd_destroy(qdd_ctx* x) { delete x; }

const char* qdd_last_error(const qdd_ctx* x) {
  return x ? x->err.c_str() : qdd_ctx::last_global().c_str();
}

qdd_status qdd_set_gauge(qdd_ctx* x, const double* links) {
  if (!x || !links) return QDD_EINVAL;
  const Geo& G = x->G;
  int64_t n = (int64_t)2 * 4 * 9 * G.Vh;
  HCK(x, launch_pack_links(G, links, x->ptr<double2>(x->lo.U[0]), x->st));
  HCK(x, launch_convert(x->ptr<double2>(x->lo.U[0]), x->ptr<float2>(x->lo.U[1]), n, x->st));
  HCK(x, launch_convert(x->ptr<double2>(x->lo.U[0]), x->ptr<__half2>(x->lo.U[2]), n, x->st));
  x->have_gauge = true;
  x->have_clover = false;
  x->have_dfl = false;
  x->blk_ready = false;
  return QDD_OK;
}

qdd_status qdd_set_params(qdd_ctx* x, double kappa, double csw) {
  if (!x) return QDD_EINVAL;
  if (!x->have_gauge) { x->fail("qdd_set_params before qdd_set_gauge"); return QDD_ESTATE; }
  if (!(kappa > 0) || !std::isfinite(csw)) { x->fail("kappa must be > 0 and c_sw finite"); return QDD_EINVAL; }
  const Geo& G = x->G;
  int* flag = x->ptr<int>(x->lo.flag);
  HCK(x, hipMemsetAsync(flag, 0, sizeof(int), x->st));
  HCK(x, launch_clover(G, x->ptr<double2>(x->lo.U[0]), 1.0 / (2.0 * kappa), csw, x->ptr<double2>(x->lo.A[0]),
                       x->ptr<double2>(x->lo.Ai[0]), flag, x->st));
  int64_t n = (int64_t)2 * 36 * G.Vh;
  HCK(x, launch_convert(x->ptr<double2>(x->lo.A[0]), x->ptr<float2>(x->lo.A[1]), n, x->st));
  HCK(x, launch_convert(x->ptr<double2>(x->lo.Ai[0]), x->ptr<float2>(x->lo.Ai[1]), n, x->st));
  HCK(x, launch_convert(x->ptr<double2>(x->lo.A[0]), x->ptr<__half2>(x->lo.A[2]), n, x->st));
  HCK(x, launch_convert(x->ptr<double2>(x->lo.Ai[0]), x->ptr<__half2>(x->lo.Ai[2]), n, x->st));
  int bad = 0;
  HCK(x, hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, x->st));
  HCK(x, hipStreamSynchronize(x->st));
  x->kappa = kappa;
  x->csw = csw;
  x->have_dfl = false;
  x->blk_ready = false;
  if (bad) {
    x->have_clover = false;
    x->fail("%d clover blocks are not positive definite", bad);
    return QDD_ESINGULAR;
  }
  x->have_clover = true;
  return QDD_OK;
}

size_t qdd_field_bytes(const qdd_ctx* x, qdd_prec prec, int nrhs, int even_only) {
  if (!x || nrhs < 1 || prec < QDD_F64 || prec > QDD_F16) return 0;
  size_t sites = (size_t)x->G.Vh * (even_only ? 1 : 2);
  size_t b = sites * 12 * elem_bytes(prec) * nrhs;
  if (prec == QDD_F16) b += sites * 4 * nrhs;  // per-site FP32 scales after the values
  return b;
}

qdd_status qdd_pack_field(qdd_ctx* x, qdd_prec prec, int nrhs, int even_only, const double* canon, void* field) {
  if (!x || !canon || !field || nrhs < 1 || nrhs > x->cfg.max_nrhs || prec < QDD_F64 || prec > QDD_F16) {
    if (x) x->fail("qdd_pack_field: invalid arguments");
    return QDD_EINVAL;
  }
  PackedView pv = x->packed(prec, nrhs, even_only, field);
  switch (prec) {
    case QDD_F64: HCK(x, launch_pack_spinor<double>(x->G, canon, pv.f64, nrhs, even_only, pv.poff, pv.spoff, x->st)); break;
    case QDD_F32: HCK(x, launch_pack_spinor<float>(x->G, canon, pv.f32, nrhs, even_only, pv.poff, pv.spoff, x->st)); break;
    default: HCK(x, launch_pack_spinor<__half>(x->G, canon, pv.f16, nrhs, even_only, pv.poff, pv.spoff, x->st)); break;
  }
  return QDD_OK;
}

qdd_status qdd_unpack_field(qdd_ctx* x, qdd_prec prec, int nrhs, int even_only, const void* field, double* canon) {
  if (!x || !canon || !field || nrhs < 1 || nrhs > x->cfg.max_nrhs || prec < QDD_F64 || prec > QDD_F16) {
    if (x) x->fail("qdd_unpack_field: invalid arguments");
    return QDD_EINVAL;
  }
  PackedView pv = x->packed(prec, nrhs, even_only, (void*)field);
  switch (prec) {
    case QDD_F64: HCK(x, launch_unpack_spinor<double>(x->G, pv.f64, canon, nrhs, even_only, pv.poff, pv.spoff, x->st)); break;
    case QDD_F32: HCK(x, launch_unpack_spinor<float>(x->G, pv.f32, canon, nrhs, even_only, pv.poff, pv.spoff, x->st)); break;
    default: HCK(x, launch_unpack_spinor<__half>(x->G, pv.f16, canon, nrhs, even_only, pv.poff, pv.spoff, x->st)); break;
  }
  return QDD_OK;
}

qdd_status qdd_dw_hat(qdd_ctx* x, qdd_prec prec, int nrhs, const void* in, void* out) {
  if (!x || !in || !out || nrhs < 1 || nrhs > x->cfg.max_nrhs || prec < QDD_F64 || prec > QDD_F16) {
    if (x) x->fail("qdd_dw_hat: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_dw_hat before qdd_set_params"); return QDD_ESTATE; }
  HCK(x, x->dhat(prec, nrhs, (void*)in, out));
  return QDD_OK;
}

qdd_status qdd_dw(qdd_ctx* x, qdd_prec prec, int nrhs, const void* in, void* out) {
  if (!x || !in || !out || nrhs < 1 || nrhs > x->cfg.max_nrhs || prec < QDD_F64 || prec > QDD_F16) {
    if (x) x->fail("qdd_dw: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_dw before qdd_set_params"); return QDD_ESTATE; }
  HCK(x, x->dw(prec, nrhs, (void*)in, out));
  return QDD_OK;
}

qdd_status qdd_dw_masses(qdd_ctx* x, qdd_prec prec, int nrhs, const double* kappas, const void* in, void* out) {
  if (!x || !in || !out || !kappas || nrhs < 1 || nrhs > x->cfg.max_nrhs || nrhs > kMaxShift || prec < QDD_F64 ||
      prec > QDD_F16) {
    if (x) x->fail("qdd_dw_masses: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_dw_masses before qdd_set_params"); return QDD_ESTATE; }
  x->dw_shift_host.assign(nrhs, 0.0);
  for (int r = 0; r < nrhs; ++r) {
    if (!(kappas[r] > 0.0)) { x->fail("qdd_dw_masses: kappa must be positive"); return QDD_EINVAL; }
    x->dw_shift_host[r] = 0.5 / kappas[r] - 0.5 / x->kappa;
  }
  double* sh = x->ptr<double>(x->lo.dw_shift);
  HCK(x, hipMemcpyAsync(sh, x->dw_shift_host.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, x->st));
  HCK(x, hipStreamSynchronize(x->st));  // the host copy of the shifts may change with the next call
  PackedView a = x->packed(prec, nrhs, 0, (void*)in), b = x->packed(prec, nrhs, 0, out);
  const LaunchCfg& c = x->launch[1][prec];
  switch (prec) {
    case QDD_F64: HCK(x, launch_dw<double>(x->G, x->op<double>(), a.f64, b.f64, a.poff, a.spoff, nrhs, c, x->st, sh)); break;
    case QDD_F32: HCK(x, launch_dw<float>(x->G, x->op<float>(), a.f32, b.f32, a.poff, a.spoff, nrhs, c, x->st, sh)); break;
    default: HCK(x, launch_dw<__half>(x->G, x->op<__half>(), a.f16, b.f16, a.poff, a.spoff, nrhs, c, x->st, sh)); break;
  }
  return QDD_OK;
}

qdd_status qdd_set_launch(qdd_ctx* x, int kernel, qdd_prec prec, int block, int nr, int xcd, int sb) {
  if (x && kernel == 2) {
    // Schwarz half-sweep kernel variant (nr), FP32 / FP16 storage only
    if (!sap_variant_ok(prec, nr) || block != 0 || xcd != 0 || sb != 0) {
      x->fail("qdd_set_launch: Schwarz variant must be 1..3 (FP32), 1..4 (FP16), other fields 0");
      return QDD_EINVAL;
    }
    x->sap_variant[prec] = nr;
    return QDD_OK;
  }
  // Dhat (not staged): + 64 walks pass B backwards
  const int xb = kernel == 0 && nr != 0 && xcd >= 64 ? xcd - 64 : xcd;
  bool ok = x && kernel >= 0 && kernel <= 1 && prec >= QDD_F64 && prec <= QDD_F16 && block >= 64 && block <= 256 &&
            (block & 63) == 0 && (nr == 0 || nr == 1 || nr == 2 || nr == 4) && xb >= 0 &&
            (xb <= (kernel == 0 && nr == 1 ? 31 : 3) || (kernel == 0 && xb >= 32 && xb <= 63 && dhat_vec_ok(prec, nr))) &&
            (sb == 0 || (sb >= 1 && sb <= block && block % sb == 0));
  // staged variant (nr = 0): Dhat only, and the tile's links + clover must fit the LDS budget
  if (ok && nr == 0) ok = kernel == 0 && staged_lds_bytes(prec, sb > 0 ? sb : block) <= kStagedLdsMax;
  if (!ok) {
    if (x) x->fail("qdd_set_launch: invalid arguments");
    return QDD_EINVAL;
  }
  x->launch[kernel][prec] = LaunchCfg{block, nr, xcd, sb == block ? 0 : sb};
  return QDD_OK;
}

qdd_status qdd_get_launch(const qdd_ctx* x, int kernel, qdd_prec prec, int* block, int* nr, int* xcd, int* sb) {
  if (!x || kernel < 0 || kernel > 2 || prec < QDD_F64 || prec > QDD_F16) return QDD_EINVAL;
  if (kernel == 2) {
    if (block) *block = 0;
    if (nr) *nr = prec == QDD_F64 ? 0 : (x->sap_variant[prec] ? x->sap_variant[prec] : sap_default_variant(prec));
    if (xcd) *xcd = 0;
    if (sb) *sb = 0;
    return QDD_OK;
  }
  const LaunchCfg& c = x->launch[kernel][prec];
  if (block) *block = c.block;
  if (nr) *nr = c.nr;
  if (xcd) *xcd = c.xcd;
  if (sb) *sb = c.sb > 0 ? c.sb : c.block;
  return QDD_OK;
}

qdd_status qdd_dw_hat_timed(qdd_ctx* x, qdd_prec prec, int nrhs, const void* in, void* out, int reps, float* ms_a,
                            float* ms_b) {
  if (!x || !in || !out || nrhs < 1 || nrhs > x->cfg.max_nrhs || prec < QDD_F64 || prec > QDD_F16 || reps < 1) {
    if (x) x->fail("qdd_dw_hat_timed: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_dw_hat_timed before qdd_set_params"); return QDD_ESTATE; }
  hipEvent_t e0, e1, e2;
  HCK(x, hipEventCreate(&e0));
  HCK(x, hipEventCreate(&e1));
  HCK(x, hipEventCreate(&e2));
  float ta = 0, tb = 0;
  hipError_t err = hipSuccess;
  for (int r = 0; r < reps && err == hipSuccess; ++r) {
    err = hipEventRecord(e0, x->st);
    if (err == hipSuccess) err = x->dhat(prec, nrhs, (void*)in, out, e1);
    if (err == hipSuccess) err = hipEventRecord(e2, x->st);
    if (err == hipSuccess) err = hipEventSynchronize(e2);
    float a = 0, b = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&a, e0, e1);
    if (err == hipSuccess) err = hipEventElapsedTime(&b, e1, e2);
    ta += a;
    tb += b;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipEventDestroy(e2);
  HCK(x, err);
  if (ms_a) *ms_a = ta / reps;
  if (ms_b) *ms_b = tb / reps;
  return QDD_OK;
}

qdd_status qdd_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || (bytes & 15)) return QDD_EINVAL;
  if (launch_copy(dst, src, bytes, (hipStream_t)stream) != hipSuccess) return QDD_EHIP;
  return QDD_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ ctx methods
std::string& qdd_ctx::last_global() {
  static thread_local std::string s;
  return s;
}

PackedView qdd_ctx::packed(qdd_prec prec, int nrhs, int even_only, void* field) const {
  PackedView v;
  int64_t n = G.Vh;
  int64_t sites = n * (even_only ? 1 : 2);
  int64_t rs = sites * 12;
  v.poff = 12 * n;  // parity offset within one rhs (elements)
  v.spoff = n;      // parity offset of the scales
  char* b = (char*)field;
  float* sc = (float*)(b + (size_t)rs * nrhs * 4);
  if (even_only && nrhs > 1) {
    // batches of even-site fields (the Dhat operands): interleaved layout
    // [12][Vh][nrhs], scales [Vh][nrhs]
    const int R = nrhs;
    v.f64 = FieldV<double>{(double2*)b, nullptr, 1, 1, (int)(n * R), R, R};
    v.f32 = FieldV<float>{(float2*)b, nullptr, 1, 1, (int)(n * R), R, R};
    v.f16 = FieldV<__half>{(__half2*)b, sc, 1, 1, (int)(n * R), R, R};
    return v;
  }
  v.f64 = FieldV<double>{(double2*)b, nullptr, rs, sites, (int)n};
  v.f32 = FieldV<float>{(float2*)b, nullptr, rs, sites, (int)n};
  v.f16 = FieldV<__half>{(__half2*)b, sc, rs, sites, (int)n};
  return v;
}

size_t qdd_ctx::dhat_tmp_bytes(qdd_prec prec, int nrhs, size_t* scale_off) const {
  // values [12][Vh][nrhs] (or [12][Vh] for one rhs), then the FP16 scales at a
  // 256-byte aligned offset
  const size_t vals = (size_t)nrhs * 12 * G.Vh * (prec == QDD_F64 ? 16 : prec == QDD_F32 ? 8 : 4);
  const size_t so = (vals + 255) & ~size_t(255);
  if (scale_off) *scale_off = so;
  return prec == QDD_F16 ? so + (size_t)nrhs * G.Vh * 4 : vals;
}

hipError_t qdd_ctx::dhat(qdd_prec prec, int nrhs, void* in, void* out, hipEvent_t mid, void* tmp) {
  PackedView a = packed(prec, nrhs, 1, in), b = packed(prec, nrhs, 1, out);
  int64_t n = G.Vh;
  const LaunchCfg& c = launch[0][prec];
  // the odd-site intermediate in the layout of the operands: in the workspace,
  // or in the buffer the caller names (dhat_tmp_bytes bytes)
  char* tv = tmp ? (char*)tmp : ptr<char>(lo.tmp_o);
  size_t so = 0;
  dhat_tmp_bytes(prec, nrhs, &so);
  float* ts = tmp ? (float*)(tv + so) : ptr<float>(lo.tmp_o_scale);
  const bool il = nrhs > 1;
  const int64_t trs = il ? 1 : 12 * n, tsrs = il ? 1 : n;
  const int tn = il ? (int)(n * nrhs) : (int)n, tss = il ? nrhs : 1;
  switch (prec) {
    case QDD_F64: {
      FieldV<double> t{(double2*)tv, nullptr, trs, tsrs, tn, tss, tss};
      return launch_dhat<double>(G, op<double>(), a.f64, t, b.f64, nrhs, c, st, 3, mid);
    }
    case QDD_F32: {
      FieldV<float> t{(float2*)tv, nullptr, trs, tsrs, tn, tss, tss};
      return launch_dhat<float>(G, op<float>(), a.f32, t, b.f32, nrhs, c, st, 3, mid);
    }
    default: {
      FieldV<__half> t{(__half2*)tv, ts, trs, tsrs, tn, tss, tss};
      return launch_dhat<__half>(G, op<__half>(), a.f16, t, b.f16, nrhs, c, st, 3, mid);
    }
  }
}

hipError_t qdd_ctx::dw(qdd_prec prec, int nrhs, void* in, void* out, const double* ce) {
  PackedView a = packed(prec, nrhs, 0, in), b = packed(prec, nrhs, 0, out);
  const LaunchCfg& c = launch[1][prec];
  switch (prec) {
    case QDD_F64: return launch_dw<double>(G, op<double>(), a.f64, b.f64, a.poff, a.spoff, nrhs, c, st, nullptr, ce);
    case QDD_F32: return launch_dw<float>(G, op<float>(), a.f32, b.f32, a.poff, a.spoff, nrhs, c, st, nullptr, ce);
    default: return launch_dw<__half>(G, op<__half>(), a.f16, b.f16, a.poff, a.spoff, nrhs, c, st, nullptr, ce);
  }
}

// ------------------------------------------------------------ mass preconditioning
qdd_status qdd_clover_logdet(qdd_ctx* x, double* logdet_even, double* logdet_odd) {
  if (!x || !logdet_even || !logdet_odd) {
    if (x) x->fail("qdd_clover_logdet: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_clover_logdet before qdd_set_params"); return QDD_ESTATE; }
  const int nb = clover_logdet_blocks(x->G.Vh);
  double* part = x->ptr<double>(x->lo.part);
  std::vector<double> h(2 * (size_t)nb);
  HCK(x, launch_clover_logdet(x->G, x->op<double>().A, part, x->st));
  HCK(x, hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, x->st));
  HCK(x, hipStreamSynchronize(x->st));
  double s[2] = {0.0, 0.0};
  for (int p = 0; p < 2; ++p)
    for (int b = 0; b < nb; ++b) s[p] += h[(size_t)p * nb + b];  // fixed order: deterministic
  if (!std::isfinite(s[0]) || !std::isfinite(s[1])) {
    x->fail("qdd_clover_logdet: a clover block is not positive definite");
    return QDD_ESINGULAR;
  }
  *logdet_even = s[0];
  *logdet_odd = s[1];
  return QDD_OK;
}

qdd_status qdd_apply_w(qdd_ctx* x, int nrhs, double dm, const void* in, void* out) {
  if (!x || !in || !out || in == out || nrhs < 1 || nrhs > x->cfg.max_nrhs || !std::isfinite(dm)) {
    if (x) x->fail("qdd_apply_w: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_apply_w before qdd_set_params"); return QDD_ESTATE; }
  HCK(x, x->dhat(QDD_F64, nrhs, (void*)in, out));
  PackedView vi = x->packed(QDD_F64, nrhs, 1, (void*)in), vo = x->packed(QDD_F64, nrhs, 1, out);
  HCK(x, launch_apply_w_finish(x->G, vi.f64, vo.f64, x->op<double>().Ainv, nrhs, dm, x->st));
  return QDD_OK;
}
