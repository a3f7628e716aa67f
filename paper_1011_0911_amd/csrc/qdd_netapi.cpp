// Learned preconditioner stage, host side: weights, forward pass, loss and
// gradient, Adam training steps, and the network stage of the two-level
// preconditioner (v = C r + N(r1) + M_sap(r2), r1 = r - D C r,
// r2 = r1 - D N(r1); the network output is dropped per right-hand side if it
// does not reduce the residual, |r2| > |r1|, or is not finite).
#include "qdd_dfl.h"
#include "qdd_net.h"

#include <cmath>
#include <vector>

using namespace qdd;

static int net_nl(const qdd_ctx* x) { return x->cfg.net_nl; }
static int64_t layer_nw(const qdd_ctx* x, int l) { return (int64_t)9 * x->cfg.net_ch[l] * x->cfg.net_ch[l + 1] * 16; }
static int64_t layer_off(const qdd_ctx* x, int l) {
  int64_t o = 0;
  for (int k = 0; k < l; ++k) o += layer_nw(x, k);
  return o;
}
static int net_maxch(const qdd_ctx* x) {
  int m = 1;
  for (int l = 0; l <= x->cfg.net_nl; ++l) m = std::max(m, x->cfg.net_ch[l]);
  return m;
}
// scratch channel fields of the forward layers: the two gradient levels (free
// during a forward pass); the backward layers run with none
static int fwd_scratch_ch(const qdd_ctx* x) { return 2 * net_maxch(x); }
// matrix-core operands of layer l, forward (adj = false) or backward (adjoint weights)
static uint16_t* layer_wmx(const qdd_ctx* x, int l, bool adj) {
  size_t o = 0;
  for (int k = 0; k < l; ++k)
    o += adj ? net_wmx_elems(x->cfg.net_ch[k + 1], x->cfg.net_ch[k], 0)
             : net_wmx_elems(x->cfg.net_ch[k], x->cfg.net_ch[k + 1], fwd_scratch_ch(x));
  return x->ptr<uint16_t>(adj ? x->lo.net_wmxa : x->lo.net_wmx) + o;
}
// activation level k (k = 0..nl), gradient buffers nl+1, nl+2
static float2* net_level(const qdd_ctx* x, int k) {
  int64_t cs = (int64_t)24 * x->G.Vh;
  return x->ptr<float2>(x->lo.net_act) + (int64_t)k * net_maxch(x) * cs;
}
static LinkV<float> links32(const qdd_ctx* x) { return x->op<float>().U; }

static qdd_status net_check(qdd_ctx* x, bool need_weights) {
  if (!x->cfg.use_net) { x->fail("network calls need use_net = 1 in the configuration"); return QDD_EINVAL; }
  if (!x->have_gauge) { x->fail("network call before qdd_set_gauge"); return QDD_ESTATE; }
  if (need_weights && !x->have_net) { x->fail("network call before qdd_net_set_weights"); return QDD_ESTATE; }
  return QDD_OK;
}

// forward: act[0] must hold the input; act[nl] receives the output; terms: BF16
// terms per activation (3 in training, the configured net_terms when applied)
static qdd_status net_forward_levels(qdd_ctx* x, int terms) {
  int64_t cs = (int64_t)24 * x->G.Vh;
  for (int l = 0; l < net_nl(x); ++l)
    HCK(x, launch_net_layer(x->G, links32(x), layer_wmx(x, l, false), x->cfg.net_ch[l], x->cfg.net_ch[l + 1],
                            net_level(x, l), net_level(x, l + 1), cs, net_level(x, net_nl(x) + 1), fwd_scratch_ch(x),
                            terms, x->st));
  return QDD_OK;
}

// recompute the BF16 compute copy and the adjoint (backward) weights
static qdd_status net_refresh_weights(qdd_ctx* x) {
  int nw = (int)x->lo.net_nw;
  uint32_t *wb = x->ptr<uint32_t>(x->lo.net_wb), *wa = x->ptr<uint32_t>(x->lo.net_wadj);
  HCK(x, launch_net_to_bf16(x->ptr<float2>(x->lo.net_w), wb, nw, x->st));
  for (int l = 0; l < net_nl(x); ++l) {
    const int cin = x->cfg.net_ch[l], cout = x->cfg.net_ch[l + 1];
    HCK(x, launch_net_adjoint(wb + layer_off(x, l), cin, cout, wa + layer_off(x, l), x->st));
    HCK(x, launch_net_wmx(wb + layer_off(x, l), cin, cout, fwd_scratch_ch(x), layer_wmx(x, l, false), x->st));
    HCK(x, launch_net_wmx(wa + layer_off(x, l), cout, cin, 0, layer_wmx(x, l, true), x->st));
  }
  return QDD_OK;
}

static double norm2_f(qdd_ctx* x, const float2* v, int64_t n, qdd_status* st) {
  double* part = x->ptr<double>(x->lo.net_loss);
  const int nb = 256;
  std::vector<double> h(nb);
  *st = QDD_OK;
  if (launch_norm2_f(v, n, part, nb, x->st) != hipSuccess ||
      hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, x->st) != hipSuccess ||
      hipStreamSynchronize(x->st) != hipSuccess) {
    x->fail("HIP error in norm");
    *st = QDD_EHIP;
    return 0;
  }
  double s = 0;
  for (double v2 : h) s += v2;
  return s;
}

// Loss over nb pairs (FP32 packed full fields, pair stride ps) and its gradient
// accumulated into net_grad (zeroed first).  loss = sum |N(r/|r|) - e/|r||^2 / Z.
static qdd_status net_loss_grad_packed(qdd_ctx* x, int nb, const float2* r, const float2* e, int64_t ps,
                                       double* loss) {
  int64_t cs = (int64_t)24 * x->G.Vh;
  int nl = net_nl(x);
  qdd_status st;
  std::vector<double> rn(nb);
  double Z = 0;
  for (int i = 0; i < nb; ++i) {
    rn[i] = std::sqrt(norm2_f(x, r + i * ps, cs, &st));
    if (st != QDD_OK) return st;
    double en = norm2_f(x, e + i * ps, cs, &st);
    if (st != QDD_OK) return st;
    Z += rn[i] > 0 ? en / (rn[i] * rn[i]) : 0.0;
  }
  if (!(Z > 0)) { x->fail("training pairs with zero error"); return QDD_EINVAL; }
  float2* grad = x->ptr<float2>(x->lo.net_grad);
  HCK(x, hipMemsetAsync(grad, 0, x->lo.net_nw * sizeof(float2), x->st));
  double* lp = x->ptr<double>(x->lo.net_loss) + 256;
  const int nlb = 256;
  double total = 0;
  std::vector<double> h(nlb);
  for (int i = 0; i < nb; ++i) {
    HCK(x, launch_scale_to_f<float2>(net_level(x, 0), r + i * ps, 1.0 / rn[i], cs, x->st));
    qdd_status s = net_forward_levels(x, 3);
    if (s != QDD_OK) return s;
    float2 *g0 = net_level(x, nl + 1), *g1 = net_level(x, nl + 2);
    HCK(x, launch_net_out_grad(net_level(x, nl), e + i * ps, (float)(1.0 / rn[i]), (float)(1.0 / Z), g0, cs, lp, nlb,
                               x->st));
    HCK(x, hipMemcpyAsync(h.data(), lp, nlb * sizeof(double), hipMemcpyDeviceToHost, x->st));
    for (int l = nl - 1; l >= 0; --l) {
      int cin = x->cfg.net_ch[l], cout = x->cfg.net_ch[l + 1];
      HCK(x, launch_net_wgrad(x->G, links32(x), cin, cout, net_level(x, l), g0, cs, x->ptr<float>(x->lo.net_gpart),
                              x->lo.net_gpart_floats, grad + layer_off(x, l), x->st));
      if (l > 0) {
        HCK(x, launch_net_layer(x->G, links32(x), layer_wmx(x, l, true), cout, cin, g0, g1, cs, nullptr, 0, 3, x->st));
        std::swap(g0, g1);
      }
    }
    HCK(x, hipStreamSynchronize(x->st));
    for (double v : h) total += v;
  }
  if (loss) *loss = total;
  return QDD_OK;
}

// ------------------------------------------------------------------ C entry points
extern "C" qdd_status qdd_net_num_weights(const qdd_ctx* x, int64_t* n) {
  if (!x || !n) return QDD_EINVAL;
  *n = x->cfg.use_net ? (int64_t)x->lo.net_nw : 0;
  return QDD_OK;
}

extern "C" qdd_status qdd_net_set_weights(qdd_ctx* x, const float* w) {
  if (!x || !w) return QDD_EINVAL;
  qdd_status s = net_check(x, false);
  if (s != QDD_OK) return s;
  HCK(x, hipMemcpyAsync(x->ptr<float2>(x->lo.net_w), w, x->lo.net_nw * sizeof(float2), hipMemcpyDeviceToDevice,
                        x->st));
  HCK(x, hipMemsetAsync(x->ptr<float4>(x->lo.net_adam), 0, x->lo.net_nw * sizeof(float4), x->st));
  s = net_refresh_weights(x);
  if (s != QDD_OK) return s;
  HCK(x, hipStreamSynchronize(x->st));
  x->net_step = 0;
  x->have_net = true;
  return QDD_OK;
}

extern "C" qdd_status qdd_net_set_terms(qdd_ctx* x, int terms) {
  if (!x) return QDD_EINVAL;
  qdd_status s = net_check(x, false);
  if (s != QDD_OK) return s;
  if (terms < 1 || terms > 3) { x->fail("qdd_net_set_terms: terms must be 1, 2 or 3"); return QDD_EINVAL; }
  x->cfg.net_terms = terms;
  return QDD_OK;
}

extern "C" qdd_status qdd_net_set_calls(qdd_ctx* x, int calls) {
  if (!x) return QDD_EINVAL;
  qdd_status s = net_check(x, false);
  if (s != QDD_OK) return s;
  if (calls < 0) { x->fail("qdd_net_set_calls: calls must be >= 0"); return QDD_EINVAL; }
  x->net_calls = calls;
  return QDD_OK;
}

extern "C" qdd_status qdd_net_get_weights(qdd_ctx* x, float* w) {
  if (!x || !w) return QDD_EINVAL;
  qdd_status s = net_check(x, true);
  if (s != QDD_OK) return s;
  HCK(x, hipMemcpyAsync(w, x->ptr<float2>(x->lo.net_w), x->lo.net_nw * sizeof(float2), hipMemcpyDeviceToDevice,
                        x->st));
  HCK(x, hipStreamSynchronize(x->st));
  return QDD_OK;
}

extern "C" qdd_status qdd_net_forward(qdd_ctx* x, const double* in_c, double* out_c) {
  if (!x || !in_c || !out_c) return QDD_EINVAL;
  qdd_status s = net_check(x, true);
  if (s != QDD_OK) return s;
  PackedView pi = x->packed(QDD_F32, 1, 0, net_level(x, 0));
  HCK(x, launch_pack_spinor<float>(x->G, in_c, pi.f32, 1, 0, pi.poff, pi.spoff, x->st));
  s = net_forward_levels(x, x->cfg.net_terms);
  if (s != QDD_OK) return s;
  PackedView po = x->packed(QDD_F32, 1, 0, net_level(x, net_nl(x)));
  HCK(x, launch_unpack_spinor<float>(x->G, po.f32, out_c, 1, 0, po.poff, po.spoff, x->st));
  HCK(x, hipStreamSynchronize(x->st));
  return QDD_OK;
}

// pairs in canonical complex128 (device); grad (device, FP32 complex) may be NULL
extern "C" qdd_status qdd_net_loss_grad(qdd_ctx* x, int nb, const double* r_c, const double* e_c, double* loss,
                                        float* grad) {
  if (!x || nb < 1 || !r_c || !e_c) return QDD_EINVAL;
  qdd_status s = net_check(x, true);
  if (s != QDD_OK) return s;
  // stage the pairs one at a time through FP32 buffers: the whole batch is
  // converted into the training buffer region of the workspace
  int64_t cs = (int64_t)24 * x->G.Vh, V12 = (int64_t)12 * x->G.V;
  if ((int64_t)2 * nb * cs * (int64_t)sizeof(float2) > (int64_t)x->lo.net_pairs_bytes) {
    x->fail("qdd_net_loss_grad: at most %lld pairs fit the workspace",
            (long long)(x->lo.net_pairs_bytes / (2 * cs * sizeof(float2))));
    return QDD_EINVAL;
  }
  float2* rp = x->ptr<float2>(x->lo.net_pairs);
  float2* ep = rp + nb * cs;
  for (int i = 0; i < nb; ++i) {
    PackedView a = x->packed(QDD_F32, 1, 0, rp + i * cs), b = x->packed(QDD_F32, 1, 0, ep + i * cs);
    HCK(x, launch_pack_spinor<float>(x->G, r_c + 2 * i * V12, a.f32, 1, 0, a.poff, a.spoff, x->st));
    HCK(x, launch_pack_spinor<float>(x->G, e_c + 2 * i * V12, b.f32, 1, 0, b.poff, b.spoff, x->st));
  }
  s = net_loss_grad_packed(x, nb, rp, ep, cs, loss);
  if (s != QDD_OK) return s;
  if (grad)
    HCK(x, hipMemcpyAsync(grad, x->ptr<float2>(x->lo.net_grad), x->lo.net_nw * sizeof(float2),
                          hipMemcpyDeviceToDevice, x->st));
  HCK(x, hipStreamSynchronize(x->st));
  return QDD_OK;
}

// one Adam step on a mini-batch of nb pairs given as packed FP32 full fields
// (qdd_field_bytes(F32, 1, 0) bytes each, consecutive)
extern "C" qdd_status qdd_net_train_step(qdd_ctx* x, int nb, const void* r, const void* e, float lr, double* loss) {
  if (!x || nb < 1 || !r || !e || !(lr > 0)) return QDD_EINVAL;
  qdd_status s = net_check(x, true);
  if (s != QDD_OK) return s;
  int64_t cs = (int64_t)24 * x->G.Vh;
  s = net_loss_grad_packed(x, nb, (const float2*)r, (const float2*)e, cs, loss);
  if (s != QDD_OK) return s;
  x->net_step++;
  HCK(x, launch_net_adam(x->ptr<float2>(x->lo.net_w), x->ptr<float2>(x->lo.net_grad), x->ptr<float4>(x->lo.net_adam),
                         (int)x->lo.net_nw, lr, x->net_step, x->st));
  s = net_refresh_weights(x);
  if (s != QDD_OK) return s;
  HCK(x, hipStreamSynchronize(x->st));
  return QDD_OK;
}

// ------------------------------------------------------------------ preconditioner stage
// r1: FP64 deflation-corrected residuals (nrhs fields, stride 24 Vh).  Writes
// vn = N(r1) (FP32, zero where rejected) and r2 = r1 - D vn (FP64, = r1 where
// rejected); tbuf: FP32 scratch of nrhs fields.  fb[j] = 1 where the network
// output was rejected.
qdd_status net_stage(qdd_ctx* x, int nrhs, const double2* r1, float2* vn, double2* r2, float2* tbuf,
                     std::vector<int>& fb) {
  int64_t cs = (int64_t)24 * x->G.Vh;
  int nl = net_nl(x);
  for (int j = 0; j < nrhs; ++j) {
    HCK(x, launch_scale_to_f<double2>(net_level(x, 0), r1 + j * cs, 1.0, cs, x->st));
    qdd_status s = net_forward_levels(x, x->cfg.net_terms);
    if (s != QDD_OK) return s;
    HCK(x, hipMemcpyAsync(vn + j * cs, net_level(x, nl), cs * sizeof(float2), hipMemcpyDeviceToDevice, x->st));
  }
  HCK(x, x->dw(QDD_F32, nrhs, vn, tbuf));
  HCK(x, hipMemcpyAsync(r2, r1, (size_t)nrhs * cs * sizeof(double2), hipMemcpyDeviceToDevice, x->st));
  HCK(x, launch_sub_f(r2, tbuf, (int64_t)nrhs * cs, x->st));
  double2 *part = x->ptr<double2>(x->lo.cpart), *nrm = x->ptr<double2>(x->lo.crn2);
  std::vector<double2> n1(nrhs), n2(nrhs);
  // both norms with one wait: the second reduction reuses part and nrm after the
  // first copy in stream order
  HCK(x, launch_dots<double2>(r1, 0, cs, 1, r1, cs, cs, nrhs, part, nrm, x->st));
  HCK(x, hipMemcpyAsync(n1.data(), nrm, nrhs * sizeof(double2), hipMemcpyDeviceToHost, x->st));
  HCK(x, launch_dots<double2>(r2, 0, cs, 1, r2, cs, cs, nrhs, part, nrm, x->st));
  HCK(x, hipMemcpyAsync(n2.data(), nrm, nrhs * sizeof(double2), hipMemcpyDeviceToHost, x->st));
  HCK(x, hipStreamSynchronize(x->st));
  fb.assign(nrhs, 0);
  for (int j = 0; j < nrhs; ++j) {
    if (std::isfinite(n2[j].x) && n2[j].x <= n1[j].x) continue;
    fb[j] = 1;
    HCK(x, hipMemcpyAsync(r2 + j * cs, r1 + j * cs, cs * sizeof(double2), hipMemcpyDeviceToDevice, x->st));
    HCK(x, hipMemsetAsync(vn + j * cs, 0, cs * sizeof(float2), x->st));
  }
  return QDD_OK;
}
