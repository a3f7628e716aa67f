// Oracle: the gauge-covariant parallel-transport convolution network used as an
// extra preconditioner stage (not in the paper; a reading of the learned stage
// this library adds).  Every layer is linear:
//   out_c(x) = sum_{c'} sum_{d} W[d][c][c'] (T_d in_{c'})(x)
// with d = 0 the identity, d = 1+2mu the forward transport
//   (T_{+mu} psi)(x) = s U_mu(x) psi(x+mu)
// and d = 2+2mu the backward transport
//   (T_{-mu} psi)(x) = s U_mu(x-mu)^dag psi(x-mu),
// s the fermion boundary sign of the hop, and W[d][c][c'] a complex 4x4 matrix
// acting on spin.  TEST INFRASTRUCTURE ONLY (see orc_core.h).
#include "orc_core.h"
#include <cstring>

namespace orc {

// (T_d psi)(x) for one site; psi is a single-channel field [V][12]
static void transport(const Geom& g, const cplx* U, const cplx* psi, int64_t x, int d, cplx* out) {
  if (d == 0) {
    for (int i = 0; i < 12; ++i) out[i] = psi[x * 12 + i];
    return;
  }
  int mu = (d - 1) / 2, dir = (d - 1) % 2;
  int64_t y = dir == 0 ? g.up(x, mu) : g.dn(x, mu);
  double s = dir == 0 ? g.sign_up(x, mu) : g.sign_up(y, mu);
  const cplx* u = dir == 0 ? link(U, x, mu) : link(U, y, mu);
  for (int sp = 0; sp < 4; ++sp)
    for (int a = 0; a < 3; ++a) {
      cplx acc = 0;
      for (int b = 0; b < 3; ++b)
        acc += (dir == 0 ? u[a * 3 + b] : std::conj(u[b * 3 + a])) * psi[y * 12 + sp * 3 + b];
      out[sp * 3 + a] = s * acc;
    }
}

// adjoint of T_d: T_{+mu}^dag = T_{-mu}, T_0^dag = T_0
static int adjoint_path(int d) { return d == 0 ? 0 : ((d - 1) % 2 == 0 ? d + 1 : d - 1); }

// One output site of a layer: out_c(x) for every output channel c.
// weights of layer: W[((d*cout + c)*cin + c')*16 + s*4 + s']
static void layer_site(const Geom& g, const cplx* U, int cin, int cout, const cplx* W, const cplx* in, int64_t x,
                       cplx* out) {
  int64_t V = g.V;
  std::vector<cplx> acc(cout * 12, 0.0);
  cplx t[12];
  for (int cp = 0; cp < cin; ++cp)
    for (int d = 0; d < 9; ++d) {
      transport(g, U, in + cp * V * 12, x, d, t);
      for (int c = 0; c < cout; ++c) {
        const cplx* w = W + ((d * cout + c) * cin + cp) * 16;
        for (int s = 0; s < 4; ++s)
          for (int a = 0; a < 3; ++a) {
            cplx z = 0;
            for (int sp = 0; sp < 4; ++sp) z += w[s * 4 + sp] * t[sp * 3 + a];
            acc[c * 12 + s * 3 + a] += z;
          }
      }
    }
  for (int c = 0; c < cout; ++c)
    for (int i = 0; i < 12; ++i) out[(c * V + x) * 12 + i] = acc[c * 12 + i];
}

void net_layer_forward(const Geom& g, const cplx* U, int cin, int cout, const cplx* W, const cplx* in, cplx* out) {
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < g.V; ++x) layer_site(g, U, cin, cout, W, in, x, out);
}

// Backward of one layer.  gy: complex gradient dl/dRe(y) + i dl/dIm(y) of the
// layer output; returns gx = sum_d T_d^dag W_d^dag gy and accumulates
// gW[d][c][c'][s][s'] += sum_{x,a} gy_c[s,a](x) conj((T_d in_{c'})[s',a](x)).
void net_layer_backward(const Geom& g, const cplx* U, int cin, int cout, const cplx* W, const cplx* in,
                        const cplx* gy, cplx* gx, cplx* gW) {
  int64_t V = g.V;
  // weight gradient: plain sum over sites (serial per weight block for determinism)
  std::vector<cplx> t(12);
  for (int d = 0; d < 9; ++d)
    for (int cp = 0; cp < cin; ++cp) {
      std::vector<cplx> part(cout * 16, 0.0);
      for (int64_t x = 0; x < V; ++x) {
        transport(g, U, in + cp * V * 12, x, d, t.data());
        for (int c = 0; c < cout; ++c)
          for (int s = 0; s < 4; ++s)
            for (int sp = 0; sp < 4; ++sp) {
              cplx z = 0;
              for (int a = 0; a < 3; ++a) z += gy[(c * V + x) * 12 + s * 3 + a] * std::conj(t[sp * 3 + a]);
              part[c * 16 + s * 4 + sp] += z;
            }
      }
      for (int c = 0; c < cout; ++c)
        for (int i = 0; i < 16; ++i) gW[((d * cout + c) * cin + cp) * 16 + i] += part[c * 16 + i];
    }
  // input gradient: u_{d,c'} = sum_c W_d[c][c']^dag gy_c, then gx_{c'} = sum_d T_d^dag u_{d,c'}
  std::vector<cplx> u((size_t)9 * cin * V * 12);
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < V; ++x)
    for (int d = 0; d < 9; ++d)
      for (int cp = 0; cp < cin; ++cp)
        for (int sp = 0; sp < 4; ++sp)
          for (int a = 0; a < 3; ++a) {
            cplx z = 0;
            for (int c = 0; c < cout; ++c) {
              const cplx* w = W + ((d * cout + c) * cin + cp) * 16;
              for (int s = 0; s < 4; ++s) z += std::conj(w[s * 4 + sp]) * gy[(c * V + x) * 12 + s * 3 + a];
            }
            u[((size_t)(d * cin + cp) * V + x) * 12 + sp * 3 + a] = z;
          }
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < V; ++x)
    for (int cp = 0; cp < cin; ++cp) {
      cplx acc[12] = {}, tt[12];
      for (int d = 0; d < 9; ++d) {
        transport(g, U, &u[(size_t)(d * cin + cp) * V * 12], x, adjoint_path(d), tt);
        for (int i = 0; i < 12; ++i) acc[i] += tt[i];
      }
      for (int i = 0; i < 12; ++i) gx[(cp * V + x) * 12 + i] = acc[i];
    }
}

static int64_t layer_wsize(int cin, int cout) { return (int64_t)9 * cout * cin * 16; }

// Whole network forward: channels ch[0] -> ch[1] -> ... -> ch[nl]
void net_forward(const Geom& g, const cplx* U, int nl, const int* ch, const cplx* W, const cplx* in, cplx* out) {
  std::vector<cplx> a(in, in + (size_t)ch[0] * g.V * 12), b;
  int64_t off = 0;
  for (int l = 0; l < nl; ++l) {
    b.assign((size_t)ch[l + 1] * g.V * 12, 0.0);
    net_layer_forward(g, U, ch[l], ch[l + 1], W + off, a.data(), b.data());
    off += layer_wsize(ch[l], ch[l + 1]);
    a.swap(b);
  }
  std::memcpy((void*)out, a.data(), sizeof(cplx) * a.size());
}

// The network output (one channel) at a list of sites only, for checks at sizes
// where the full forward pass is too slow: layer l is evaluated on the sites
// within nl - l hops of the listed ones (the only activations the output there
// depends on), with the per-site arithmetic of net_layer_forward.  out: [nsites][12].
void net_forward_on_sites(const Geom& g, const cplx* U, int nl, const int* ch, const cplx* W, const cplx* in,
                          const int64_t* sites, int nsites, cplx* out) {
  const int64_t V = g.V;
  // need[l]: sites where the activation of level l is needed
  std::vector<std::vector<uint8_t>> need(nl + 1, std::vector<uint8_t>(V, 0));
  for (int i = 0; i < nsites; ++i) need[nl][sites[i]] = 1;
  for (int l = nl - 1; l >= 1; --l)
    for (int64_t x = 0; x < V; ++x) {
      if (!need[l + 1][x]) continue;
      need[l][x] = 1;
      for (int mu = 0; mu < 4; ++mu) {
        need[l][g.up(x, mu)] = 1;
        need[l][g.dn(x, mu)] = 1;
      }
    }
  std::vector<cplx> a(in, in + (size_t)ch[0] * V * 12), b;
  int64_t off = 0;
  for (int l = 0; l < nl; ++l) {
    b.assign((size_t)ch[l + 1] * V * 12, 0.0);
    std::vector<int64_t> xs;
    for (int64_t x = 0; x < V; ++x)
      if (need[l + 1][x]) xs.push_back(x);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)xs.size(); ++k) layer_site(g, U, ch[l], ch[l + 1], W + off, a.data(), xs[k], b.data());
    off += layer_wsize(ch[l], ch[l + 1]);
    a.swap(b);
  }
  for (int i = 0; i < nsites; ++i)
    for (int k = 0; k < 12; ++k) out[i * 12 + k] = a[sites[i] * 12 + k];
}

// Loss l = sum_i |N(r_i/|r_i|) - e_i/|r_i||^2 / sum_i |e_i/|r_i||^2 over a batch of
// single-channel pairs, and its complex gradient with respect to all weights.
double net_loss_grad(const Geom& g, const cplx* U, int nl, const int* ch, const cplx* W, int nb, const cplx* r,
                     const cplx* e, cplx* grad) {
  int64_t V12 = g.V * 12;
  int64_t nw = 0;
  for (int l = 0; l < nl; ++l) nw += layer_wsize(ch[l], ch[l + 1]);
  if (grad) for (int64_t i = 0; i < nw; ++i) grad[i] = 0;
  std::vector<double> scale(nb);
  double Z = 0;
  for (int i = 0; i < nb; ++i) {
    scale[i] = 1.0 / std::sqrt(norm2(r + i * V12, V12));
    Z += norm2(e + i * V12, V12) * scale[i] * scale[i];
  }
  double loss = 0;
  for (int i = 0; i < nb; ++i) {
    std::vector<std::vector<cplx>> act(nl + 1);
    act[0].resize(V12);
    for (int64_t k = 0; k < V12; ++k) act[0][k] = r[i * V12 + k] * scale[i];
    int64_t off = 0;
    std::vector<int64_t> offs(nl);
    for (int l = 0; l < nl; ++l) {
      offs[l] = off;
      act[l + 1].assign((size_t)ch[l + 1] * V12, 0.0);
      net_layer_forward(g, U, ch[l], ch[l + 1], W + off, act[l].data(), act[l + 1].data());
      off += layer_wsize(ch[l], ch[l + 1]);
    }
    std::vector<cplx> gy(V12);
    for (int64_t k = 0; k < V12; ++k) {
      cplx diff = act[nl][k] - e[i * V12 + k] * scale[i];
      loss += std::norm(diff) / Z;
      gy[k] = 2.0 * diff / Z;
    }
    if (!grad) continue;
    for (int l = nl - 1; l >= 0; --l) {
      std::vector<cplx> gx((size_t)ch[l] * V12);
      net_layer_backward(g, U, ch[l], ch[l + 1], W + offs[l], act[l].data(), gy.data(), gx.data(), grad + offs[l]);
      gy.swap(gx);
    }
  }
  return loss;
}

}  // namespace orc
