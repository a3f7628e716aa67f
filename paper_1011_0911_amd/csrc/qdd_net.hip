// Gauge-covariant parallel-transport convolution network (the learned
// preconditioner stage this library adds inside flexible GCR).  Layer:
//   out_c(x) = sum_{c'} sum_{d=0..8} W[d][c][c'] (T_d in_{c'})(x)
// d = 0 identity, d = 1+2mu: (T psi)(x) = U_mu(x) psi(x+mu), d = 2+2mu:
// (T psi)(x) = U_mu(x-mu)^dag psi(x-mu) (boundary sign inside the stored links);
// W[d][c][c'] a complex 4x4 spin matrix.  Weights are used in BF16 (FP32 master
// copy for the optimiser), activations and accumulation in FP32.
//
// Because W acts on spin and T on colour, the input gradient of a layer,
//   gx_{c'} = sum_{c,d} T_d^dag W[d][c][c']^dag gy_c,
// is again a layer with weights W'[adj(d)][c'][c] = W[d][c][c']^dag (adj swaps
// +mu and -mu): the same kernel runs forward and backward.
#include "qdd_kernels.h"
#include "qdd_net.h"

#include <algorithm>

namespace qdd {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f_to_bf16(float f) {
  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

// Weight gradient on the matrix cores.  For each transport d,
//   dl/dW[d][c][c'][sa][sb] = sum_{x, a} gy_c(x)[sa, a] conj((T_d in_c')(x)[sb, a])
// is, in real form, the product P = G T over k = (site, colour): rows of G
// m = (c, sa, re/im) (8 cout), columns of T n = (c', sb, re/im) (8 cin); then
// Re = P[r][r] + P[i][i], Im = P[i][r] - P[r][i].  A workgroup (4 wavefronts)
// takes one d and a range of sites, stages 16 sites at a time into LDS (G as
// [m][k], the transported inputs T as [n][k]; the row stride of 52 words puts
// the 64 lanes of an operand read on distinct banks) and accumulates its share of the
// 16x16 output tiles with v_mfma_f32_16x16x4f32 (FP32 products, exact); the
// per-workgroup partial products are summed in a fixed order in FP64
// (k_net_wgrad_reduce), so the gradient is deterministic.
constexpr int kWgTileSites = 16;
constexpr int kWgLd = 52;  // LDS row stride (floats) of the [m][k] / [n][k] tiles, >= 3 kWgTileSites
// Site range r and transport d of workgroup b (nwx ranges x 9 transports).
// Workgroups go to the 8 XCDs round-robin (b mod 8), each with its own L2; the
// nine transports of one range go to consecutive workgroups of one XCD, so the
// range's output gradient and inputs come from HBM about once instead of nine
// times.  (Range-major order where nwx is not a multiple of 8.)
__device__ inline void wgrad_block(int b, int nwx, int& r, int& d) {
  if (nwx & 7) {
    r = b % nwx;
    d = b / nwx;
    return;
  }
  const int q = b >> 3;  // rank within the XCD
  d = q % 9;
  r = (q / 9) * 8 + (b & 7);
}
template <int TPW>
__global__ void __launch_bounds__(256) k_net_wgrad_mx(Geo g, LinkV<float> U, int cin, int cout, const float2* in,
                                                      const float2* gy, int64_t cs, int nwx, int sites_per_wg,
                                                      float* part) {
  extern __shared__ float wl[];
  const int M16 = 16 * ((8 * cout + 15) / 16), N16 = 16 * ((8 * cin + 15) / 16);
  float* gl = wl;                  // [M16][kWgLd]: G[m][k]
  float* tlw = wl + M16 * kWgLd;   // [N16][kWgLd]: T[n][k]
  int rg, d;
  wgrad_block(blockIdx.x, nwx, rg, d);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ntile = (M16 / 16) * (N16 / 16), ntn = N16 / 16;
  f4v acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = f4v{0.f, 0.f, 0.f, 0.f};
  const int s_begin = rg * sites_per_wg, s_end = min(g.V, s_begin + sites_per_wg);
  // staging roles: lane t < 16 cin stages the transported input (site t % 16,
  // channel t / 16); every lane stages up to 12 output-gradient elements.  The
  // loads of the next tile are issued before the matrix-core phase of the
  // current one.
  const bool has_t = (int)threadIdx.x < kWgTileSites * cin;
  const int t_sl = threadIdx.x % kWgTileSites, t_cp = threadIdx.x / kWgTileSites;
  const int ng = kWgTileSites * cout * 12;
  float2 psp[12], pu[9], pg[12];
  bool pval = false;
  auto prefetch = [&](int s0) {
    pval = false;
    if (has_t && s0 + t_sl < s_end) {
      const int s = s0 + t_sl;
      const int p = s >= g.Vh, i = s - p * g.Vh;
      const float2* f = in + t_cp * cs;
      pval = true;
      if (d == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) psp[k] = f[(int64_t)p * 12 * g.Vh + (int64_t)k * g.Vh + i];
      } else {
        int x[4];
        site_coords(g, p, i, x);
        const int mu = (d - 1) >> 1, dir = (d - 1) & 1;
        const int j = nbr_idx(g, x, mu, dir == 0 ? 1 : -1);
        const float2* fb = f + (int64_t)(1 - p) * 12 * g.Vh + j;
#pragma unroll
        for (int k = 0; k < 12; ++k) psp[k] = fb[(int64_t)k * g.Vh];
        const float2* ub = U.p + (int64_t)(((dir == 0 ? p : 1 - p) * 4 + mu) * 9) * U.n + (dir == 0 ? i : j);
#pragma unroll
        for (int k = 0; k < 9; ++k) pu[k] = ub[(int64_t)k * U.n];
      }
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const int e = threadIdx.x + q * 256;
      pg[q] = make_float2(0.f, 0.f);
      if (e < ng) {
        const int sl = e % kWgTileSites, rest = e / kWgTileSites;
        const int kc = rest % 12, c = rest / 12, s = s0 + sl;
        if (s < s_end) {
          const int p = s >= g.Vh, i = s - p * g.Vh;
          pg[q] = gy[c * cs + (int64_t)p * 12 * g.Vh + (int64_t)kc * g.Vh + i];
        }
      }
    }
  };
  prefetch(s_begin);
  for (int s0 = s_begin; s0 < s_end; s0 += kWgTileSites) {
    __syncthreads();
    if (has_t) {
      cx<float> tr[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) tr[k] = {0.f, 0.f};
      if (pval && d == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) tr[k] = {psp[k].x, psp[k].y};
      } else if (pval) {
        const int dir = (d - 1) & 1;
#pragma unroll
        for (int sb = 0; sb < 4; ++sb)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            cx<float> z{0.f, 0.f};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const cx<float> sv{psp[sb * 3 + b].x, psp[sb * 3 + b].y};
              z = dir == 0 ? fma_c(cx<float>{pu[a * 3 + b].x, pu[a * 3 + b].y}, sv, z)
                           : fmac_c(cx<float>{pu[b * 3 + a].x, pu[b * 3 + a].y}, sv, z);
            }
            tr[sb * 3 + a] = z;
          }
      }
#pragma unroll
      for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          float* r = tlw + (t_cp * 8 + sb * 2) * kWgLd + 3 * t_sl + a;
          r[0] = tr[sb * 3 + a].re;
          r[kWgLd] = tr[sb * 3 + a].im;
        }
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < ng) {
        const int sl = e % kWgTileSites, rest = e / kWgTileSites;
        const int kc = rest % 12, c = rest / 12;
        const int sa = kc / 3, a = kc - 3 * sa;
        float* r = gl + (c * 8 + sa * 2) * kWgLd + 3 * sl + a;
        r[0] = pg[q].x;
        r[kWgLd] = pg[q].y;
      }
    }
    if (s0 + kWgTileSites < s_end) prefetch(s0 + kWgTileSites);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wv + 4 * q;
      if (t >= ntile) break;
      const int mt = t / ntn, nt = t - mt * ntn;
      f4v c4 = acc[q];
      const float* ga = gl + (16 * mt + (lane & 15)) * kWgLd + (lane >> 4);
      const float* tb = tlw + (16 * nt + (lane & 15)) * kWgLd + (lane >> 4);
#pragma unroll
      for (int ks = 0; ks < 3 * kWgTileSites / 4; ++ks)
        c4 = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[4 * ks], tb[4 * ks], c4, 0, 0, 0);
      acc[q] = c4;
    }
  }
  // partial product of this workgroup: part[(range * 9 + d)][m][n]
  float* pw = part + ((int64_t)rg * 9 + d) * M16 * N16;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int t = wv + 4 * q;
    if (t >= ntile) break;
    const int mt = t / ntn, nt = t - mt * ntn;
#pragma unroll
    for (int r = 0; r < 4; ++r) pw[(16 * mt + 4 * (lane >> 4) + r) * N16 + 16 * nt + (lane & 15)] = acc[q][r];
  }
}

// grad[w] += sum over workgroups (fixed order, FP64) of the complex combination
// of the real partial products
__global__ void k_net_wgrad_reduce(const float* part, int nwg, int cin, int cout, float2* grad) {
  const int nw = 9 * cout * cin * 16;
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const int M16 = 16 * ((8 * cout + 15) / 16), N16 = 16 * ((8 * cin + 15) / 16);
  const int ss = w & 15, sa = ss >> 2, sb = ss & 3;
  int rest = w >> 4;
  const int cp = rest % cin;
  rest /= cin;
  const int c = rest % cout, d = rest / cout;
  const int mr = c * 8 + sa * 2, nr = cp * 8 + sb * 2;
  double re = 0, im = 0;
  for (int b = 0; b < nwg; ++b) {
    const float* P = part + ((int64_t)b * 9 + d) * M16 * N16;
    const float rr = P[mr * N16 + nr], ri = P[mr * N16 + nr + 1];
    const float ir = P[(mr + 1) * N16 + nr], ii = P[(mr + 1) * N16 + nr + 1];
    re += (double)rr + (double)ii;
    im += (double)ir - (double)ri;
  }
  grad[w] = make_float2(grad[w].x + (float)re, grad[w].y + (float)im);
}

// squared norm partials of an FP32 array: part[b]
__global__ void k_norm2_f(const float2* x, int64_t n, double* part) {
  __shared__ double sh[4];
  double acc = 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    float2 a = x[t];
    acc += (double)a.x * a.x + (double)a.y * a.y;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
    part[blockIdx.x] = s;
  }
}
hipError_t launch_norm2_f(const float2* x, int64_t n, double* part, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2_f, dim3(nb), dim3(256), 0, st, x, n, part);
  return hipGetLastError();
}

// y = a * x (FP32 <- FP32 or FP64)
template <class E>
__global__ void k_scale_to_f(float2* y, const E* x, double a, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    E v = x[t];
    y[t] = make_float2((float)(a * v.x), (float)(a * v.y));
  }
}
template <class E>
hipError_t launch_scale_to_f(float2* y, const E* x, double a, int64_t n, hipStream_t st) {
  int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL((k_scale_to_f<E>), dim3(nb), dim3(256), 0, st, y, x, a, n);
  return hipGetLastError();
}
template hipError_t launch_scale_to_f<float2>(float2*, const float2*, double, int64_t, hipStream_t);
template hipError_t launch_scale_to_f<double2>(float2*, const double2*, double, int64_t, hipStream_t);

// e = float(psi) - e   (errors of harvested iterates from the final solution)
__global__ void k_err_from(float2* e, const double2* psi, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double2 p = psi[t];
    float2 v = e[t];
    e[t] = make_float2((float)(p.x - v.x), (float)(p.y - v.y));
  }
}
hipError_t launch_err_from(float2* e, const double2* psi, int64_t n, hipStream_t st) {
  int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_err_from, dim3(nb), dim3(256), 0, st, e, psi, n);
  return hipGetLastError();
}

// a -= b  (FP64 -= FP32)
__global__ void k_sub_f(double2* a, const float2* b, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double2 v = a[t];
    float2 w = b[t];
    a[t] = make_double2(v.x - w.x, v.y - w.y);
  }
}
hipError_t launch_sub_f(double2* a, const float2* b, int64_t n, hipStream_t st) {
  int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_sub_f, dim3(nb), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}

// BF16 compute copy of the FP32 master weights
__global__ void k_net_to_bf16(const float2* w, uint32_t* wb, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) wb[t] = (uint32_t)f_to_bf16(w[t].x) | ((uint32_t)f_to_bf16(w[t].y) << 16);
}

// adjoint weights of one layer: W'[adj(d)][c'][c] = W[d][c][c']^dag (BF16 in, BF16 out)
__global__ void k_net_adjoint(const uint32_t* wb, int cin, int cout, uint32_t* wa) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int n = 9 * cout * cin * 16;
  if (t >= n) return;
  int ss = t & 15, rest = t >> 4;
  int sa = ss >> 2, sb = ss & 3;
  int cp = rest % cin;
  rest /= cin;
  int c = rest % cout, d = rest / cout;
  int ad = d == 0 ? 0 : (((d - 1) & 1) == 0 ? d + 1 : d - 1);
  uint32_t v = wb[t];
  uint32_t conjv = (v & 0xffffu) | ((v ^ 0x80000000u) & 0xffff0000u);  // negate the imaginary part
  // W'[ad][cp][c][sb][sa] = conj(W[d][c][cp][sa][sb])
  wa[(((int64_t)ad * cin + cp) * cout + c) * 16 + sb * 4 + sa] = conjv;
}

// output gradient and loss: gy = 2 (y - e s) / Z, loss partial = |y - e s|^2 / Z
__global__ void k_net_out_grad(const float2* y, const float2* e, float escale, float invZ, float2* gy, int64_t n,
                               double* part) {
  __shared__ double sh[4];
  double acc = 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    float2 a = y[t], b = e[t];
    float dx = a.x - escale * b.x, dy = a.y - escale * b.y;
    gy[t] = make_float2(2.f * dx * invZ, 2.f * dy * invZ);
    acc += ((double)dx * dx + (double)dy * dy) * invZ;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
    part[blockIdx.x] = s;
  }
}

// Adam on the real and imaginary parts of the FP32 master weights
__global__ void k_net_adam(float2* w, const float2* g, float4* mv, int n, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float4 s = mv[t];
  float2 gg = g[t];
  s.x = b1 * s.x + (1 - b1) * gg.x;
  s.y = b1 * s.y + (1 - b1) * gg.y;
  s.z = b2 * s.z + (1 - b2) * gg.x * gg.x;
  s.w = b2 * s.w + (1 - b2) * gg.y * gg.y;
  mv[t] = s;
  float2 v = w[t];
  v.x -= lr * (s.x / c1) / (sqrtf(s.z / c2) + eps);
  v.y -= lr * (s.y / c1) / (sqrtf(s.w / c2) + eps);
  w[t] = v;
}

// ------------------------------------------ layer on the matrix cores (MFMA)
// For every site x and colour a the layer is one matrix-vector product
//   out[(c, sa)](x, a) = sum_{d, c', sb} W[d][c][c'][sa][sb] T_d[(c', sb)](x, a),
// T_d the link-transported inputs, so a tile of sites is a GEMM with the site
// and colour as the column index.  In real form, rows m = (c, sa, re/im) and
// k = ((d, c'), sb, re/im) flattened over all nine transports (K = 72 cin,
// zero-padded to a multiple of 32): A = [[Wre, -Wim], [Wim, Wre]] per
// (c, sa | d, c', sb) block.  The weights are BF16 (A exact in BF16); each FP32
// transported input is split exactly into three BF16 terms, t = hi + mid + lo
// (8 + 8 + at most 8 significant bits), and A t = A hi + A mid + A lo runs on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation: the products are exact and
// the result is as accurate as an FP32 product, at three BF16 matrix
// operations per FP32 one of a quarter the depth.
// A workgroup of 4 wavefronts takes kNetTile = 64 sites (192 columns = 12
// column tiles of 16) and walks K in slabs of one MFMA depth: wavefront w
// computes the transported input of the slab's (d, c') pair for the 64 sites,
// one per lane (wave-uniform field and link bases, 32-bit lane offsets), into
// LDS as the three terms, [term][column][k] (k fastest: one 16-byte read per
// lane and operand), and runs the MFMAs of its 3 column tiles and all MT row
// tiles.  The slab takes 46 KB of LDS, leaving room for more than one
// workgroup per compute unit.  The
// A operands come prearranged (k_net_wmx) in the lane order of the
// instruction: lane l holds A[l%16][8(l/16) .. 8(l/16)+7], B[8(l/16) ..][l%16],
// and D rows 4(l/16)+r, column l%16 (measured with an in-bounds probe).
// K order (net_pair): the k groups g = 0..3 of a slab hold four (d, c') pairs.
// Per input channel c' one slab takes the four transports along the two
// fastest-running site coordinates (d = 5..8: their reads of c' fall on nearly
// the same neighbour sites, so three of four hit the cache) and the next the
// four along the others (d = 1..4); the untransported d = 0 pairs of four
// channels share the last slabs.  Wavefront g thus stages only transports 5 + g
// (even slabs) and 1 + g (odd slabs) and keeps each link across the channels.
constexpr int kNetTile = 64;
constexpr int kNetKs = 32;             // k rows per slab (one MFMA depth): 4 (d, c') pairs x 4 spins x re/im
constexpr int kNetLd = kNetKs + 8;     // LDS row stride of a column (BF16 elements)
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

// Layer forms.  Transport first (the general one): k = (d, c', sb, re/im) over
// nd = 9 transports, rows (c, sa, re/im).  Weights first, for a layer with one
// output channel and several inputs: since W acts on spin and channel and T_d
// on colour and position, out(x) = sum_d T_d z_d(x) with the site-local
// z_d = sum_c' W[d][0][c'] in_c', so the GEMM takes only the untransported
// inputs (nd = 1) and has the nine z_d as its output channels (cz = 9), and
// k_net_gather then applies 8 transports per site instead of 8 per input
// channel.
__host__ __device__ inline int net_mt(int cz) { return (8 * cz + 15) / 16; }
__host__ __device__ inline int net_kb(int cin, int nd) { return (8 * nd * cin + 31) / 32; }
// pair e = d cin + c' of k group g in slab sk, or -1 (zero column); for nd = 9
// the 2 cin transport slabs and ceil(cin / 4) untransported ones make up
// net_kb = ceil(9 cin / 4) exactly
__host__ __device__ inline int net_pair(int sk, int g, int cin, int nd) {
  if (nd == 1) return 4 * sk + g < cin ? 4 * sk + g : -1;
  if (sk < 2 * cin) return ((sk & 1) ? 1 + g : 5 + g) * cin + (sk >> 1);
  const int cp = 4 * (sk - 2 * cin) + g;
  return cp < cin ? cp : -1;
}
bool net_weights_first(int cin, int cout, int scratch_ch) { return cout == 1 && cin > 1 && scratch_ch >= 9; }

// prearranged A operands of one layer: wmx[(mt * KB + kb) * 64 + lane][0..7]
// (wf: the weights-first form)
__global__ void k_net_wmx(const uint32_t* wb, int cin, int cout, int wf, uint16_t* wmx) {
  const int cz = wf ? 9 * cout : cout, nd = wf ? 1 : 9;
  const int MT = net_mt(cz), KB = net_kb(cin, nd);
  const int64_t n = (int64_t)MT * KB * 64 * 8;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = (int)(t & 7), lane = (int)((t >> 3) & 63);
  const int64_t blk = t >> 9;
  const int kb = (int)(blk % KB), mt = (int)(blk / KB);
  const int m = 16 * mt + (lane & 15), e = net_pair(kb, lane >> 4, cin, nd);
  const int ch = m >> 3, sa = (m >> 1) & 3, ri_o = m & 1;
  uint16_t v = 0;
  if (ch < cz && e >= 0) {
    const int sb = (i >> 1) & 3, ri_i = i & 1;
    const int d = wf ? ch / cout : e / cin, cp = wf ? e : e - d * cin, c = wf ? ch - d * cout : ch;
    const uint32_t w = wb[((int64_t)(d * cout + c) * cin + cp) * 16 + sa * 4 + sb];
    const uint16_t wr = (uint16_t)(w & 0xffffu), wi = (uint16_t)(w >> 16);
    v = ri_o == ri_i ? wr : (ri_o == 0 ? (uint16_t)(wi ^ 0x8000u) : wi);
  }
  wmx[t] = v;
}

// cz output channels (cout, or the 9 cout z_d of the weights-first form), nd
// transports per input channel (9, or 1 for the weights-first form); TM BF16
// terms per transported input: 3 is the exact split (FP32 accuracy), 2 and 1
// keep the leading 16 or 8 significant bits (relative rounding error at most
// 2^-16 or 2^-8 per element), for inference where that suffices
template <int MT, int TM>
__global__ void __launch_bounds__(256) k_net_layer_mx(Geo g, LinkV<float> U, const uint4* wmx, int cin, int cz,
                                                      int nd, const float2* in, float2* out, int64_t cs) {
  extern __shared__ uint4 tl4[];  // [TM terms][3 kNetTile columns][kNetLd] BF16
  uint16_t* tl = reinterpret_cast<uint16_t*>(tl4);
  constexpr int N = 3 * kNetTile;
  // wv through readfirstlane: the compiler then knows that the pair, the
  // transport direction and the field bases derived from it are uniform (scalar
  // address arithmetic, uniform branches instead of selects)
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int s0 = blockIdx.x * kNetTile;
  const int KB = net_kb(cin, nd);
  // staging role: wavefront wv stages the (d, c') pair net_pair(sk, wv) of slab sk
  // for the tile's 64 sites, one per lane; the pair, the parity of the tile (the tiles
  // never straddle the parity boundary, Vh being a multiple of kNetTile) and
  // so the field and link bases are uniform across the wavefront
  const int s = s0 + lane;
  const bool live = s < g.V;
  const int p = s0 >= g.Vh, i = live ? s - p * g.Vh : 0;
  int x[4];
  site_coords(g, p, i, x);
  f4v acc[MT][3];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[mt][j] = f4v{0.f, 0.f, 0.f, 0.f};
  // operands of this lane's staging item (the input spinor, at the neighbour
  // for a transport, and the link), loaded two slabs ahead into one of two
  // buffers, so that the loads have two matrix-core phases to arrive in (one
  // slab ahead from one buffer for MT > 6, where the second buffer would cost
  // the second wavefront per SIMD)
  struct Item {
    float2 psp[12], pu[9];
    int pd;  // transport of the loaded item (-1: none, zero column)
    int ud;  // transport whose link pu holds (kept while the next item of the buffer has the same)
  };
  Item it0, it1;
  it0.pd = it1.pd = it0.ud = it1.ud = -1;
  // (lanes past the end of the lattice load site i = 0 of the parity, a valid
  // address, and stage zeros: no divergent branch around the loads, so the
  // bases stay scalar)
  auto prefetch = [&](Item& it, int sk) {
    const int e = net_pair(sk, wv, cin, nd);
    it.pd = e >= 0 ? e / cin : -1;
    const int pd = it.pd;
    if (pd < 0) return;
    const int cp = e - pd * cin;
    const float2* f = in + cp * cs;
    if (pd == 0) {
      const float2* fb = f + (int64_t)p * 12 * g.Vh;
#pragma unroll
      for (int k = 0; k < 12; ++k) it.psp[k] = ld_off(fb + (int64_t)k * g.Vh, (uint32_t)i * 8u);
    } else {
      const int mu = (pd - 1) >> 1, dir = (pd - 1) & 1;
      const int j = nbr_idx(g, x, mu, dir == 0 ? 1 : -1);
      const float2* fb = f + (int64_t)(1 - p) * 12 * g.Vh;
#pragma unroll
      for (int k = 0; k < 12; ++k) it.psp[k] = ld_off(fb + (int64_t)k * g.Vh, (uint32_t)j * 8u);
      if (pd != it.ud) {
        const float2* ub = U.p + (int64_t)(((dir == 0 ? p : 1 - p) * 4 + mu) * 9) * U.n;
        const uint32_t uo = (uint32_t)(dir == 0 ? i : j) * 8u;
#pragma unroll
        for (int k = 0; k < 9; ++k) it.pu[k] = ld_off(ub + (int64_t)k * U.n, uo);
        it.ud = pd;
      }
    }
  };
  auto slab = [&](int sk, Item& it, int ahead) {
    // A operands of the slab (latency hidden behind the staging below)
    uint4 aop[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) aop[mt] = wmx[((int64_t)mt * KB + sk) * 64 + lane];
    __syncthreads();
    {
      const int pd = it.pd;
      cx<float> tr[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) tr[k] = {0.f, 0.f};
      if (live && pd == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) tr[k] = {it.psp[k].x, it.psp[k].y};
      } else if (live && pd > 0 && ((pd - 1) & 1) == 0) {  // forward transport U psi(x + mu)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            cx<float> z{0.f, 0.f};
#pragma unroll
            for (int b = 0; b < 3; ++b)
              z = fma_c(cx<float>{it.pu[a * 3 + b].x, it.pu[a * 3 + b].y},
                        cx<float>{it.psp[sb * 3 + b].x, it.psp[sb * 3 + b].y}, z);
            tr[sb * 3 + a] = z;
          }
      } else if (live && pd > 0) {  // backward transport U^dag psi(x - mu)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            cx<float> z{0.f, 0.f};
#pragma unroll
            for (int b = 0; b < 3; ++b)
              z = fmac_c(cx<float>{it.pu[b * 3 + a].x, it.pu[b * 3 + a].y},
                         cx<float>{it.psp[sb * 3 + b].x, it.psp[sb * 3 + b].y}, z);
            tr[sb * 3 + a] = z;
          }
      }
      if (sk + ahead < KB) prefetch(it, sk + ahead);
      // BF16 split of each (re, im) pair, rounded to nearest by the packed
      // conversion: hi = bf16(t), mid = bf16(t - hi) (exact difference),
      // lo = t - hi - mid (exact, at most 8 significant bits), the first TM of
      // them; 8 consecutive k (sb, re/im) per column and term
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        uint32_t hw[TM][4];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
          f2v v = {tr[sb * 3 + a].re, tr[sb * 3 + a].im};
#pragma unroll
          for (int tm = 0; tm < TM; ++tm) {
            const bf2v t2 = __builtin_convertvector(v, bf2v);
            uint32_t w;
            __builtin_memcpy(&w, &t2, 4);
            hw[tm][sb] = w;
            if (tm + 1 < TM) v = v - f2v{__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u)};
          }
        }
        const int n = 3 * lane + a;
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
          *reinterpret_cast<uint4*>(tl + ((int64_t)tm * N + n) * kNetLd + 8 * wv) =
              make_uint4(hw[tm][0], hw[tm][1], hw[tm][2], hw[tm][3]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int tm = 0; tm < TM; ++tm) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int n = (3 * wv + j) * 16 + (lane & 15);
        const uint4 bw = *reinterpret_cast<const uint4*>(tl + ((int64_t)tm * N + n) * kNetLd + 8 * (lane >> 4));
        bf8v b;
        __builtin_memcpy(&b, &bw, 16);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          bf8v av;
          __builtin_memcpy(&av, &aop[mt], 16);
          acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b, acc[mt][j], 0, 0, 0);
        }
      }
    }
  };
  // slabs in pairs, even ones from buffer 0 and odd ones from buffer 1 (KB is
  // uniform: every wavefront takes the same branches and barriers)
  prefetch(it0, 0);
  if constexpr (MT <= 6) {
    if (KB > 1) prefetch(it1, 1);
    for (int sk = 0; sk < KB; sk += 2) {
      slab(sk, it0, 2);
      if (sk + 1 < KB) slab(sk + 1, it1, 2);
    }
  } else {
    for (int sk = 0; sk < KB; ++sk) slab(sk, it0, 1);
  }
  // lane holds rows m = 16 mt + 4 (lane/16) + r: r = 0,1 are (re, im) of (c, sa),
  // r = 2,3 those of (c, sa + 1); column n = 16 nt + lane%16 = (site, colour).
  // The results go out through LDS, eight channels at a time, as [c][component][site]
  // so that every store covers 64 consecutive sites of one component plane.
  float2* ob = reinterpret_cast<float2*>(tl4);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if (8 * half >= cz) break;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int n = (3 * wv + j) * 16 + (lane & 15);
      const int sl2 = n / 3, a = n - 3 * sl2;
#pragma unroll
      for (int mt = 4 * half; mt < 4 * half + 4; ++mt) {
        if (mt >= MT) break;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int m = mt * 16 + 4 * (lane >> 4) + 2 * h;
          const int c = m >> 3, sa = (m >> 1) & 3;
          ob[((c - 8 * half) * 12 + sa * 3 + a) * kNetTile + sl2] = make_float2(acc[mt][j][2 * h], acc[mt][j][2 * h + 1]);
        }
      }
    }
    __syncthreads();
    const int nc = min(8, cz - 8 * half);
    for (int e = threadIdx.x; e < nc * 12 * kNetTile; e += blockDim.x) {
      const int sl2 = e % kNetTile, kc = (e / kNetTile) % 12, c = 8 * half + e / (12 * kNetTile);
      const int s2 = s0 + sl2;
      if (s2 < g.V) out[c * cs + (int64_t)p * 12 * g.Vh + (int64_t)kc * g.Vh + (s2 - p * g.Vh)] = ob[e];
    }
  }
}

// out_c(x) = z_{0,c}(x) + sum_{d=1..8} (T_d z_{d,c})(x), z channel d cout + c:
// the transports of the weights-first form, one lane per site and channel
__global__ void __launch_bounds__(256) k_net_gather(Geo g, LinkV<float> U, const float2* z, int cout, float2* out,
                                                    int64_t cs) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (s >= g.V) return;
  const int p = s >= g.Vh, i = s - p * g.Vh;
  int x[4];
  site_coords(g, p, i, x);
  cx<float> acc[12];
  {
    const float2* f = z + (int64_t)c * cs + (int64_t)p * 12 * g.Vh + i;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {f[(int64_t)k * g.Vh].x, f[(int64_t)k * g.Vh].y};
  }
#pragma unroll 1
  for (int d = 1; d < 9; ++d) {
    const int mu = (d - 1) >> 1, dir = (d - 1) & 1;
    const int j = nbr_idx(g, x, mu, dir == 0 ? 1 : -1);
    cx<float> u[9], sp[12];
    if (dir == 0) ld_link(U, p, mu, i, u);
    else ld_link(U, 1 - p, mu, j, u);
    const float2* f = z + (int64_t)(d * cout + c) * cs + (int64_t)(1 - p) * 12 * g.Vh + j;
#pragma unroll
    for (int k = 0; k < 12; ++k) sp[k] = {f[(int64_t)k * g.Vh].x, f[(int64_t)k * g.Vh].y};
#pragma unroll
    for (int sb = 0; sb < 4; ++sb)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cx<float> t = acc[sb * 3 + a];
#pragma unroll
        for (int b = 0; b < 3; ++b)
          t = dir == 0 ? fma_c(u[a * 3 + b], sp[sb * 3 + b], t) : fmac_c(u[b * 3 + a], sp[sb * 3 + b], t);
        acc[sb * 3 + a] = t;
      }
  }
  float2* o = out + (int64_t)c * cs + (int64_t)p * 12 * g.Vh + i;
#pragma unroll
  for (int k = 0; k < 12; ++k) o[(int64_t)k * g.Vh] = make_float2(acc[k].re, acc[k].im);
}

// ------------------------------------------------------------------ launchers
hipError_t launch_net_layer(const Geo& g, const LinkV<float>& U, const uint16_t* wmx, int cin, int cout,
                            const float2* in, float2* out, int64_t cs, float2* scratch, int scratch_ch, int terms,
                            hipStream_t st) {
  if (cin < 1 || cout < 1 || cout > 16 || terms < 1 || terms > 3) return hipErrorInvalidValue;
  const bool wf = net_weights_first(cin, cout, scratch_ch);
  if (wf && !scratch) return hipErrorInvalidValue;
  const int cz = wf ? 9 * cout : cout, nd = wf ? 1 : 9;
  float2* dst = wf ? scratch : out;
  if (g.Vh % kNetTile) return hipErrorInvalidValue;  // tiles must not straddle the parity boundary
  const dim3 grid((g.V + kNetTile - 1) / kNetTile), blk(256);
  const size_t lds = std::max((size_t)terms * 3 * kNetTile * kNetLd * sizeof(uint16_t),  // K slab
                              (size_t)8 * 12 * kNetTile * sizeof(float2));               // output, 8 channels
  const uint4* w = reinterpret_cast<const uint4*>(wmx);
  switch (net_mt(cz) * 4 + terms) {
#define NET_MX(M, T) \
  case M * 4 + T: hipLaunchKernelGGL((k_net_layer_mx<M, T>), grid, blk, lds, st, g, U, w, cin, cz, nd, in, dst, cs); break;
#define NET_MX3(M) NET_MX(M, 1) NET_MX(M, 2) NET_MX(M, 3)
    NET_MX3(1) NET_MX3(2) NET_MX3(3) NET_MX3(4) NET_MX3(5) NET_MX3(6) NET_MX3(7) NET_MX3(8)
#undef NET_MX3
#undef NET_MX
    default: return hipErrorInvalidValue;
  }
  if (wf) hipLaunchKernelGGL(k_net_gather, dim3((g.V + 255) / 256, cout), dim3(256), 0, st, g, U, scratch, cout, out, cs);
  return hipGetLastError();
}

size_t net_wmx_elems(int cin, int cout, int scratch_ch) {
  const bool wf = net_weights_first(cin, cout, scratch_ch);
  return (size_t)net_mt(wf ? 9 * cout : cout) * net_kb(cin, wf ? 1 : 9) * 64 * 8;
}

hipError_t launch_net_wmx(const uint32_t* wb, int cin, int cout, int scratch_ch, uint16_t* wmx, hipStream_t st) {
  const int64_t n = (int64_t)net_wmx_elems(cin, cout, scratch_ch);
  hipLaunchKernelGGL(k_net_wmx, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, wb, cin, cout,
                     (int)net_weights_first(cin, cout, scratch_ch), wmx);
  return hipGetLastError();
}

// workgroups over the sites of the weight-gradient kernel: at most 512, at
// least 8 tiles of 16 sites each
static int wgrad_groups(int64_t V) {
  const int64_t tiles = (V + kWgTileSites - 1) / kWgTileSites;
  return (int)std::min<int64_t>(512, std::max<int64_t>(1, tiles / 8));
}
size_t net_wgrad_part_floats(int64_t V, int cin, int cout) {
  const int M16 = 16 * ((8 * cout + 15) / 16), N16 = 16 * ((8 * cin + 15) / 16);
  return (size_t)wgrad_groups(V) * 9 * M16 * N16;
}

hipError_t launch_net_wgrad(const Geo& g, const LinkV<float>& U, int cin, int cout, const float2* in,
                            const float2* gy, int64_t cs, float* part, size_t part_floats, float2* grad,
                            hipStream_t st) {
  if (cin < 1 || cout < 1 || cin > 16 || cout > 16 || part_floats < net_wgrad_part_floats(g.V, cin, cout))
    return hipErrorInvalidValue;
  const int nw = 9 * cout * cin * 16;
  const int M16 = 16 * ((8 * cout + 15) / 16), N16 = 16 * ((8 * cin + 15) / 16);
  const int ntile = (M16 / 16) * (N16 / 16), tpw = (ntile + 3) / 4;
  const int nwx = wgrad_groups(g.V);
  const int spw = ((g.V + nwx - 1) / nwx + kWgTileSites - 1) / kWgTileSites * kWgTileSites;
  const size_t lds = (size_t)(M16 + N16) * kWgLd * sizeof(float);
  const dim3 grid(nwx * 9), blk(256);
  if (tpw <= 2)
    hipLaunchKernelGGL((k_net_wgrad_mx<2>), grid, blk, lds, st, g, U, cin, cout, in, gy, cs, nwx, spw, part);
  else if (tpw <= 4)
    hipLaunchKernelGGL((k_net_wgrad_mx<4>), grid, blk, lds, st, g, U, cin, cout, in, gy, cs, nwx, spw, part);
  else if (tpw <= 9)
    hipLaunchKernelGGL((k_net_wgrad_mx<9>), grid, blk, lds, st, g, U, cin, cout, in, gy, cs, nwx, spw, part);
  else
    hipLaunchKernelGGL((k_net_wgrad_mx<16>), grid, blk, lds, st, g, U, cin, cout, in, gy, cs, nwx, spw, part);
  hipLaunchKernelGGL(k_net_wgrad_reduce, dim3((nw + 255) / 256), dim3(256), 0, st, part, nwx, cin, cout, grad);
  return hipGetLastError();
}

hipError_t launch_net_to_bf16(const float2* w, uint32_t* wb, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_net_to_bf16, dim3((n + 255) / 256), dim3(256), 0, st, w, wb, n);
  return hipGetLastError();
}

hipError_t launch_net_adjoint(const uint32_t* wb, int cin, int cout, uint32_t* wa, hipStream_t st) {
  int n = 9 * cout * cin * 16;
  hipLaunchKernelGGL(k_net_adjoint, dim3((n + 255) / 256), dim3(256), 0, st, wb, cin, cout, wa);
  return hipGetLastError();
}

hipError_t launch_net_out_grad(const float2* y, const float2* e, float escale, float invZ, float2* gy, int64_t n,
                               double* part, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_net_out_grad, dim3(nb), dim3(256), 0, st, y, e, escale, invZ, gy, n, part);
  return hipGetLastError();
}

hipError_t launch_net_adam(float2* w, const float2* g, float4* mv, int n, float lr, int step, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_net_adam, dim3((n + 255) / 256), dim3(256), 0, st, w, g, mv, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace qdd
