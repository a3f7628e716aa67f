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

namespace qdd {

__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ inline uint16_t f_to_bf16(float f) {
  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

// one lane per site and output-channel group of CG channels; blockIdx.y = group
template <int CG>
__global__ void __launch_bounds__(128) k_net_layer(Geo g, LinkV<float> U, const uint32_t* Wb, int cin, int cout,
                                                   const float2* in, float2* out, int64_t cs) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.V) return;
  int s = (int)t;
  int p = s >= g.Vh, i = s - p * g.Vh;
  int c0 = blockIdx.y * CG;
  int x[4];
  site_coords(g, p, i, x);
  cx<float> acc[CG][12];
#pragma unroll
  for (int q = 0; q < CG; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {0.f, 0.f};
  for (int cp = 0; cp < cin; ++cp) {
    const float2* f = in + cp * cs;
    for (int d = 0; d < 9; ++d) {
      cx<float> tr[12];
      if (d == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          float2 v = f[(int64_t)p * 12 * g.Vh + (int64_t)k * g.Vh + i];
          tr[k] = {v.x, v.y};
        }
      } else {
        int mu = (d - 1) >> 1, dir = (d - 1) & 1;
        int j = nbr_idx(g, x, mu, dir == 0 ? 1 : -1);
        cx<float> u[9], sp[12];
        const float2* fb = f + (int64_t)(1 - p) * 12 * g.Vh + j;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          float2 v = fb[(int64_t)k * g.Vh];
          sp[k] = {v.x, v.y};
        }
        if (dir == 0) ld_link(U, p, mu, i, u);
        else ld_link(U, 1 - p, mu, j, u);
#pragma unroll
        for (int sp_i = 0; sp_i < 4; ++sp_i)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            cx<float> z{0.f, 0.f};
#pragma unroll
            for (int b = 0; b < 3; ++b)
              z = dir == 0 ? fma_c(u[a * 3 + b], sp[sp_i * 3 + b], z) : fmac_c(u[b * 3 + a], sp[sp_i * 3 + b], z);
            tr[sp_i * 3 + a] = z;
          }
      }
#pragma unroll
      for (int q = 0; q < CG; ++q) {
        int c = c0 + q;
        if (c < cout) {
          const uint32_t* w = Wb + ((int64_t)(d * cout + c) * cin + cp) * 16;
#pragma unroll
          for (int sa = 0; sa < 4; ++sa)
#pragma unroll
            for (int sb = 0; sb < 4; ++sb) {
              uint32_t wv = w[sa * 4 + sb];
              cx<float> ww{bf16_to_f((uint16_t)(wv & 0xffffu)), bf16_to_f((uint16_t)(wv >> 16))};
#pragma unroll
              for (int a = 0; a < 3; ++a) acc[q][sa * 3 + a] = fma_c(ww, tr[sb * 3 + a], acc[q][sa * 3 + a]);
            }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CG; ++q) {
    int c = c0 + q;
    if (c < cout) {
      float2* o = out + c * cs + (int64_t)p * 12 * g.Vh + i;
#pragma unroll
      for (int k = 0; k < 12; ++k) o[(int64_t)k * g.Vh] = make_float2(acc[q][k].re, acc[q][k].im);
    }
  }
}

// weight gradient partial sums: part[wg][((d*cout + c)*cin + c')*16 + s*4 + s'] =
//   sum over the workgroup's sites and colours of gy_c[s] conj((T_d in_c')[s'])
// Site chunks of the transported inputs and of gy are staged in LDS.
constexpr int kWgSites = 4;
// weights are split over blockIdx.y in ranges of 32 per lane (256 lanes)
__global__ void __launch_bounds__(256) k_net_wgrad(Geo g, LinkV<float> U, int cin, int cout, const float2* in,
                                                   const float2* gy, int64_t cs, int sites_per_wg, float2* part) {
  const int w0 = blockIdx.y * 32 * 256;
  extern __shared__ float2 lds[];
  float2* tl = lds;                                   // [d][c'][site][12]
  float2* gl = lds + 9 * cin * kWgSites * 12;         // [c][site][12]
  const int nw = 9 * cout * cin * 16;
  float2 acc[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) acc[q] = make_float2(0.f, 0.f);
  int s_begin = blockIdx.x * sites_per_wg, s_end = min(g.V, s_begin + sites_per_wg);
  for (int s0 = s_begin; s0 < s_end; s0 += kWgSites) {
    int nsc = min(kWgSites, s_end - s0);
    // stage transported inputs: one lane per (d, c', site, colour-spin row)
    int ntr = 9 * cin * nsc;
    for (int e = threadIdx.x; e < ntr; e += blockDim.x) {
      int sl = e % nsc, rest = e / nsc;
      int cp = rest % cin, d = rest / cin;
      int s = s0 + sl;
      int p = s >= g.Vh, i = s - p * g.Vh;
      const float2* f = in + cp * cs;
      float2* dst = tl + ((d * cin + cp) * kWgSites + sl) * 12;
      if (d == 0) {
        for (int k = 0; k < 12; ++k) dst[k] = f[(int64_t)p * 12 * g.Vh + (int64_t)k * g.Vh + i];
      } else {
        int x[4];
        site_coords(g, p, i, x);
        int mu = (d - 1) >> 1, dir = (d - 1) & 1;
        int j = nbr_idx(g, x, mu, dir == 0 ? 1 : -1);
        cx<float> u[9];
        if (dir == 0) ld_link(U, p, mu, i, u);
        else ld_link(U, 1 - p, mu, j, u);
        const float2* fb = f + (int64_t)(1 - p) * 12 * g.Vh + j;
        for (int sp = 0; sp < 4; ++sp)
          for (int a = 0; a < 3; ++a) {
            cx<float> z{0.f, 0.f};
            for (int b = 0; b < 3; ++b) {
              float2 v = fb[(int64_t)(sp * 3 + b) * g.Vh];
              z = dir == 0 ? fma_c(u[a * 3 + b], cx<float>{v.x, v.y}, z) : fmac_c(u[b * 3 + a], cx<float>{v.x, v.y}, z);
            }
            dst[sp * 3 + a] = make_float2(z.re, z.im);
          }
      }
    }
    int ng = cout * nsc * 12;
    for (int e = threadIdx.x; e < ng; e += blockDim.x) {
      int k = e % 12, rest = e / 12;
      int sl = rest % nsc, c = rest / nsc;
      int s = s0 + sl;
      int p = s >= g.Vh, i = s - p * g.Vh;
      gl[(c * kWgSites + sl) * 12 + k] = gy[c * cs + (int64_t)p * 12 * g.Vh + (int64_t)k * g.Vh + i];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      int w = w0 + threadIdx.x + q * blockDim.x;
      if (w >= nw) continue;
      int ss = w & 15, rest = w >> 4;
      int sa = ss >> 2, sb = ss & 3;
      int cp = rest % cin;
      rest /= cin;
      int c = rest % cout, d = rest / cout;
      cx<float> z{acc[q].x, acc[q].y};
      for (int sl = 0; sl < nsc; ++sl)
        for (int a = 0; a < 3; ++a) {
          float2 gv = gl[(c * kWgSites + sl) * 12 + sa * 3 + a];
          float2 tv = tl[((d * cin + cp) * kWgSites + sl) * 12 + sb * 3 + a];
          // gy * conj(t)
          z = fmac_c(cx<float>{tv.x, tv.y}, cx<float>{gv.x, gv.y}, z);
        }
      acc[q] = make_float2(z.re, z.im);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    int w = w0 + threadIdx.x + q * blockDim.x;
    if (w < nw) part[(int64_t)blockIdx.x * nw + w] = acc[q];
  }
}

// grad[w] += sum over workgroups of part[wg][w] (fixed order: deterministic)
__global__ void k_net_wgrad_reduce(const float2* part, int nwg, int nw, float2* grad) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  double re = 0, im = 0;
  for (int b = 0; b < nwg; ++b) {
    float2 v = part[(int64_t)b * nw + w];
    re += v.x;
    im += v.y;
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
// and colour as the column index.  In real form (rows (c, sa, re/im), k index
// (c', sb, re/im)): A = [[Wre, -Wim], [Wim, Wre]] per (c, sa | c', sb) block.
// A workgroup of 2 wavefronts takes kNetTile sites (3 kNetTile columns = 6
// column tiles of 16); for each direction d the transported inputs of the
// tile are computed into LDS as T[k][n] and the waves run
// v_mfma_f32_16x16x4f32 over them (FP32 operands: the BF16 weights convert
// exactly, the activations stay FP32), each wave owning 3 column tiles and
// all MT row tiles.  Operand layout of 16x16x4: lane l holds A[l%16][l/16],
// B[l/16][l%16] and D rows 4(l/16)+r, column l%16.
constexpr int kNetTile = 32;
typedef float f4v __attribute__((ext_vector_type(4)));

template <int MT>
__global__ void __launch_bounds__(128) k_net_layer_mx(Geo g, LinkV<float> U, const uint32_t* Wb, int cin, int cout,
                                                      const float2* in, float2* out, int64_t cs) {
  extern __shared__ float tl[];  // [8 cin][3 kNetTile]
  constexpr int N = 3 * kNetTile;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int s0 = blockIdx.x * kNetTile;
  const int K = 8 * cin;
  f4v acc[MT][3];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[mt][j] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int d = 0; d < 9; ++d) {
    // transported inputs of the tile: one (site, input channel) pair per item
    __syncthreads();
    for (int e = threadIdx.x; e < kNetTile * cin; e += blockDim.x) {
      const int sl = e % kNetTile, cp = e / kNetTile;
      const int s = s0 + sl;
      cx<float> tr[12];
      if (s < g.V) {
        const int p = s >= g.Vh, i = s - p * g.Vh;
        const float2* f = in + cp * cs;
        if (d == 0) {
#pragma unroll
          for (int k = 0; k < 12; ++k) {
            float2 v = f[(int64_t)p * 12 * g.Vh + (int64_t)k * g.Vh + i];
            tr[k] = {v.x, v.y};
          }
        } else {
          const int mu = (d - 1) >> 1, dir = (d - 1) & 1;
          int x[4];
          site_coords(g, p, i, x);
          const int j = nbr_idx(g, x, mu, dir == 0 ? 1 : -1);
          cx<float> u[9], sp[12];
          const float2* fb = f + (int64_t)(1 - p) * 12 * g.Vh + j;
#pragma unroll
          for (int k = 0; k < 12; ++k) {
            float2 v = fb[(int64_t)k * g.Vh];
            sp[k] = {v.x, v.y};
          }
          if (dir == 0) ld_link(U, p, mu, i, u);
          else ld_link(U, 1 - p, mu, j, u);
#pragma unroll
          for (int sb = 0; sb < 4; ++sb)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              cx<float> z{0.f, 0.f};
#pragma unroll
              for (int b = 0; b < 3; ++b)
                z = dir == 0 ? fma_c(u[a * 3 + b], sp[sb * 3 + b], z) : fmac_c(u[b * 3 + a], sp[sb * 3 + b], z);
              tr[sb * 3 + a] = z;
            }
        }
      } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) tr[k] = {0.f, 0.f};
      }
#pragma unroll
      for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int n = sl * 3 + a, k0 = cp * 8 + sb * 2;
          tl[k0 * N + n] = tr[sb * 3 + a].re;
          tl[(k0 + 1) * N + n] = tr[sb * 3 + a].im;
        }
    }
    __syncthreads();
    // acc += A_d T_d over k in steps of 4
    for (int kk = 0; kk < K; kk += 4) {
      const int k = kk + (lane >> 4);
      const int cp = k >> 3, sb = (k >> 1) & 3, ri_i = k & 1;
      f4v bq[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) bq[j] = f4v{tl[k * N + (3 * wv + j) * 16 + (lane & 15)], 0.f, 0.f, 0.f};
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int m = mt * 16 + (lane & 15);
        const int c = m >> 3, sa = (m >> 1) & 3, ri_o = m & 1;
        float av = 0.f;
        if (c < cout) {
          const uint32_t w = Wb[((int64_t)(d * cout + c) * cin + cp) * 16 + sa * 4 + sb];
          const float wr = bf16_to_f((uint16_t)(w & 0xffffu)), wi = bf16_to_f((uint16_t)(w >> 16));
          av = ri_o == ri_i ? wr : (ri_o == 0 ? -wi : wi);
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bq[j][0], acc[mt][j], 0, 0, 0);
      }
    }
  }
  // lane holds rows m = 16 mt + 4 (lane/16) + r: r = 0,1 are (re, im) of (c, sa),
  // r = 2,3 those of (c, sa + 1); column n = 16 nt + lane%16 = (site, colour)
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int n = (3 * wv + j) * 16 + (lane & 15);
    const int sl = n / 3, a = n - 3 * sl, s = s0 + sl;
    if (s >= g.V) continue;
    const int p = s >= g.Vh, i = s - p * g.Vh;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = mt * 16 + 4 * (lane >> 4) + 2 * h;
        const int c = m >> 3, sa = (m >> 1) & 3;
        if (c < cout)
          out[c * cs + (int64_t)p * 12 * g.Vh + (int64_t)(sa * 3 + a) * g.Vh + i] =
              make_float2(acc[mt][j][2 * h], acc[mt][j][2 * h + 1]);
      }
    }
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_net_layer(const Geo& g, const LinkV<float>& U, const uint32_t* Wb, int cin, int cout,
                            const float2* in, float2* out, int64_t cs, hipStream_t st) {
  // matrix-core path (cout <= 16 -> at most 8 row tiles of 16)
  const int mt = (8 * cout + 15) / 16;
  const dim3 grid((g.V + kNetTile - 1) / kNetTile), blk(128);
  const size_t lds = (size_t)8 * cin * 3 * kNetTile * sizeof(float);
  switch (mt) {
#define NET_MX(M) \
  case M: hipLaunchKernelGGL((k_net_layer_mx<M>), grid, blk, lds, st, g, U, Wb, cin, cout, in, out, cs); break;
    NET_MX(1) NET_MX(2) NET_MX(3) NET_MX(4) NET_MX(5) NET_MX(6) NET_MX(7) NET_MX(8)
#undef NET_MX
    default: {
      constexpr int CG = 4;
      dim3 grid2((g.V + 127) / 128, (cout + CG - 1) / CG);
      hipLaunchKernelGGL((k_net_layer<CG>), grid2, dim3(128), 0, st, g, U, Wb, cin, cout, in, out, cs);
    }
  }
  return hipGetLastError();
}

hipError_t launch_net_wgrad(const Geo& g, const LinkV<float>& U, int cin, int cout, const float2* in,
                            const float2* gy, int64_t cs, float2* part, int nwg, float2* grad, hipStream_t st) {
  int nw = 9 * cout * cin * 16;
  int spw = (g.V + nwg - 1) / nwg;
  size_t lds = (size_t)(9 * cin + cout) * kWgSites * 12 * sizeof(float2);
  dim3 grid(nwg, (nw + 32 * 256 - 1) / (32 * 256));
  hipLaunchKernelGGL(k_net_wgrad, grid, dim3(256), lds, st, g, U, cin, cout, in, gy, cs, spw, part);
  hipLaunchKernelGGL(k_net_wgrad_reduce, dim3((nw + 255) / 256), dim3(256), 0, st, part, nwg, nw, grad);
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
