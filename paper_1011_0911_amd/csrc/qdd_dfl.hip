// Local deflation kernels (the "locally deflated" part of the paper's solver,
// Sect. 3-4, Table 1): block orthonormalisation of the deflation fields, the
// block-restricted hops that build the little Dirac operator, block inner
// products (Gram matrices, restriction), prolongation and the little-operator
// apply.  The lattice is cut into deflation blocks of bs[0] x .. x bs[3] sites;
// the little operator couples every block with itself (hops inside the block)
// and with its 8 face neighbours (hops across one face).
#include "qdd_kernels.h"
#include "qdd_dfl_kernels.h"

namespace qdd {

// global (parity, index) of local site s of block b
__device__ inline void block_site(const Geo& g, const DflGeo& d, int b, int s, int x[4], int& p, int& i) {
  int bc[4], y[4];
  int r = b;
  bc[3] = r % d.nb[3];
  r /= d.nb[3];
  bc[2] = r % d.nb[2];
  r /= d.nb[2];
  bc[1] = r % d.nb[1];
  bc[0] = r / d.nb[1];
  r = s;
  y[3] = r % d.bs[3];
  r /= d.bs[3];
  y[2] = r % d.bs[2];
  r /= d.bs[2];
  y[1] = r % d.bs[1];
  y[0] = r / d.bs[1];
  for (int m = 0; m < 4; ++m) x[m] = bc[m] * d.bs[m] + y[m];
  p = (x[0] + x[1] + x[2] + x[3]) & 1;
  i = lex_of(g, x) >> 1;
}

__device__ inline int block_of(const DflGeo& d, const int x[4]) {
  return (((x[0] / d.bs[0]) * d.nb[1] + x[1] / d.bs[1]) * d.nb[2] + x[2] / d.bs[2]) * d.nb[3] + x[3] / d.bs[3];
}

// neighbouring block across face f = 1 + 2 mu + dir (dir 0 up, 1 down)
__device__ inline int block_nbr(const DflGeo& d, int b, int f) {
  int bc[4];
  int r = b;
  bc[3] = r % d.nb[3];
  r /= d.nb[3];
  bc[2] = r % d.nb[2];
  r /= d.nb[2];
  bc[1] = r % d.nb[1];
  bc[0] = r / d.nb[1];
  int mu = (f - 1) >> 1, dir = (f - 1) & 1;
  bc[mu] = dir == 0 ? (bc[mu] + 1) % d.nb[mu] : (bc[mu] + d.nb[mu] - 1) % d.nb[mu];
  return ((bc[0] * d.nb[1] + bc[1]) * d.nb[2] + bc[2]) * d.nb[3] + bc[3];
}

// deflation block of a workgroup: hardware workgroup ids go round-robin over the
// 8 XCDs, so every XCD is given a contiguous range of blocks.  With 4^4 blocks a
// block row holds 2 sites of a parity, and the blocks next to each other in x3
// share the cache lines of the parity-split fields: walked on one XCD they are
// fetched once into its L2 instead of once per XCD.
__device__ inline int xcd_block(int bid, int nblk) {
  return (nblk & 7) == 0 ? (bid & 7) * (nblk >> 3) + (bid >> 3) : bid;
}

template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// sum over the workgroup (result in every lane); sh: >= 2 * nwaves doubles
__device__ inline cx<double> group_sum(cx<double> v, double* sh) {
  double re = wave_sum(v.re), im = wave_sum(v.im);
  int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[2 * w] = re;
    sh[2 * w + 1] = im;
  }
  __syncthreads();
  cx<double> s{0.0, 0.0};
  for (int k = 0; k < nw; ++k) {
    s.re += sh[2 * k];
    s.im += sh[2 * k + 1];
  }
  return s;
}

// Orthonormalise, on every block, the block restrictions of the Ns fields:
// for l ascending, two passes of w_l -= <w_k, w_l>_b w_k (k < l, sequentially),
// then w_l /= |w_l|_b.  One workgroup per block, one lane per site; the field
// being orthonormalised stays in registers while the earlier ones stream
// through, so every w_k is read once per pass and w_l written once.  W: FP64
// full fields, field l at W + l * vs.
__global__ void __launch_bounds__(1024) k_block_orth(Geo g, DflGeo d, double2* W, int64_t vs, int Ns) {
  __shared__ double sh[32];
  const int nsb = d.bs[0] * d.bs[1] * d.bs[2] * d.bs[3];
  const int s = threadIdx.x;
  const bool on = s < nsb;
  const int blk = xcd_block(blockIdx.x, d.nblk);
  int64_t off = 0;
  if (on) {
    int x[4], p, i;
    block_site(g, d, blk, s, x, p, i);
    off = (int64_t)p * 12 * g.Vh + i;
  }
  for (int l = 0; l < Ns; ++l) {
    double2* wl = W + l * vs + off;
    cx<double> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      double2 b = on ? wl[(int64_t)c * g.Vh] : make_double2(0.0, 0.0);
      v[c] = {b.x, b.y};
    }
    for (int pass = 0; pass < 2; ++pass)
      for (int k = 0; k < l; ++k) {
        const double2* wk = W + k * vs + off;
        cx<double> a[12], acc{0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          double2 t = on ? wk[(int64_t)c * g.Vh] : make_double2(0.0, 0.0);
          a[c] = {t.x, t.y};
          acc = fmac_c(a[c], v[c], acc);
        }
        const cx<double> pr = group_sum(acc, sh);
        const cx<double> mp{-pr.re, -pr.im};
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = fma_c(mp, a[c], v[c]);
      }
    cx<double> nn{0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 12; ++c) nn.re = fmar(v[c].re, v[c].re, fmar(v[c].im, v[c].im, nn.re));
    const cx<double> tot = group_sum(nn, sh);
    const double sc = tot.re > 0 ? 1.0 / sqrt(tot.re) : 0.0;
    if (on) {
#pragma unroll
      for (int c = 0; c < 12; ++c) wl[(int64_t)c * g.Vh] = make_double2(v[c].re * sc, v[c].im * sc);
    }
    __syncthreads();  // w_l is read by every later l
  }
}

// F_l = block part of D W_l for every field l (FP64):
//   mode 0: F = A W - 1/2 H_inside W          (hops inside the deflation block)
//   mode f = 1 + 2 mu + dir: F = -1/2 (hop across the face f) W at the sites on
//            that face, 0 elsewhere
template <int MODE>
__global__ void __launch_bounds__(128) k_dfl_hops(Geo g, DflGeo d, LinkV<double> U, CloverV<double> A,
                                                  const double2* W, int64_t vs, double2* F, int Ns) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)g.V * Ns) return;
  int l = (int)(t / g.V), s = (int)(t % g.V);
  int p = s >= g.Vh, i = s - p * g.Vh;
  int x[4];
  site_coords(g, p, i, x);
  FieldV<double> w{(double2*)W + l * vs, nullptr, 0, 0, g.Vh};
  FieldV<double> src = w, self = w;
  src.p += (int64_t)(1 - p) * 12 * g.Vh;
  self.p += (int64_t)p * 12 * g.Vh;
  cx<double> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = {0.0, 0.0};
  cx<double> sp[12], h[6], gg[6], u[9];
  auto hop = [&](auto mu_c, auto sg_c) {
    constexpr int MU = decltype(mu_c)::value, SG = decltype(sg_c)::value;
    int j = nbr_idx(g, x, MU, SG);
    ld_spinor(src, 0, j, sp);
    project<double, MU, SG>(sp, h);
    if constexpr (SG > 0) {
      ld_link(U, p, MU, i, u);
      su3_mul_half<double, false>(u, h, gg);
    } else {
      ld_link(U, 1 - p, MU, j, u);
      su3_mul_half<double, true>(u, h, gg);
    }
    reconstruct_add<double, MU, SG>(gg, acc);
  };
  auto inside = [&](int mu, int dir) {
    int pos = x[mu] % d.bs[mu];
    return dir == 0 ? pos != d.bs[mu] - 1 : pos != 0;
  };
  if constexpr (MODE == 0) {
    if (inside(0, 0)) hop(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{});
    if (inside(0, 1)) hop(std::integral_constant<int, 0>{}, std::integral_constant<int, -1>{});
    if (inside(1, 0)) hop(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{});
    if (inside(1, 1)) hop(std::integral_constant<int, 1>{}, std::integral_constant<int, -1>{});
    if (inside(2, 0)) hop(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{});
    if (inside(2, 1)) hop(std::integral_constant<int, 2>{}, std::integral_constant<int, -1>{});
    if (inside(3, 0)) hop(std::integral_constant<int, 3>{}, std::integral_constant<int, 1>{});
    if (inside(3, 1)) hop(std::integral_constant<int, 3>{}, std::integral_constant<int, -1>{});
    cx<double> o[12];
    ld_spinor(self, 0, i, sp);
    clover_apply<double>(A, p, i, sp, o);
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = o[k] - 0.5 * acc[k];
  } else {
    constexpr int MU = (MODE - 1) >> 1, DIR = (MODE - 1) & 1;
    if (!inside(MU, DIR)) {
      hop(std::integral_constant<int, MU>{}, std::integral_constant<int, DIR == 0 ? 1 : -1>{});
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = -0.5 * acc[k];
    }
  }
  FieldV<double> out{F + l * vs + (int64_t)p * 12 * g.Vh, nullptr, 0, 0, g.Vh};
  st_spinor(out, 0, i, acc);
}

// out[b][kx][ky] (row stride ldo, block stride bso) = sum over the sites of block
// b of sum_c conj(X_kx) Y_ky.  X: nx fields at stride xvs, Y: ny fields at
// stride yvs (full-field layout).  Site chunks of both sets are staged in LDS.
template <class EX, class EY>
__global__ void __launch_bounds__(256) k_block_dots(Geo g, DflGeo d, const EX* X, int64_t xvs, int nx, const EY* Y,
                                                    int64_t yvs, int ny, double2* out, int64_t bso, int64_t ldo,
                                                    int64_t kys, int cs) {
  extern __shared__ double2 lds[];
  double2* xs = lds;                   // [nx][cs][12]
  double2* ys = lds + nx * cs * 12;    // [ny][cs][12]
  const int nsb = d.bs[0] * d.bs[1] * d.bs[2] * d.bs[3];
  const int np = nx * ny, blk = xcd_block(blockIdx.x, d.nblk);
  cx<double> acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  for (int s0 = 0; s0 < nsb; s0 += cs) {
    int nsc = min(cs, nsb - s0);
    int tot = (nx + ny) * nsc * 12;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
      int c = e % 12, rest = e / 12;
      int s = rest % nsc, v = rest / nsc;
      int x[4], p, i;
      block_site(g, d, blk, s0 + s, x, p, i);
      int64_t o = (int64_t)p * 12 * g.Vh + (int64_t)c * g.Vh + i;
      if (v < nx) {
        cx<double> z = cvt_any(X[v * xvs + o]);
        xs[(v * cs + s) * 12 + c] = make_double2(z.re, z.im);
      } else {
        cx<double> z = cvt_any(Y[(v - nx) * yvs + o]);
        ys[((v - nx) * cs + s) * 12 + c] = make_double2(z.re, z.im);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int pr = threadIdx.x + q * blockDim.x;
      if (pr < np) {
        int kx = pr / ny, ky = pr % ny;
        for (int s = 0; s < nsc; ++s)
#pragma unroll
          for (int c = 0; c < 12; ++c) {
            double2 a = xs[(kx * cs + s) * 12 + c], b = ys[(ky * cs + s) * 12 + c];
            acc[q] = fmac_c(cx<double>{a.x, a.y}, cx<double>{b.x, b.y}, acc[q]);
          }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int pr = threadIdx.x + q * blockDim.x;
    if (pr < np) {
      int kx = pr / ny, ky = pr % ny;
      out[(int64_t)blk * bso + (int64_t)kx * ldo + (int64_t)ky * kys] = make_double2(acc[q].re, acc[q].im);
    }
  }
}

// out_r(x) = sum_k W_k(x) c[r][b(x)][k] (+ optional add of out), for nrhs rhs;
// c: [rhs][nblk][Ns] FP64; W fields at stride wvs; out fields at stride ovs
template <class EW, class EO>
__global__ void __launch_bounds__(256) k_prolong(Geo g, DflGeo d, const EW* W, int64_t wvs, int Ns,
                                                 const double2* c, int64_t nc, EO* out, int64_t ovs, int nrhs) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.V) return;
  int s = (int)t;
  int p = s >= g.Vh, i = s - p * g.Vh;
  int x[4];
  site_coords(g, p, i, x);
  int b = block_of(d, x);
  int64_t o = (int64_t)p * 12 * g.Vh + i;
  for (int r0 = 0; r0 < nrhs; r0 += 4) {
    cx<double> acc[4][12];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[q][k] = {0.0, 0.0};
    for (int k = 0; k < Ns; ++k) {
      cx<double> w[12];
#pragma unroll
      for (int cc = 0; cc < 12; ++cc) w[cc] = cvt_any(W[k * wvs + o + (int64_t)cc * g.Vh]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (r0 + q < nrhs) {
          double2 cv = c[(r0 + q) * nc + (int64_t)b * Ns + k];
          cx<double> z{cv.x, cv.y};
#pragma unroll
          for (int cc = 0; cc < 12; ++cc) acc[q][cc] = fma_c(z, w[cc], acc[q][cc]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (r0 + q < nrhs)
#pragma unroll
        for (int cc = 0; cc < 12; ++cc) out[(r0 + q) * ovs + o + (int64_t)cc * g.Vh] = to_elem<EO>(acc[q][cc]);
  }
}

// little-operator apply: out[r][b][k] = sum_f sum_l A[b][f][k][l] in[r][nbr(b,f)][l]
__global__ void __launch_bounds__(256) k_coarse_apply(DflGeo d, const double2* Am, int Ns, const double2* in,
                                                      double2* out, int64_t nc, int nrhs) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t tot = (int64_t)nrhs * d.nblk * Ns;
  if (t >= tot) return;
  int r = (int)(t % nrhs);
  int64_t rest = t / nrhs;
  int k = (int)(rest % Ns), b = (int)(rest / Ns);
  cx<double> acc{0.0, 0.0};
  for (int f = 0; f < 9; ++f) {
    int bb = f == 0 ? b : block_nbr(d, b, f);
    const double2* row = Am + (((int64_t)b * 9 + f) * Ns + k) * Ns;
    const double2* v = in + r * nc + (int64_t)bb * Ns;
    for (int l = 0; l < Ns; ++l) {
      double2 a = row[l], z = v[l];
      acc = fma_c(cx<double>{a.x, a.y}, cx<double>{z.x, z.y}, acc);
    }
  }
  out[r * nc + (int64_t)b * Ns + k] = make_double2(acc.re, acc.im);
}

// ---------------------------------------------------------------- launchers
hipError_t launch_block_orth(const Geo& g, const DflGeo& d, double2* W, int64_t vs, int Ns, hipStream_t st) {
  int nsb = d.bs[0] * d.bs[1] * d.bs[2] * d.bs[3];
  if (nsb > 1024) return hipErrorInvalidValue;
  int thr = ((nsb + 63) / 64) * 64;  // one lane per site
  hipLaunchKernelGGL(k_block_orth, dim3(d.nblk), dim3(thr), 0, st, g, d, W, vs, Ns);
  return hipGetLastError();
}

hipError_t launch_dfl_hops(const Geo& g, const DflGeo& d, const DevOp<double>& op, const double2* W, int64_t vs,
                           double2* F, int Ns, int mode, hipStream_t st) {
  int64_t n = (int64_t)g.V * Ns;
  dim3 grid((unsigned)((n + 127) / 128)), blk(128);
  switch (mode) {
#define M(k) \
  case k: hipLaunchKernelGGL(k_dfl_hops<k>, grid, blk, 0, st, g, d, op.U, op.A, W, vs, F, Ns); break;
    M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8)
#undef M
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class EX, class EY>
hipError_t launch_block_dots(const Geo& g, const DflGeo& d, const EX* X, int64_t xvs, int nx, const EY* Y,
                             int64_t yvs, int ny, double2* out, int64_t bso, int64_t ldo, int64_t kys,
                             hipStream_t st) {
  if (nx * ny > 1024) return hipErrorInvalidValue;
  int cs = (int)(65536 / ((size_t)(nx + ny) * 12 * sizeof(double2)));
  if (cs < 1) return hipErrorInvalidValue;
  cs = cs > 16 ? 16 : cs;
  size_t lds = (size_t)(nx + ny) * cs * 12 * sizeof(double2);
  hipLaunchKernelGGL((k_block_dots<EX, EY>), dim3(d.nblk), dim3(256), lds, st, g, d, X, xvs, nx, Y, yvs, ny, out,
                     bso, ldo, kys, cs);
  return hipGetLastError();
}

template <class EW, class EO>
hipError_t launch_prolong(const Geo& g, const DflGeo& d, const EW* W, int64_t wvs, int Ns, const double2* c,
                          int64_t nc, EO* out, int64_t ovs, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_prolong<EW, EO>), dim3((g.V + 255) / 256), dim3(256), 0, st, g, d, W, wvs, Ns, c, nc, out,
                     ovs, nrhs);
  return hipGetLastError();
}

hipError_t launch_coarse_apply(const DflGeo& d, const double2* A, int Ns, const double2* in, double2* out,
                               int64_t nc, int nrhs, hipStream_t st) {
  int64_t tot = (int64_t)nrhs * d.nblk * Ns;
  hipLaunchKernelGGL(k_coarse_apply, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, d, A, Ns, in, out, nc,
                     nrhs);
  return hipGetLastError();
}

template hipError_t launch_block_dots<double2, double2>(const Geo&, const DflGeo&, const double2*, int64_t, int,
                                                        const double2*, int64_t, int, double2*, int64_t, int64_t,
                                                        int64_t, hipStream_t);
template hipError_t launch_block_dots<float2, double2>(const Geo&, const DflGeo&, const float2*, int64_t, int,
                                                       const double2*, int64_t, int, double2*, int64_t, int64_t,
                                                       int64_t, hipStream_t);
template hipError_t launch_block_dots<float2, float2>(const Geo&, const DflGeo&, const float2*, int64_t, int,
                                                      const float2*, int64_t, int, double2*, int64_t, int64_t,
                                                      int64_t, hipStream_t);

template <class E>
__global__ void k_add(E* y, const E* x, double a, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    cx<double> v = cvt_any(y[t]), w = cvt_any(x[t]);
    y[t] = to_elem<E>(v + a * w);
  }
}
template <class E>
hipError_t launch_add(E* y, const E* x, double a, int64_t n, hipStream_t st) {
  int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL((k_add<E>), dim3(nb), dim3(256), 0, st, y, x, a, n);
  return hipGetLastError();
}
template hipError_t launch_add<double2>(double2*, const double2*, double, int64_t, hipStream_t);
template hipError_t launch_add<float2>(float2*, const float2*, double, int64_t, hipStream_t);
template hipError_t launch_prolong<double2, double2>(const Geo&, const DflGeo&, const double2*, int64_t, int,
                                                     const double2*, int64_t, double2*, int64_t, int, hipStream_t);
template hipError_t launch_prolong<float2, float2>(const Geo&, const DflGeo&, const float2*, int64_t, int,
                                                   const double2*, int64_t, float2*, int64_t, int, hipStream_t);
template hipError_t launch_prolong<float2, double2>(const Geo&, const DflGeo&, const float2*, int64_t, int,
                                                    const double2*, int64_t, double2*, int64_t, int, hipStream_t);

}  // namespace qdd
