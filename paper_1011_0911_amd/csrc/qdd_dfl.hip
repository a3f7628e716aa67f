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

// ---------------------------------------------------------------- block products on the matrix cores
// C_b = X_b^dag Y_b for every block b as one real GEMM on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  Over k' = (site, component, re/im) the rows of the
// left operand are the x fields [Re X | Im X], the columns of the right operand
// are (Re Y, Im Y) for Re C and (Im Y, -Re Y) for Im C:
//   Re C = sum (Xr Yr + Xi Yi),   Im C = sum (Xr Yi - Xi Yr).
// The block is walked one x3 row at a time: the row's sites of either parity are
// bs3/2 consecutive entries of that parity's array, so one staging unit (field,
// parity, component) is a contiguous run.  Any fixed order of k' serves, as long
// as X and Y use the same one.  The four wavefronts take a quarter of the k'
// steps of every row each, and their partial tiles are added in wavefront order,
// so the result is deterministic.  Face products (face = 1 + 2 mu + dir, mu < 3)
// visit only the block rows on that face, where the face fields are non-zero.
typedef double dv4 __attribute__((ext_vector_type(4)));
constexpr int kMmMaxT = 8;   // 16 x 16 output tiles per workgroup
constexpr int kMmPre = 9;    // staged elements of X (and of Y) per lane and row, at most

struct MmShape {
  int MT, NT;   // row tiles (x fields), column tiles (2 ny real columns)
  int rows;     // staged LDS rows: 16 MT x-rows (+ ny y-rows) + one zero row
  int ybase;    // first y-row (0 when Y is X)
  int ld;       // LDS row stride in doubles
};

__host__ __device__ inline MmShape mm_shape(int nx, int ny, int sym, int h) {
  MmShape m;
  m.MT = (nx + 15) / 16;
  m.NT = (2 * ny + 15) / 16;
  m.ybase = sym ? 0 : 16 * m.MT;
  m.rows = 16 * m.MT + (sym ? 0 : ny) + 1;
  // 48 h doubles of one row plus 4: 8 x odd words between rows, so the 16 rows
  // of an operand read fall on distinct bank groups
  m.ld = 48 * h + 4;
  return m;
}

// X in the parity-split field layout (field v at X + v * xvs), or block-major
// (XB): block b, field v, row q, element (p * 12 + c) * h + k at
// X[((b * nx + v) * nrow + q) * 24 h + (p * 12 + c) * h + k], so that a row of
// a field is one contiguous run.  PX / PY: staged elements of X / Y per lane and
// row, held in registers; the loads are issued unconditionally (slots past the
// end reload element 0 and skip the store), so no branch separates them.
template <class EX, class EY, int MAXT, int PX, int PY, bool XB>
__global__ void __launch_bounds__(256) k_block_mm(Geo g, DflGeo d, const EX* X, int64_t xvs, int nx, const EY* Y,
                                                  int64_t yvs, int ny, int sym, double2* out, int64_t bso,
                                                  int64_t ldo, int64_t kys, int face) {
  extern __shared__ double sm[];
  const int h = d.bs[3] >> 1;
  const MmShape m = mm_shape(nx, ny, sym, h);
  const int T = m.MT * m.NT, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int blk = xcd_block(blockIdx.x, d.nblk);
  const int nsb12 = d.bs[0] * d.bs[1] * d.bs[2] * d.bs[3] * 12;
  int bc[4];
  {
    int r = blk;
    bc[3] = r % d.nb[3];
    r /= d.nb[3];
    bc[2] = r % d.nb[2];
    r /= d.nb[2];
    bc[1] = r % d.nb[1];
    bc[0] = r / d.nb[1];
  }
  // rows of the walk: all (y0, y1, y2), or those on the face
  int ext[3] = {d.bs[0], d.bs[1], d.bs[2]}, fmu = -1, fpos = 0;
  if (face > 0 && ((face - 1) >> 1) < 3) {
    fmu = (face - 1) >> 1;
    fpos = ((face - 1) & 1) == 0 ? d.bs[fmu] - 1 : 0;
    ext[fmu] = 1;
  }
  const int nrow = ext[0] * ext[1] * ext[2];
  // zero the padding rows (x rows nx..16MT-1 and the last row), never staged
  for (int e = threadIdx.x; e < (16 * m.MT - nx + 1) * m.ld; e += blockDim.x) {
    const int r = e / m.ld, c = e - r * m.ld;
    sm[(r < 16 * m.MT - nx ? nx + r : m.rows - 1) * m.ld + c] = 0.0;
  }
  // per-lane operand addresses of every tile
  int acol[MAXT], bcol[MAXT];
  double bsg[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int mt = t < T ? t / m.NT : 0, nt = t < T ? t - (t / m.NT) * m.NT : 0;
    acol[t] = (16 * mt + (lane & 15)) * m.ld + (lane >> 4);
    const int j = 16 * nt + (lane & 15), kq = lane >> 4;
    if (j < ny) {
      bcol[t] = (m.ybase + j) * m.ld + kq;
      bsg[t] = 1.0;
    } else if (j < 2 * ny) {
      bcol[t] = (m.ybase + j - ny) * m.ld + (kq ^ 1);
      bsg[t] = (kq & 1) ? -1.0 : 1.0;
    } else {
      bcol[t] = (m.rows - 1) * m.ld + kq;
      bsg[t] = 1.0;
    }
  }
  dv4 acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = dv4{0.0, 0.0, 0.0, 0.0};
  // Staging of one row.  Element e of a field set = ((v * 2 + p) * 12 + c) * h + k
  // (field v, parity p, component c, k-th site of the row's run); its offset from
  // the row's start and its LDS slot do not depend on the row.
  const int nex = nx * 24 * h, ney = sym ? 0 : ny * 24 * h;
  constexpr int PY1 = PY > 0 ? PY : 1;
  int goffx[PX], loffx[PX], goffy[PY1], loffy[PY1];
#pragma unroll
  for (int j = 0; j < PX; ++j) {
    const int e = threadIdx.x + 256 * j;
    const int k = e % h, u = e / h, c = u % 12, t = u / 12, p = t & 1, v = t >> 1;
    const int el = (p * 12 + c) * h + k;
    goffx[j] = e < nex ? (XB ? v * nsb12 + el : (int)(v * xvs + p * 12 * g.Vh + c * g.Vh + k)) : 0;
    loffx[j] = e < nex ? v * m.ld + 2 * el : -1;
  }
#pragma unroll
  for (int j = 0; j < PY1; ++j) {
    const int e = threadIdx.x + 256 * j;
    const int k = e % h, u = e / h, c = u % 12, t = u / 12, p = t & 1, v = t >> 1;
    goffy[j] = PY > 0 && e < ney ? (int)(v * yvs + p * 12 * g.Vh + c * g.Vh + k) : 0;
    loffy[j] = PY > 0 && e < ney ? (m.ybase + v) * m.ld + 2 * ((p * 12 + c) * h + k) : -1;
  }
  // parity-split start index of a row, and its index in the full walk
  auto row_start = [&](int q, int& qf) {
    int y[3];
    y[2] = q % ext[2];
    y[1] = (q / ext[2]) % ext[1];
    y[0] = q / (ext[2] * ext[1]);
    if (fmu >= 0) y[fmu] = fpos;
    qf = (y[0] * d.bs[1] + y[1]) * d.bs[2] + y[2];
    const int row = ((bc[0] * d.bs[0] + y[0]) * g.L[1] + bc[1] * d.bs[1] + y[1]) * g.L[2] + bc[2] * d.bs[2] + y[2];
    return row * g.Lh3 + bc[3] * h;
  };
  EX px[2][PX];
  EY py[2][PY1];
  auto prefetch = [&](EX* bx, EY* by, int q) {
    int qf;
    const int i0 = row_start(q, qf);
    const EX* xr = XB ? X + (int64_t)blk * nx * nsb12 + qf * 24 * h : X + i0;
#pragma unroll
    for (int j = 0; j < PX; ++j) bx[j] = xr[goffx[j]];
    if (PY > 0) {
      const EY* yr = Y + i0;
#pragma unroll
      for (int j = 0; j < PY; ++j) by[j] = yr[goffy[j]];
    }
  };
  const int spw = 3 * h;  // k' steps of 4 per wavefront and row
  auto row_step = [&](EX* bx, EY* by, int q) {
    __syncthreads();  // the previous row's operands are consumed
#pragma unroll
    for (int j = 0; j < PX; ++j) {
      const cx<double> z = cvt_any(bx[j]);
      if (loffx[j] >= 0) {
        sm[loffx[j]] = z.re;
        sm[loffx[j] + 1] = z.im;
      }
    }
#pragma unroll
    for (int j = 0; j < PY; ++j) {
      const cx<double> z = cvt_any(by[j]);
      if (loffy[j] >= 0) {
        sm[loffy[j]] = z.re;
        sm[loffy[j] + 1] = z.im;
      }
    }
    __syncthreads();
    // issued on every row (the last rows reload the last one, unused) so that no
    // branch separates the loads
    prefetch(bx, by, min(q + 2, nrow - 1));
    for (int ks = w * spw; ks < (w + 1) * spw; ++ks) {
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        if (t < T) {
          const double a = sm[acol[t] + 4 * ks], b = bsg[t] * sm[bcol[t] + 4 * ks];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        }
      }
    }
  };
  prefetch(px[0], py[0], 0);
  prefetch(px[1], py[1], min(1, nrow - 1));
  for (int q = 0; q < nrow; q += 2) {
    row_step(px[0], py[0], q);
    if (q + 1 < nrow) row_step(px[1], py[1], q + 1);
  }
  // partial tiles of the four wavefronts, added in wavefront order into P
  double* ex = sm;                       // [4][256]
  double* P = sm + 1024;                 // [16 MT][16 NT]
  const int pn = 16 * m.NT;
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    if (t < T) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) ex[w * 256 + lane * 4 + r] = acc[t][r];
      __syncthreads();
      const int e = threadIdx.x, l = e >> 2, r = e & 3, mt = t / m.NT, nt = t - mt * m.NT;
      // FP64 16x16x4 output: register r of lane l holds row 4 r + l / 16, column l mod 16
      P[(16 * mt + 4 * r + (l >> 4)) * pn + 16 * nt + (l & 15)] = ex[e] + ex[256 + e] + ex[512 + e] + ex[768 + e];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nx * ny; e += blockDim.x) {
    const int i = e / ny, j = e - i * ny;
    out[(int64_t)blk * bso + (int64_t)i * ldo + (int64_t)j * kys] = make_double2(P[i * pn + j], P[i * pn + ny + j]);
  }
}

// Block-major copy of Ns fields (the X layout of k_block_mm with XB), one
// thread per output element.
template <class EO>
__global__ void k_to_blocks(Geo g, DflGeo d, const double2* W, int64_t vs, int Ns, EO* out) {
  const int h = d.bs[3] >> 1, rl = 24 * h, nrow = d.bs[0] * d.bs[1] * d.bs[2];
  const int64_t n = (int64_t)d.nblk * Ns * nrow * rl;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
    const int el = (int)(o % rl);
    int64_t t = o / rl;
    const int q = (int)(t % nrow);
    t /= nrow;
    const int v = (int)(t % Ns), b = (int)(t / Ns);
    const int k = el % h, pc = el / h, c = pc % 12, p = pc / 12;
    int r = b, bc[4];
    bc[3] = r % d.nb[3];
    r /= d.nb[3];
    bc[2] = r % d.nb[2];
    r /= d.nb[2];
    bc[1] = r % d.nb[1];
    bc[0] = r / d.nb[1];
    const int y2 = q % d.bs[2], y1 = (q / d.bs[2]) % d.bs[1], y0 = q / (d.bs[2] * d.bs[1]);
    const int row = ((bc[0] * d.bs[0] + y0) * g.L[1] + bc[1] * d.bs[1] + y1) * g.L[2] + bc[2] * d.bs[2] + y2;
    const int i = row * g.Lh3 + bc[3] * h + k;
    out[o] = to_elem<EO>(cvt_any(W[v * vs + (int64_t)p * 12 * g.Vh + (int64_t)c * g.Vh + i]));
  }
}

// ---------------------------------------------------------------- block orthonormalisation (CholeskyQR)
// For every block the Gram matrix G = W_b^dag W_b (from k_block_mm) is factored
// as G = R^dag R (R upper triangular, positive diagonal) and R^{-1} formed; then
// W_b <- W_b R^{-1} gives the same orthonormal fields as Gram-Schmidt in field
// order (the QR factorisation with positive diagonal is unique).  Two rounds
// make the result orthonormal to working precision for block condition numbers
// up to ~1e7.  A non-positive pivot (fields dependent on the block) drops that
// field on the block (its column of R^{-1} is zero).
// One wavefront per block; G and R in LDS (Ns <= 32).
__global__ void __launch_bounds__(64) k_block_chol(const double2* G, int Ns, double2* Rinv) {
  __shared__ double2 R[32 * 33], Xl[32 * 33];
  const int b = blockIdx.x, lane = threadIdx.x, ldr = 33;
  const double2* Gb = G + (int64_t)b * Ns * Ns;
  for (int e = lane; e < Ns * Ns; e += 64) R[(e / Ns) * ldr + e % Ns] = Gb[e];
  __syncthreads();
  for (int j = 0; j < Ns; ++j) {
    const double piv = R[j * ldr + j].x;
    const double dj = piv > 0 ? sqrt(piv) : 0.0, inv = piv > 0 ? 1.0 / dj : 0.0;
    __syncthreads();
    // row j of R: R[j][l] = A[j][l] / d for l >= j
    for (int l = j + lane; l < Ns; l += 64) {
      const double2 a = R[j * ldr + l];
      R[j * ldr + l] = l == j ? make_double2(dj, 0.0) : make_double2(a.x * inv, a.y * inv);
    }
    __syncthreads();
    // trailing update A[i][l] -= conj(R[j][i]) R[j][l], j < i <= l
    const int n = Ns - j - 1;
    for (int e = lane; e < n * n; e += 64) {
      const int i = j + 1 + e / n, l = j + 1 + e % n;
      if (l < i) continue;
      const double2 ri = R[j * ldr + i], rl = R[j * ldr + l];
      double2 a = R[i * ldr + l];
      a.x -= ri.x * rl.x + ri.y * rl.y;
      a.y -= ri.x * rl.y - ri.y * rl.x;
      R[i * ldr + l] = a;
    }
    __syncthreads();
  }
  // R^{-1} column by column (lane l, column in LDS): X[l][l] = 1 / R[l][l],
  // X[i][l] = -(sum_{k=i+1..l} R[i][k] X[k][l]) / R[i][i]
  double2* Xb = Rinv + (int64_t)b * Ns * Ns;
  for (int l = lane; l < Ns; l += 64) {
    for (int i = 0; i < Ns; ++i) Xl[i * ldr + l] = make_double2(0.0, 0.0);
    const double dl = R[l * ldr + l].x;
    if (dl > 0) {
      Xl[l * ldr + l] = make_double2(1.0 / dl, 0.0);
      for (int i = l - 1; i >= 0; --i) {
        double sr = 0, si = 0;
        for (int k = i + 1; k <= l; ++k) {
          const double2 r = R[i * ldr + k], x = Xl[k * ldr + l];
          sr += r.x * x.x - r.y * x.y;
          si += r.x * x.y + r.y * x.x;
        }
        const double di = R[i * ldr + i].x;
        Xl[i * ldr + l] = di > 0 ? make_double2(-sr / di, -si / di) : make_double2(0.0, 0.0);
      }
    }
    for (int i = 0; i < Ns; ++i) Xb[i * Ns + l] = Xl[i * ldr + l];
  }
}

// W_b <- W_b R^{-1} on every block: out_l = sum_{k<=l} W_k X[k][l] at every
// (site, component); one workgroup per block, one lane per site, X in LDS.
template <int NSM>
__global__ void __launch_bounds__(256) k_block_rmul(Geo g, DflGeo d, double2* W, int64_t vs, int Ns,
                                                    const double2* Rinv) {
  __shared__ double2 Xs[NSM * NSM];
  const int blk = xcd_block(blockIdx.x, d.nblk);
  for (int e = threadIdx.x; e < Ns * Ns; e += blockDim.x) Xs[e] = Rinv[(int64_t)blk * Ns * Ns + e];
  __syncthreads();
  const int nsb = d.bs[0] * d.bs[1] * d.bs[2] * d.bs[3];
  for (int s = threadIdx.x; s < nsb; s += blockDim.x) {
    int x[4], p, i;
    block_site(g, d, blk, s, x, p, i);
    double2* base = W + (int64_t)p * 12 * g.Vh + i;
    for (int c = 0; c < 12; ++c) {
      cx<double> v[NSM];
#pragma unroll
      for (int k = 0; k < NSM; ++k)
        if (k < Ns) v[k] = cvt_any(base[k * vs + (int64_t)c * g.Vh]);
#pragma unroll
      for (int l = NSM - 1; l >= 0; --l) {
        if (l < Ns) {
          cx<double> a{0.0, 0.0};
#pragma unroll
          for (int k = 0; k <= l; ++k) a = fma_c(v[k], cvt_any(Xs[k * Ns + l]), a);
          v[l] = a;  // v[k], k < l, still hold the input fields
        }
      }
#pragma unroll
      for (int k = 0; k < NSM; ++k)
        if (k < Ns) base[k * vs + (int64_t)c * g.Vh] = make_double2(v[k].re, v[k].im);
    }
  }
}

// out_r(x) = sum_k W_k(x) c[r][b(x)][k], for nrhs rhs;
// c: [rhs][nblk][Ns] FP64; W fields at stride wvs; out fields at stride ovs.
// A lane takes one site, NC of its 12 components and NQ right-hand sides at a
// time; the 12 / NC component slices of a site go to different lanes (slice
// slowest, so a wavefront reads 64 consecutive sites of one component array).
// With NC = 6 and NQ = 8 an 8-rhs batch reads each basis element once instead
// of once per 4 rhs; the sum over k runs in the same order either way.
template <class EW, class EO, int NQ, int NC>
__global__ void __launch_bounds__(256) k_prolong(Geo g, DflGeo d, const EW* W, int64_t wvs, int Ns,
                                                 const double2* c, int64_t nc, EO* out, int64_t ovs, int nrhs) {
  constexpr int NS = 12 / NC;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)g.V * NS) return;
  const int sl = (int)(t / g.V);
  int s = (int)(t - (int64_t)sl * g.V);
  int p = s >= g.Vh, i = s - p * g.Vh;
  int x[4];
  site_coords(g, p, i, x);
  int b = block_of(d, x);
  int64_t o = (int64_t)p * 12 * g.Vh + i + (int64_t)sl * NC * g.Vh;
  for (int r0 = 0; r0 < nrhs; r0 += NQ) {
    cx<double> acc[NQ][NC];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int k = 0; k < NC; ++k) acc[q][k] = {0.0, 0.0};
    for (int k = 0; k < Ns; ++k) {
      cx<double> w[NC];
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) w[cc] = cvt_any(W[k * wvs + o + (int64_t)cc * g.Vh]);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (r0 + q < nrhs) {
          double2 cv = c[(r0 + q) * nc + (int64_t)b * Ns + k];
          cx<double> z{cv.x, cv.y};
#pragma unroll
          for (int cc = 0; cc < NC; ++cc) acc[q][cc] = fma_c(z, w[cc], acc[q][cc]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (r0 + q < nrhs)
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) out[(r0 + q) * ovs + o + (int64_t)cc * g.Vh] = to_elem<EO>(acc[q][cc]);
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

// The same apply with one wavefront per block: for each of the 9 couplings the
// Ns x Ns block of A (rows padded to Ns + 1 so that lanes on consecutive rows
// read distinct LDS banks) and the neighbour's coarse vectors of all right-hand
// sides are staged in LDS with coalesced loads; each lane then accumulates one
// row k for 4 right-hand sides.  The sums run in the same order as above.
template <int NG>
__global__ void __launch_bounds__(64) k_coarse_apply_lds(DflGeo d, const double2* Am, int Ns, const double2* in,
                                                         double2* out, int64_t nc, int nrhs) {
  extern __shared__ double2 cl[];
  const int lda = Ns + 1;
  double2* As = cl;             // [Ns][Ns + 1]
  double2* Is = cl + Ns * lda;  // [nrhs][Ns]
  const int b = xcd_block(blockIdx.x, d.nblk), lane = threadIdx.x;
  const int ngr = Ns * ((nrhs + 3) >> 2);
  cx<double> acc[NG][4];
#pragma unroll
  for (int j = 0; j < NG; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[j][i] = {0.0, 0.0};
  for (int f = 0; f < 9; ++f) {
    const int bb = f == 0 ? b : block_nbr(d, b, f);
    const double2* Ab = Am + ((int64_t)b * 9 + f) * Ns * Ns;
    __syncthreads();  // the previous coupling's operands are consumed
    for (int e = lane; e < Ns * Ns; e += 64) {
      const int k = e / Ns;
      As[k * lda + e - k * Ns] = Ab[e];
    }
    for (int e = lane; e < nrhs * Ns; e += 64) {
      const int r = e / Ns;
      Is[e] = in[r * nc + (int64_t)bb * Ns + e - r * Ns];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      const int gi = lane + 64 * j;
      if (gi < ngr) {
        const int k = gi % Ns, r0 = 4 * (gi / Ns);
        for (int l = 0; l < Ns; ++l) {
          const double2 a = As[k * lda + l];
          const cx<double> av{a.x, a.y};
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (r0 + i < nrhs) acc[j][i] = fma_c(av, cvt_any(Is[(r0 + i) * Ns + l]), acc[j][i]);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NG; ++j) {
    const int gi = lane + 64 * j;
    if (gi < ngr) {
      const int k = gi % Ns, r0 = 4 * (gi / Ns);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (r0 + i < nrhs) out[(r0 + i) * nc + (int64_t)b * Ns + k] = make_double2(acc[j][i].re, acc[j][i].im);
    }
  }
}

// ---------------------------------------------------------------- launchers
template <class EX, class EY>
hipError_t launch_block_mm(const Geo& g, const DflGeo& d, const EX* X, int64_t xvs, int nx, const EY* Y, int64_t yvs,
                           int ny, int sym, double2* out, int64_t bso, int64_t ldo, int64_t kys, int face,
                           hipStream_t st);

static bool mm_offsets_ok(int nx, int64_t xvs, int ny, int64_t yvs);

hipError_t launch_block_orth(const Geo& g, const DflGeo& d, double2* W, int64_t vs, int Ns, double2* work,
                             hipStream_t st) {
  int nsb = d.bs[0] * d.bs[1] * d.bs[2] * d.bs[3];
  if (work && Ns <= 32 && block_mm_fits(Ns, Ns, 1, d) && mm_offsets_ok(Ns, vs, 0, 0)) {
    // CholeskyQR, two rounds: Gram on the matrix cores, factor and R^{-1} per
    // block, W <- W R^{-1}
    double2 *G = work, *Ri = work + (int64_t)d.nblk * Ns * Ns;
    for (int round = 0; round < 2; ++round) {
      hipError_t e = launch_block_mm<double2, double2>(g, d, W, vs, Ns, W, vs, Ns, 1, G, (int64_t)Ns * Ns, Ns, 1, 0,
                                                       st);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_block_chol, dim3(d.nblk), dim3(64), 0, st, G, Ns, Ri);
      if (Ns <= 8) hipLaunchKernelGGL((k_block_rmul<8>), dim3(d.nblk), dim3(256), 0, st, g, d, W, vs, Ns, Ri);
      else if (Ns <= 16) hipLaunchKernelGGL((k_block_rmul<16>), dim3(d.nblk), dim3(256), 0, st, g, d, W, vs, Ns, Ri);
      else if (Ns <= 24) hipLaunchKernelGGL((k_block_rmul<24>), dim3(d.nblk), dim3(256), 0, st, g, d, W, vs, Ns, Ri);
      else hipLaunchKernelGGL((k_block_rmul<32>), dim3(d.nblk), dim3(256), 0, st, g, d, W, vs, Ns, Ri);
    }
    return hipGetLastError();
  }
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

// LDS bytes of the matrix-core block product (0 if it does not apply)
static size_t block_mm_lds(int nx, int ny, int sym, const DflGeo& d) {
  const int h = d.bs[3] / 2;
  const MmShape m = mm_shape(nx, ny, sym, h);
  if (m.MT * m.NT > kMmMaxT || h < 1 || (d.bs[3] & 1)) return 0;  // rows of even length only
  if ((std::max(nx, sym ? 0 : ny) * 24 * h + 255) / 256 > kMmPre) return 0;  // a row in the register set

  const size_t stage = (size_t)m.rows * m.ld, red = 1024 + (size_t)256 * m.MT * m.NT;
  const size_t bytes = 8 * (stage > red ? stage : red);
  return bytes <= 96 * 1024 ? bytes : 0;
}
bool block_mm_fits(int nx, int ny, int sym, const DflGeo& d) { return block_mm_lds(nx, ny, sym, d) != 0; }
// the staging keeps element offsets in 32 bits
static bool mm_offsets_ok(int nx, int64_t xvs, int ny, int64_t yvs) {
  return (int64_t)nx * xvs < ((int64_t)1 << 31) && (int64_t)ny * yvs < ((int64_t)1 << 31);
}

template <class EX, class EY, bool XB>
static hipError_t mm_dispatch(const Geo& g, const DflGeo& d, const EX* X, int64_t xvs, int nx, const EY* Y,
                              int64_t yvs, int ny, int sym, double2* out, int64_t bso, int64_t ldo, int64_t kys,
                              int face, size_t lds, hipStream_t st) {
  const int h = d.bs[3] / 2;
  const MmShape m = mm_shape(nx, ny, sym, h);
  // register sets sized to the shape: tiles, and staged elements of X and Y per lane and row
  const int T = m.MT * m.NT, px = (nx * 24 * h + 255) / 256, py = sym ? 0 : (ny * 24 * h + 255) / 256;
  const int PXs = px <= 2 ? 2 : px <= 5 ? 5 : 9;
  const int PYs = py == 0 ? 0 : py <= 2 ? 2 : py <= PXs ? PXs : 9;
  const int key = (T <= 2 ? 0 : 100) + PXs * 10 + PYs;
#define MM(MT_, PX_, PY_)                                                                                            \
  case (MT_ == 2 ? 0 : 100) + PX_ * 10 + PY_:                                                                        \
    hipLaunchKernelGGL((k_block_mm<EX, EY, MT_, PX_, PY_, XB>), dim3(d.nblk), dim3(256), lds, st, g, d, X, xvs, nx, \
                       Y, yvs, ny, sym, out, bso, ldo, kys, face);                                                  \
    break;
  switch (key) {
    MM(2, 2, 0) MM(2, 2, 2) MM(2, 5, 0) MM(2, 5, 2) MM(2, 5, 5) MM(2, 9, 0) MM(2, 9, 2) MM(2, 9, 9)
    MM(8, 2, 0) MM(8, 2, 2) MM(8, 5, 0) MM(8, 5, 2) MM(8, 5, 5) MM(8, 9, 0) MM(8, 9, 2) MM(8, 9, 9)
    default: return hipErrorInvalidValue;
  }
#undef MM
  return hipGetLastError();
}

template <class EX, class EY>
hipError_t launch_block_mm(const Geo& g, const DflGeo& d, const EX* X, int64_t xvs, int nx, const EY* Y, int64_t yvs,
                           int ny, int sym, double2* out, int64_t bso, int64_t ldo, int64_t kys, int face,
                           hipStream_t st) {
  const size_t lds = block_mm_lds(nx, ny, sym, d);
  if (!lds) return hipErrorInvalidValue;
  return mm_dispatch<EX, EY, false>(g, d, X, xvs, nx, Y, yvs, ny, sym, out, bso, ldo, kys, face, lds, st);
}

// The matrix-core product takes at most kMmMaxT output tiles and the VALU one
// 1024 field pairs, so wider products run in chunks of Y fields.  X block-major
// (XB) takes the matrix-core product only.
template <class EX, class EY, bool XB>
static hipError_t block_dots_impl(const Geo& g, const DflGeo& d, const EX* X, int64_t xvs, int nx, const EY* Y,
                                  int64_t yvs, int ny, double2* out, int64_t bso, int64_t ldo, int64_t kys,
                                  hipStream_t st, int face) {
  if (nx < 1 || ny < 1) return hipErrorInvalidValue;
  const bool mm = block_mm_fits(nx, 1, 0, d) && mm_offsets_ok(XB ? 0 : nx, xvs, ny, yvs);
  if (XB && !mm) return hipErrorInvalidValue;
  int nyc = ny;
  if (mm)
    while (!block_mm_fits(nx, nyc, 0, d)) nyc = (nyc + 1) / 2;
  else
    nyc = std::min(ny, std::max(1, 1024 / nx));
  for (int j0 = 0; j0 < ny; j0 += nyc) {
    const int n = std::min(nyc, ny - j0);
    const EY* Yc = Y + j0 * yvs;
    double2* oc = out + j0 * kys;
    if (mm) {
      hipError_t e = mm_dispatch<EX, EY, XB>(g, d, X, xvs, nx, Yc, yvs, n, 0, oc, bso, ldo, kys, face,
                                             block_mm_lds(nx, n, 0, d), st);
      if (e != hipSuccess) return e;
      continue;
    }
    if constexpr (!XB) {
      if (nx * n > 1024) return hipErrorInvalidValue;
      int cs = (int)(65536 / ((size_t)(nx + n) * 12 * sizeof(double2)));
      if (cs < 1) return hipErrorInvalidValue;
      cs = cs > 16 ? 16 : cs;
      size_t lds = (size_t)(nx + n) * cs * 12 * sizeof(double2);
      hipLaunchKernelGGL((k_block_dots<EX, EY>), dim3(d.nblk), dim3(256), lds, st, g, d, X, xvs, nx, Yc, yvs, n, oc,
                         bso, ldo, kys, cs);
    }
  }
  return hipGetLastError();
}

template <class EX, class EY>
hipError_t launch_block_dots(const Geo& g, const DflGeo& d, const EX* X, int64_t xvs, int nx, const EY* Y,
                             int64_t yvs, int ny, double2* out, int64_t bso, int64_t ldo, int64_t kys,
                             hipStream_t st, int face) {
  return block_dots_impl<EX, EY, false>(g, d, X, xvs, nx, Y, yvs, ny, out, bso, ldo, kys, st, face);
}

hipError_t launch_block_dots_xb(const Geo& g, const DflGeo& d, const float2* Xb, int nx, const double2* Y,
                                int64_t yvs, int ny, double2* out, int64_t bso, int64_t ldo, int64_t kys,
                                hipStream_t st) {
  return block_dots_impl<float2, double2, true>(g, d, Xb, 0, nx, Y, yvs, ny, out, bso, ldo, kys, st, 0);
}

bool block_major_ok(const DflGeo& d) { return (d.bs[3] & 1) == 0; }

hipError_t launch_to_blocks(const Geo& g, const DflGeo& d, const double2* W, int64_t vs, int Ns, float2* out,
                            hipStream_t st) {
  if (!block_major_ok(d)) return hipErrorInvalidValue;
  const int64_t n = (int64_t)Ns * 24 * g.Vh;
  hipLaunchKernelGGL((k_to_blocks<float2>), dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)), dim3(256), 0,
                     st, g, d, W, vs, Ns, out);
  return hipGetLastError();
}

template <class EW, class EO>
hipError_t launch_prolong(const Geo& g, const DflGeo& d, const EW* W, int64_t wvs, int Ns, const double2* c,
                          int64_t nc, EO* out, int64_t ovs, int nrhs, hipStream_t st) {
  if (nrhs > 4)
    hipLaunchKernelGGL((k_prolong<EW, EO, 8, 6>), dim3((unsigned)((2 * (int64_t)g.V + 255) / 256)), dim3(256), 0, st,
                       g, d, W, wvs, Ns, c, nc, out, ovs, nrhs);
  else
    hipLaunchKernelGGL((k_prolong<EW, EO, 4, 12>), dim3((g.V + 255) / 256), dim3(256), 0, st, g, d, W, wvs, Ns, c,
                       nc, out, ovs, nrhs);
  return hipGetLastError();
}

hipError_t launch_coarse_apply(const DflGeo& d, const double2* A, int Ns, const double2* in, double2* out,
                               int64_t nc, int nrhs, hipStream_t st) {
  const int ngr = Ns * ((nrhs + 3) / 4);
  const size_t lds = ((size_t)Ns * (Ns + 1) + (size_t)nrhs * Ns) * sizeof(double2);
  if (ngr <= 256 && lds <= 48 * 1024) {
    if (ngr <= 64)
      hipLaunchKernelGGL((k_coarse_apply_lds<1>), dim3(d.nblk), dim3(64), lds, st, d, A, Ns, in, out, nc, nrhs);
    else if (ngr <= 128)
      hipLaunchKernelGGL((k_coarse_apply_lds<2>), dim3(d.nblk), dim3(64), lds, st, d, A, Ns, in, out, nc, nrhs);
    else
      hipLaunchKernelGGL((k_coarse_apply_lds<4>), dim3(d.nblk), dim3(64), lds, st, d, A, Ns, in, out, nc, nrhs);
    return hipGetLastError();
  }
  int64_t tot = (int64_t)nrhs * d.nblk * Ns;
  hipLaunchKernelGGL(k_coarse_apply, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, d, A, Ns, in, out, nc,
                     nrhs);
  return hipGetLastError();
}

template hipError_t launch_block_dots<double2, double2>(const Geo&, const DflGeo&, const double2*, int64_t, int,
                                                        const double2*, int64_t, int, double2*, int64_t, int64_t,
                                                        int64_t, hipStream_t, int);
template hipError_t launch_block_dots<float2, double2>(const Geo&, const DflGeo&, const float2*, int64_t, int,
                                                       const double2*, int64_t, int, double2*, int64_t, int64_t,
                                                       int64_t, hipStream_t, int);
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
