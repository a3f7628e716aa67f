// Dirichlet block solves D_Lambda psi = eta on every block of the lattice (the
// block inversions of the DD-HMC forces, which the paper does with BiCGstab,
// Sect. 3), FP64, on gfx950.
//
// Every block is an independent system, so one workgroup takes one (block,
// right-hand side) and runs the whole solve: the source is reduced to the
// block's even sites, b = eta_e - D_eo,L A_o^{-1} eta_o, BiCGstab (van der Vorst)
// on Dhat_Lambda = A_e - D_eo,L A_o^{-1} D_oe,L iterates until |r| <= tol |b| or
// maxit, and psi_o = A_o^{-1}(eta_o - D_oe,L psi_e) is reconstructed.  Inner
// products are reduced inside the workgroup (fixed order: deterministic), so a
// solve is one launch with no host synchronisation between iterations.  The
// links and clover blocks are first gathered into a block-major layout (the
// sites of one block and parity contiguous, block-local lexicographic order),
// so every pass over a block reads contiguous memory; hops that leave the block
// are dropped (D_Lambda is D restricted to the block).
#include "qdd_kernels.h"

namespace qdd {

typedef cx<double> zd;

// block-local coordinates y of the site with block-local index ql and parity p
// (the block origin has even coordinates: block-local and global parity agree)
__device__ inline void blk_coords(const BlkGeo& B, int p, int ql, int y[4]) {
  const int h3 = B.bs[3] >> 1;
  const int row = ql / h3, h = ql - row * h3;
  y[2] = row % B.bs[2];
  const int t = row / B.bs[2];
  y[1] = t % B.bs[1];
  y[0] = t / B.bs[1];
  y[3] = 2 * h + ((p + y[0] + y[1] + y[2]) & 1);
}
__device__ inline int blk_local(const BlkGeo& B, const int y[4]) {
  return (((y[0] * B.bs[1] + y[1]) * B.bs[2] + y[2]) * B.bs[3] + y[3]) >> 1;
}
// global coordinates of block b's site with local coordinates y
__device__ inline void blk_global(const BlkGeo& B, int b, const int y[4], int x[4]) {
  int c = b;
  x[3] = (c % B.nb[3]) * B.bs[3] + y[3];
  c /= B.nb[3];
  x[2] = (c % B.nb[2]) * B.bs[2] + y[2];
  c /= B.nb[2];
  x[1] = (c % B.nb[1]) * B.bs[1] + y[1];
  x[0] = (c / B.nb[1]) * B.bs[0] + y[0];
}

// links and clover blocks (both parities) into the block-major layout: entry q
// = b * neb + local index of the parity-p site takes the site's lattice index
__global__ void k_blk_gather(Geo g, BlkGeo B, const double2* U, const double2* A, const double2* Ai, double2* BU,
                             double2* BA, double2* BAi) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= g.V) return;
  const int p = tid >= g.Vh, q = tid - p * g.Vh;
  const int b = q / B.neb, ql = q - b * B.neb;
  int y[4], x[4];
  blk_coords(B, p, ql, y);
  blk_global(B, b, y, x);
  const int64_t i = lex_of(g, x) >> 1, n = g.Vh;
  for (int k = 0; k < 36; ++k) BU[(p * 36 + k) * n + q] = U[(p * 36 + k) * n + i];  // [p][mu][9]
  for (int k = 0; k < 36; ++k) {
    BA[(p * 36 + k) * n + q] = A[(p * 36 + k) * n + i];
    BAi[(p * 36 + k) * n + q] = Ai[(p * 36 + k) * n + i];
  }
}

// acc += c0 H_Lambda f at the parity-p site q (local coordinates y) of block b
template <int MU, int SG>
__device__ inline void blk_hop_dir(const BlkGeo& B, const LinkV<double>& U, const FieldV<double>& f, int b, int p, int q,
                                   const int y[4], double c0, zd (&acc)[12]) {
  const bool inside = SG > 0 ? y[MU] + 1 < B.bs[MU] : y[MU] > 0;
  if (!inside) return;
  int yn[4] = {y[0], y[1], y[2], y[3]};
  yn[MU] += SG;
  const int qn = b * B.neb + blk_local(B, yn);
  zd u[9], s[12], h[6], gg[6];
  if (SG > 0) ld_link_u<double>(U, p, MU, q, u);
  else ld_link_u<double>(U, 1 - p, MU, qn, u);
  ld_spinor<double, true>(f, 0, qn, s);
  project<double, MU, SG>(s, h);
  su3_mul_half<double, (SG < 0)>(u, h, gg);
  reconstruct_add<double, MU, SG>(gg, acc, c0);
}
__device__ inline void blk_hop(const BlkGeo& B, const LinkV<double>& U, const FieldV<double>& f, int b, int p, int q,
                               const int y[4], double c0, zd (&acc)[12]) {
  // scheduling barriers bound the loads in flight (and so the registers)
  blk_hop_dir<0, 1>(B, U, f, b, p, q, y, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  blk_hop_dir<0, -1>(B, U, f, b, p, q, y, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  blk_hop_dir<1, 1>(B, U, f, b, p, q, y, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  blk_hop_dir<1, -1>(B, U, f, b, p, q, y, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  blk_hop_dir<2, 1>(B, U, f, b, p, q, y, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  blk_hop_dir<2, -1>(B, U, f, b, p, q, y, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  blk_hop_dir<3, 1>(B, U, f, b, p, q, y, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  blk_hop_dir<3, -1>(B, U, f, b, p, q, y, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
}

// sum of v[0..N) over the workgroup (wavefront shuffles, then the per-wavefront
// partials in wavefront order); every thread gets the sums
template <int N>
__device__ inline void wg_sum(double (&v)[N], double* lds) {
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) lds[wave * N + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[w * N + k];
    v[k] = s;
  }
  __syncthreads();
}

__device__ inline zd cdiv(zd a, zd b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// component k of a vector at block-major site q (wave-uniform base, 32-bit
// offset: the component bases stay in scalar registers)
__device__ inline zd ldc(const FieldV<double>& f, int k, int q) {
  const double2 v = ld_off<double2>(f.p + (int64_t)k * f.n, (uint32_t)q * 16u);
  return {v.x, v.y};
}
__device__ inline void stc(const FieldV<double>& f, int k, int q, zd v) {
  st_off<double2>(f.p + (int64_t)k * f.n, (uint32_t)q * 16u, make_double2(v.re, v.im));
}

__device__ inline FieldV<double> vec_of(double2* base, int k, int Vh) {
  return FieldV<double>{base + (int64_t)k * 12 * Vh, nullptr, (int64_t)12 * Vh, (int64_t)Vh, Vh};
}

// one workgroup per (block, right-hand side); work: per rhs 8 vectors [12][Vh]
// (x, r, rh, p, v, s, t on the even sites, w the odd-site intermediate)
__global__ void __launch_bounds__(512) k_blk_bicgstab(Geo g, BlkGeo B, LinkV<double> BU, CloverV<double> BA,
                                                      CloverV<double> BAi, double2* work, const double2* eta,
                                                      double2* psi, double tol, int maxit, int* iters, double* res) {
  __shared__ double red[8 * 4];
  const int b = blockIdx.x, rr = blockIdx.y;  // grid (blocks, rhs): both scalar
  const int nt = blockDim.x, neb = B.neb, q0 = b * neb;
  double2* base = work + (int64_t)rr * 8 * 12 * g.Vh;
  const FieldV<double> X = vec_of(base, 0, g.Vh), R = vec_of(base, 1, g.Vh), RH = vec_of(base, 2, g.Vh),
                       P = vec_of(base, 3, g.Vh), Vv = vec_of(base, 4, g.Vh), Sv = vec_of(base, 5, g.Vh),
                       Tv = vec_of(base, 6, g.Vh), W = vec_of(base, 7, g.Vh);
  const double2* et = eta + (int64_t)rr * g.V * 12;
  double2* ps = psi + (int64_t)rr * g.V * 12;
  auto ld_can = [&](const double2* f, const int x[4], zd s[12]) {
    const double2* a = f + (int64_t)lex_of(g, x) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = {a[k].x, a[k].y};
  };
  auto st_can = [&](double2* f, const int x[4], const zd s[12]) {
    double2* a = f + (int64_t)lex_of(g, x) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = make_double2(s[k].re, s[k].im);
  };
  // pass A of Dhat_Lambda: W_o = A_o^{-1} H_Lambda in
  auto pass_a = [&](const FieldV<double>& in) {
    for (int ql = threadIdx.x; ql < neb; ql += nt) {
      int y[4];
      blk_coords(B, 1, ql, y);
      zd acc[12], o[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = {0.0, 0.0};
      blk_hop(B, BU, in, b, 1, q0 + ql, y, 1.0, acc);
      clover_apply_u<double>(BAi, 1, q0 + ql, acc, o);
      st_spinor<double, true>(W, 0, q0 + ql, o);
    }
    __syncthreads();
  };
  // pass B at one even site: out = A_e in - 1/4 H_Lambda W_o
  auto dhat_site = [&](const FieldV<double>& in, int ql, zd o[12]) {
    int y[4];
    blk_coords(B, 0, ql, y);
    zd acc[12], s[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {0.0, 0.0};
    blk_hop(B, BU, W, b, 0, q0 + ql, y, -0.25, acc);
    ld_spinor<double, true>(in, 0, q0 + ql, s);
    clover_apply_u<double>(BA, 0, q0 + ql, s, o);
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = o[k] + acc[k];
  };

  // reduced source b = eta_e + 1/2 H_Lambda (A_o^{-1} eta_o); r = rh = b; x = p = v = 0
  for (int ql = threadIdx.x; ql < neb; ql += nt) {
    int y[4], x[4];
    blk_coords(B, 1, ql, y);
    blk_global(B, b, y, x);
    zd e[12], o[12];
    ld_can(et, x, e);
    clover_apply_u<double>(BAi, 1, q0 + ql, e, o);
    st_spinor<double, true>(W, 0, q0 + ql, o);
  }
  __syncthreads();
  double acc1[1] = {0.0};
  for (int ql = threadIdx.x; ql < neb; ql += nt) {
    int y[4], x[4];
    blk_coords(B, 0, ql, y);
    blk_global(B, b, y, x);
    zd e[12], z[12];
    ld_can(et, x, e);
    blk_hop(B, BU, W, b, 0, q0 + ql, y, 0.5, e);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      z[k] = {0.0, 0.0};
      acc1[0] += e[k].re * e[k].re + e[k].im * e[k].im;
    }
    st_spinor<double, true>(R, 0, q0 + ql, e);
    st_spinor<double, true>(RH, 0, q0 + ql, e);
    st_spinor<double, true>(X, 0, q0 + ql, z);
    st_spinor<double, true>(P, 0, q0 + ql, z);
    st_spinor<double, true>(Vv, 0, q0 + ql, z);
  }
  wg_sum<1>(acc1, red);
  const double bn2 = acc1[0];
  zd rho{1.0, 0.0}, alpha{1.0, 0.0}, omega{1.0, 0.0}, rho_new{bn2, 0.0};
  double rn2 = bn2;
  int it = 0;
  bool broke = false;
  while (rn2 > tol * tol * bn2 && it < maxit) {
    const zd beta = cdiv(rho_new, rho) * cdiv(alpha, omega);
    // p = r + beta (p - omega v)
    for (int ql = threadIdx.x; ql < neb; ql += nt)
#pragma unroll 4
      for (int k = 0; k < 12; ++k) {
        const int q = q0 + ql;
        stc(P, k, q, ldc(R, k, q) + beta * (ldc(P, k, q) - omega * ldc(Vv, k, q)));
      }
    __syncthreads();
    // v = Dhat_L p, (rh, v)
    pass_a(P);
    double d1[2] = {0.0, 0.0};
    for (int ql = threadIdx.x; ql < neb; ql += nt) {
      zd o[12];
      dhat_site(P, ql, o);
      st_spinor<double, true>(Vv, 0, q0 + ql, o);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const zd h = ldc(RH, k, q0 + ql);
        d1[0] += h.re * o[k].re + h.im * o[k].im;
        d1[1] += h.re * o[k].im - h.im * o[k].re;
      }
    }
    wg_sum<2>(d1, red);
    if (d1[0] == 0.0 && d1[1] == 0.0) {
      broke = true;
      break;
    }
    alpha = cdiv(rho_new, zd{d1[0], d1[1]});
    // s = r - alpha v
    for (int ql = threadIdx.x; ql < neb; ql += nt)
#pragma unroll 4
      for (int k = 0; k < 12; ++k) {
        const int q = q0 + ql;
        stc(Sv, k, q, ldc(R, k, q) - alpha * ldc(Vv, k, q));
      }
    __syncthreads();
    // t = Dhat_L s, (t, s), (t, t)
    pass_a(Sv);
    double d2[3] = {0.0, 0.0, 0.0};
    for (int ql = threadIdx.x; ql < neb; ql += nt) {
      zd o[12];
      dhat_site(Sv, ql, o);
      st_spinor<double, true>(Tv, 0, q0 + ql, o);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const zd sk = ldc(Sv, k, q0 + ql);
        d2[0] += o[k].re * sk.re + o[k].im * sk.im;
        d2[1] += o[k].re * sk.im - o[k].im * sk.re;
        d2[2] += o[k].re * o[k].re + o[k].im * o[k].im;
      }
    }
    wg_sum<3>(d2, red);
    if (d2[2] == 0.0) {
      broke = true;
      break;
    }
    omega = zd{d2[0] / d2[2], d2[1] / d2[2]};
    // x += alpha p + omega s, r = s - omega t; (rh, r), |r|^2
    double d3[3] = {0.0, 0.0, 0.0};
    for (int ql = threadIdx.x; ql < neb; ql += nt)
#pragma unroll 4
      for (int k = 0; k < 12; ++k) {
        const int q = q0 + ql;
        const zd sk = ldc(Sv, k, q), h = ldc(RH, k, q);
        stc(X, k, q, ldc(X, k, q) + alpha * ldc(P, k, q) + omega * sk);
        const zd r = sk - omega * ldc(Tv, k, q);
        stc(R, k, q, r);
        d3[0] += h.re * r.re + h.im * r.im;
        d3[1] += h.re * r.im - h.im * r.re;
        d3[2] += r.re * r.re + r.im * r.im;
      }
    wg_sum<3>(d3, red);
    rho = rho_new;
    rho_new = zd{d3[0], d3[1]};
    rn2 = d3[2];
    ++it;
  }
  // psi_e = x; psi_o = A_o^{-1} (eta_o + 1/2 H_Lambda x)
  for (int ql = threadIdx.x; ql < neb; ql += nt) {
    int y[4], x[4];
    blk_coords(B, 0, ql, y);
    blk_global(B, b, y, x);
    zd s[12];
    ld_spinor<double, true>(X, 0, q0 + ql, s);
    st_can(ps, x, s);
  }
  for (int ql = threadIdx.x; ql < neb; ql += nt) {
    int y[4], x[4];
    blk_coords(B, 1, ql, y);
    blk_global(B, b, y, x);
    zd e[12], o[12];
    ld_can(et, x, e);
    blk_hop(B, BU, X, b, 1, q0 + ql, y, 0.5, e);
    clover_apply_u<double>(BAi, 1, q0 + ql, e, o);
    st_can(ps, x, o);
  }
  if (threadIdx.x == 0) {
    iters[rr * B.nblk + b] = broke ? -1 : it;
    res[rr * B.nblk + b] = bn2 > 0 ? sqrt(rn2 / bn2) : 0.0;
  }
}

hipError_t launch_blk_gather(const Geo& g, const BlkGeo& B, const double2* U, const double2* A, const double2* Ai,
                             double2* BU, double2* BA, double2* BAi, hipStream_t st) {
  hipLaunchKernelGGL(k_blk_gather, dim3((g.V + 255) / 256), dim3(256), 0, st, g, B, U, A, Ai, BU, BA, BAi);
  return hipGetLastError();
}

hipError_t launch_blk_bicgstab(const Geo& g, const BlkGeo& B, const double2* BU, const double2* BA,
                               const double2* BAi, double2* work, const double2* eta, double2* psi, int nrhs,
                               double tol, int maxit, int* iters, double* res, hipStream_t st) {
  const int nt = B.neb >= 512 ? 512 : (B.neb + 63) / 64 * 64;
  hipLaunchKernelGGL(k_blk_bicgstab, dim3(B.nblk, nrhs), dim3(nt), 0, st, g, B, LinkV<double>{BU, g.Vh},
                     CloverV<double>{BA, g.Vh}, CloverV<double>{BAi, g.Vh}, work, eta, psi, tol, maxit, iters, res);
  return hipGetLastError();
}

}  // namespace qdd
