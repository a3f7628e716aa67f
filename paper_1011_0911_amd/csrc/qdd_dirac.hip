// Clover-Wilson operator kernels (Eq. 1) and the even-odd Schur complement
// Dhat = D_ee - D_eo D_oo^{-1} D_oe (Eq. 2) on gfx950.
//
// Hopping sum H psi(x) = sum_mu [ (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu) ]
// (boundary sign inside the stored links).  With D = A - H/2:
//   pass A (odd sites):  t_o = A_o^{-1} H_oe psi_e
//   pass B (even sites): out_e = A_e psi_e - (1/4) H_eo t_o      = Dhat psi_e
//   full D (both):       out_p = A_p psi_p - (1/2) H_{p,1-p} psi_{1-p}
// One lane per site and NR right-hand sides per lane: a link is loaded once and
// applied to all NR spinors.  Blocks are remapped so that each of the 8 XCDs
// works on one contiguous slab of the lattice (neighbours share its L2).
#include "qdd_kernels.h"

namespace qdd {

template <class S, int MU, int NR>
__device__ inline void hop_dir(const Geo& g, const LinkV<S>& U, const FieldV<S>& in, int r0, int nr, int p, int i,
                               const int x[4], cx<typename St<S>::T> (&acc)[NR][12]) {
  typedef typename St<S>::T T;
  cx<T> u[9], s[12], h[6], gg[6];
  int j = nbr_idx(g, x, MU, +1);
  ld_link(U, p, MU, i, u);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      ld_spinor(in, r0 + q, j, s);
      project<T, MU, +1>(s, h);
      su3_mul_half<T, false>(u, h, gg);
      reconstruct_add<T, MU, +1>(gg, acc[q]);
    }
  }
  j = nbr_idx(g, x, MU, -1);
  ld_link(U, 1 - p, MU, j, u);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      ld_spinor(in, r0 + q, j, s);
      project<T, MU, -1>(s, h);
      su3_mul_half<T, true>(u, h, gg);
      reconstruct_add<T, MU, -1>(gg, acc[q]);
    }
  }
}

template <class S, int NR>
__device__ inline void hop_all(const Geo& g, const LinkV<S>& U, const FieldV<S>& in, int r0, int nr, int p, int i,
                               const int x[4], cx<typename St<S>::T> (&acc)[NR][12]) {
  hop_dir<S, 0, NR>(g, U, in, r0, nr, p, i, x, acc);
  hop_dir<S, 1, NR>(g, U, in, r0, nr, p, i, x, acc);
  hop_dir<S, 2, NR>(g, U, in, r0, nr, p, i, x, acc);
  hop_dir<S, 3, NR>(g, U, in, r0, nr, p, i, x, acc);
}

// block -> (site tile, rhs group), XCD-aware: consecutive hardware block ids go
// round-robin over the 8 XCDs, so give each XCD a contiguous range of tiles.
__device__ inline void map_block(int nblk, int nrg, int xcd_remap, int& tile, int& rg) {
  int b = blockIdx.x;
  if (xcd_remap && (nblk % 8) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  rg = b % nrg;
  tile = b / nrg;
}

template <class S, int NR>
__global__ void __launch_bounds__(256) k_dhat_a(Geo g, LinkV<S> U, CloverV<S> Ai, FieldV<S> in_e, FieldV<S> t_o,
                                                int nrhs, int nrg, int xcd) {
  typedef typename St<S>::T T;
  int tile, rg;
  map_block(gridDim.x, nrg, xcd, tile, rg);
  int i = tile * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  int r0 = rg * NR;
  int nr = min(NR, nrhs - r0);
  int x[4];
  site_coords(g, 1, i, x);
  cx<T> acc[NR][12];
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {T(0), T(0)};
  hop_all<S, NR>(g, U, in_e, r0, nr, 1, i, x, acc);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      cx<T> o[12];
      clover_apply<S>(Ai, 1, i, acc[q], o);
      st_spinor(t_o, r0 + q, i, o);
    }
  }
}

template <class S, int NR>
__global__ void __launch_bounds__(256) k_dhat_b(Geo g, LinkV<S> U, CloverV<S> A, FieldV<S> in_e, FieldV<S> t_o,
                                                FieldV<S> out_e, int nrhs, int nrg, int xcd) {
  typedef typename St<S>::T T;
  int tile, rg;
  map_block(gridDim.x, nrg, xcd, tile, rg);
  int i = tile * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  int r0 = rg * NR;
  int nr = min(NR, nrhs - r0);
  int x[4];
  site_coords(g, 0, i, x);
  cx<T> acc[NR][12];
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {T(0), T(0)};
  hop_all<S, NR>(g, U, t_o, r0, nr, 0, i, x, acc);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      cx<T> s[12], o[12];
      ld_spinor(in_e, r0 + q, i, s);
      clover_apply<S>(A, 0, i, s, o);
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = o[k] - T(0.25) * acc[q][k];
      st_spinor(out_e, r0 + q, i, o);
    }
  }
}

// full D on both parities; in/out: full fields (parity p at offset p*poff elements)
template <class S, int NR>
__global__ void __launch_bounds__(256) k_dw(Geo g, LinkV<S> U, CloverV<S> A, FieldV<S> in, FieldV<S> out,
                                            int64_t poff, int64_t spoff, int nrhs, int nrg, int xcd) {
  typedef typename St<S>::T T;
  int tile, rg;
  map_block(gridDim.x, nrg, xcd, tile, rg);
  int tiles_per_parity = (g.Vh + blockDim.x - 1) / blockDim.x;
  int p = tile >= tiles_per_parity;
  int i = (tile - p * tiles_per_parity) * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  int r0 = rg * NR;
  int nr = min(NR, nrhs - r0);
  int x[4];
  site_coords(g, p, i, x);
  FieldV<S> src = in, self = in, dst = out;
  src.p += (1 - p) * poff;
  self.p += p * poff;
  dst.p += p * poff;
  if (src.scale) {
    src.scale += (1 - p) * spoff;
    self.scale += p * spoff;
    dst.scale += p * spoff;
  }
  cx<T> acc[NR][12];
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {T(0), T(0)};
  hop_all<S, NR>(g, U, src, r0, nr, p, i, x, acc);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      cx<T> s[12], o[12];
      ld_spinor(self, r0 + q, i, s);
      clover_apply<S>(A, p, i, s, o);
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = o[k] - T(0.5) * acc[q][k];
      st_spinor(dst, r0 + q, i, o);
    }
  }
}

// ----------------------------------------------------------------- launchers
static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

template <class S, int NR>
static hipError_t launch_dhat_nr(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> tmp, FieldV<S> out,
                                 int nrhs, const LaunchCfg& c, hipStream_t st) {
  int nrg = ceil_div(nrhs, NR);
  int tiles = ceil_div(g.Vh, c.block);
  dim3 grid(tiles * nrg), blk(c.block);
  hipLaunchKernelGGL((k_dhat_a<S, NR>), grid, blk, 0, st, g, op.U, op.Ainv, in, tmp, nrhs, nrg, c.xcd);
  hipLaunchKernelGGL((k_dhat_b<S, NR>), grid, blk, 0, st, g, op.U, op.A, in, tmp, out, nrhs, nrg, c.xcd);
  return hipGetLastError();
}

template <class S>
hipError_t launch_dhat(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> tmp, FieldV<S> out, int nrhs,
                       const LaunchCfg& c, hipStream_t st) {
  switch (c.nr) {
    case 1: return launch_dhat_nr<S, 1>(g, op, in, tmp, out, nrhs, c, st);
    case 2: return launch_dhat_nr<S, 2>(g, op, in, tmp, out, nrhs, c, st);
    case 4: return launch_dhat_nr<S, 4>(g, op, in, tmp, out, nrhs, c, st);
    default: return hipErrorInvalidValue;
  }
}

template <class S, int NR>
static hipError_t launch_dw_nr(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> out, int64_t poff,
                               int64_t spoff, int nrhs, const LaunchCfg& c, hipStream_t st) {
  int nrg = ceil_div(nrhs, NR);
  int tiles = 2 * ceil_div(g.Vh, c.block);
  hipLaunchKernelGGL((k_dw<S, NR>), dim3(tiles * nrg), dim3(c.block), 0, st, g, op.U, op.A, in, out, poff, spoff,
                     nrhs, nrg, c.xcd);
  return hipGetLastError();
}

template <class S>
hipError_t launch_dw(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> out, int64_t poff, int64_t spoff,
                     int nrhs, const LaunchCfg& c, hipStream_t st) {
  switch (c.nr) {
    case 1: return launch_dw_nr<S, 1>(g, op, in, out, poff, spoff, nrhs, c, st);
    case 2: return launch_dw_nr<S, 2>(g, op, in, out, poff, spoff, nrhs, c, st);
    case 4: return launch_dw_nr<S, 4>(g, op, in, out, poff, spoff, nrhs, c, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_dhat<double>(const Geo&, const DevOp<double>&, FieldV<double>, FieldV<double>,
                                        FieldV<double>, int, const LaunchCfg&, hipStream_t);
template hipError_t launch_dhat<float>(const Geo&, const DevOp<float>&, FieldV<float>, FieldV<float>, FieldV<float>,
                                       int, const LaunchCfg&, hipStream_t);
template hipError_t launch_dhat<__half>(const Geo&, const DevOp<__half>&, FieldV<__half>, FieldV<__half>,
                                        FieldV<__half>, int, const LaunchCfg&, hipStream_t);
template hipError_t launch_dw<double>(const Geo&, const DevOp<double>&, FieldV<double>, FieldV<double>, int64_t,
                                      int64_t, int, const LaunchCfg&, hipStream_t);
template hipError_t launch_dw<float>(const Geo&, const DevOp<float>&, FieldV<float>, FieldV<float>, int64_t, int64_t,
                                     int, const LaunchCfg&, hipStream_t);
template hipError_t launch_dw<__half>(const Geo&, const DevOp<__half>&, FieldV<__half>, FieldV<__half>, int64_t,
                                      int64_t, int, const LaunchCfg&, hipStream_t);

}  // namespace qdd
