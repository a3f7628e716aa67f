// Clover-Wilson operator kernels (Eq. 1) and the even-odd Schur complement
// Dhat = D_ee - D_eo D_oo^{-1} D_oe (Eq. 2) on gfx950.
//
// Hopping sum H psi(x) = sum_mu [ (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu) ]
// (boundary sign inside the stored links).  With D = A - H/2:
//   pass A (odd sites):  t_o = A_o^{-1} H_oe psi_e
//   pass B (even sites): out_e = A_e psi_e - (1/4) H_eo t_o      = Dhat psi_e
//   full D (both):       out_p = A_p psi_p - (1/2) H_{p,1-p} psi_{1-p}
// A lane handles one site and NR right-hand sides (a link is loaded once and
// applied to all NR spinors); a block holds sb sites times block/sb lane groups
// that take further right-hand sides, so one wavefront can cover several
// right-hand sides of the same sites and fetch each link once for all of them.
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

// block b of nblk (of one parity) -> (site tile, rhs group).
// order 0: linear.  order >= 1: hardware block ids go round-robin over the 8
// XCDs, so every XCD is given a contiguous range of tiles (a slab of the
// lattice whose neighbours share its L2).  order 2 additionally walks the tiles
// of an XCD's slab of L0/8 time slices with the time slice fastest, then x1,
// then the tile within the (x2, x3) row: the time and x1 neighbours of a site
// are then touched within a few tiles, while the lexicographic walk reaches the
// time neighbours only one whole time slice later, after they have left the L2.
__device__ inline void map_block(const Geo& g, int b, int nblk, int nrg, int sb, int order, int& tile, int& rg) {
  if (order >= 1 && (nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  rg = b % nrg;
  tile = b / nrg;
  int row = g.L[2] * g.Lh3;  // sites of one (x0, x1) row of a parity
  if (order == 2 && (g.L[0] & 7) == 0 && row % sb == 0 && (nblk / nrg) * sb == g.Vh) {
    int S = g.L[0] >> 3, tpr = row / sb, per_xcd = S * g.L[1] * tpr;
    int k = tile / per_xcd, t = tile - k * per_xcd;
    int s = t % S, rest = t / S;
    int x1 = rest % g.L[1], qd = rest / g.L[1];
    tile = ((k * S + s) * g.L[1] + x1) * tpr + qd;
  }
}

// lane -> (site i, first rhs r0): sb sites x (blockDim / sb) rhs groups of NR
template <int NR>
__device__ inline bool lane_site(const Geo& g, int tile, int rg, int sb, int nrhs, int& i, int& r0) {
  i = tile * sb + (int)(threadIdx.x % sb);
  r0 = (rg * (int)(blockDim.x / sb) + (int)(threadIdx.x / sb)) * NR;
  return i < g.Vh && r0 < nrhs;
}

template <class S, int NR>
__global__ void __launch_bounds__(256) k_dhat_a(Geo g, LinkV<S> U, CloverV<S> Ai, FieldV<S> in_e, FieldV<S> t_o,
                                                int nrhs, int nrg, int order, int sb) {
  typedef typename St<S>::T T;
  int tile, rg, i, r0;
  map_block(g, blockIdx.x, gridDim.x, nrg, sb, order, tile, rg);
  if (!lane_site<NR>(g, tile, rg, sb, nrhs, i, r0)) return;
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
                                                FieldV<S> out_e, int nrhs, int nrg, int order, int sb) {
  typedef typename St<S>::T T;
  int tile, rg, i, r0;
  map_block(g, blockIdx.x, gridDim.x, nrg, sb, order, tile, rg);
  if (!lane_site<NR>(g, tile, rg, sb, nrhs, i, r0)) return;
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

// full D on both parities; in/out: full fields (parity p at offset p*poff
// elements); the two halves of the grid are walked like two Dhat passes
template <class S, int NR>
__global__ void __launch_bounds__(256) k_dw(Geo g, LinkV<S> U, CloverV<S> A, FieldV<S> in, FieldV<S> out,
                                            int64_t poff, int64_t spoff, int nrhs, int nrg, int order, int sb) {
  typedef typename St<S>::T T;
  int nh = gridDim.x >> 1;
  int p = (int)blockIdx.x >= nh;
  int tile, rg, i, r0;
  map_block(g, blockIdx.x - p * nh, nh, nrg, sb, order, tile, rg);
  if (!lane_site<NR>(g, tile, rg, sb, nrhs, i, r0)) return;
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
                                 int nrhs, const LaunchCfg& c, hipStream_t st, int pass, hipEvent_t ev) {
  int sb = c.sb > 0 ? c.sb : c.block;
  int nrg = ceil_div(nrhs, NR * (c.block / sb));
  int tiles = ceil_div(g.Vh, sb);
  dim3 grid(tiles * nrg), blk(c.block);
  if (pass & 1)
    hipLaunchKernelGGL((k_dhat_a<S, NR>), grid, blk, 0, st, g, op.U, op.Ainv, in, tmp, nrhs, nrg, c.xcd, sb);
  if (ev) hipEventRecord(ev, st);
  if (pass & 2)
    hipLaunchKernelGGL((k_dhat_b<S, NR>), grid, blk, 0, st, g, op.U, op.A, in, tmp, out, nrhs, nrg, c.xcd, sb);
  return hipGetLastError();
}

template <class S>
hipError_t launch_dhat(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> tmp, FieldV<S> out, int nrhs,
                       const LaunchCfg& c, hipStream_t st, int pass, hipEvent_t ev) {
  switch (c.nr) {
    case 1: return launch_dhat_nr<S, 1>(g, op, in, tmp, out, nrhs, c, st, pass, ev);
    case 2: return launch_dhat_nr<S, 2>(g, op, in, tmp, out, nrhs, c, st, pass, ev);
    case 4: return launch_dhat_nr<S, 4>(g, op, in, tmp, out, nrhs, c, st, pass, ev);
    default: return hipErrorInvalidValue;
  }
}

template <class S, int NR>
static hipError_t launch_dw_nr(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> out, int64_t poff,
                               int64_t spoff, int nrhs, const LaunchCfg& c, hipStream_t st) {
  int sb = c.sb > 0 ? c.sb : c.block;
  int nrg = ceil_div(nrhs, NR * (c.block / sb));
  int tiles = 2 * ceil_div(g.Vh, sb);
  hipLaunchKernelGGL((k_dw<S, NR>), dim3(tiles * nrg), dim3(c.block), 0, st, g, op.U, op.A, in, out, poff, spoff,
                     nrhs, nrg, c.xcd, sb);
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

#define INST(S)                                                                                                     \
  template hipError_t launch_dhat<S>(const Geo&, const DevOp<S>&, FieldV<S>, FieldV<S>, FieldV<S>, int,             \
                                     const LaunchCfg&, hipStream_t, int, hipEvent_t);                               \
  template hipError_t launch_dw<S>(const Geo&, const DevOp<S>&, FieldV<S>, FieldV<S>, int64_t, int64_t, int,        \
                                   const LaunchCfg&, hipStream_t);
INST(double)
INST(float)
INST(__half)
#undef INST

}  // namespace qdd
