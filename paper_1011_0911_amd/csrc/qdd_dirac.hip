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

// COMP: links read as their first two rows (the third rebuilt, with the time
// boundary sign of the stored link)
template <class S, int MU, int NR, bool O32, bool NT = false, bool COMP = false>
__device__ inline void hop_dir(const Geo& g, const LinkV<S>& U, const FieldV<S>& in, int r0, int nr, int p, int i,
                               const int x[4], typename St<S>::T c0, cx<typename St<S>::T> (&acc)[NR][12]) {
  typedef typename St<S>::T T;
  cx<T> u[9], s[12], h[6], gg[6];
  int j = nbr_idx(g, x, MU, +1);
  if constexpr (COMP) ld_link_u12<S, NT>(U, p, MU, i, T(MU == 0 && x[0] == g.L[0] - 1 ? g.bc : 1), u);
  else ld_link_u<S, NT>(U, p, MU, i, u);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      T sc = ld_spinor_raw<S, O32>(in, r0 + q, j, s);
      project<T, MU, +1>(s, h);
      su3_mul_half<T, false>(u, h, gg);
      reconstruct_add<T, MU, +1>(gg, acc[q], c0 * sc);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  j = nbr_idx(g, x, MU, -1);
  if constexpr (COMP) ld_link_u12<S, NT>(U, 1 - p, MU, j, T(MU == 0 && x[0] == 0 ? g.bc : 1), u);
  else ld_link_u<S, NT>(U, 1 - p, MU, j, u);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      T sc = ld_spinor_raw<S, O32>(in, r0 + q, j, s);
      project<T, MU, -1>(s, h);
      su3_mul_half<T, true>(u, h, gg);
      reconstruct_add<T, MU, -1>(gg, acc[q], c0 * sc);
    }
  }
}

// acc += c0 H in (H: the hopping sum over the 8 neighbours); NT: links are
// read with streaming loads (each is read once per pass); COMP: see hop_dir
template <class S, int NR, bool O32, bool NT = false, bool COMP = false>
__device__ inline void hop_all(const Geo& g, const LinkV<S>& U, const FieldV<S>& in, int r0, int nr, int p, int i,
                               const int x[4], typename St<S>::T c0, cx<typename St<S>::T> (&acc)[NR][12]) {
  // scheduling barriers between the directions bound the number of loads in
  // flight per lane (and so the registers); the other waves hide the latency
  hop_dir<S, 0, NR, O32, NT, COMP>(g, U, in, r0, nr, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_dir<S, 1, NR, O32, NT, COMP>(g, U, in, r0, nr, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_dir<S, 2, NR, O32, NT, COMP>(g, U, in, r0, nr, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_dir<S, 3, NR, O32, NT, COMP>(g, U, in, r0, nr, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
}

// block b of nblk (of one parity) -> (site tile, rhs group).
// order 0: linear.  order >= 1: hardware block ids go round-robin over the 8
// XCDs, so every XCD is given a contiguous range of tiles (a slab of the
// lattice whose neighbours share its L2).  order 1: slabs of L0/8 time slices
// walked lexicographically.  order 2: the same slabs walked with the time slice
// fastest, then x1, then the tile within the (x2, x3) row: the time and x1
// neighbours of a site are then touched within a few tiles, while the
// lexicographic walk reaches the time neighbours only one whole time slice
// later, after they have left the L2.  order 3: slabs of L1/8 x1 planes
// (through all time slices), walked one time slice after the other, row by
// row: a step (one time slice of the slab) touches its own spinors and those of
// the two neighbouring steps, which stay in the XCD's L2; only the x1 faces of
// the slab reach into the slabs of other XCDs.
// order + 4: the walk runs backwards (every XCD's range from its end), so a
// pass that reads what the previous pass wrote starts with the most recently
// written data, which the memory-side cache may still hold.
__device__ inline void map_block(const Geo& g, int b, int nblk, int nrg, int sb, int order, int& tile, int& rg) {
  const bool rev = (order & 4) != 0;
  order &= 3;
  if (order >= 1 && (nblk & 7) == 0) {
    const int per = nblk >> 3, j = b >> 3;
    b = (b & 7) * per + (rev ? per - 1 - j : j);
  } else if (rev) {
    b = nblk - 1 - b;
  }
  rg = b % nrg;
  tile = b / nrg;
  const int row = g.L[2] * g.Lh3;  // sites of one (x0, x1) row of a parity
  if (row % sb != 0 || (nblk / nrg) * sb != g.Vh) return;
  const int tpr = row / sb;
  if (order == 2 && (g.L[0] & 7) == 0) {
    const int S = g.L[0] >> 3, per_xcd = S * g.L[1] * tpr;
    const int k = tile / per_xcd, t = tile - k * per_xcd;
    const int s = t % S, rest = t / S;
    const int x1 = rest % g.L[1], qd = rest / g.L[1];
    tile = ((k * S + s) * g.L[1] + x1) * tpr + qd;
  } else if (order == 3 && (g.L[1] & 7) == 0) {
    const int X = g.L[1] >> 3, per_xcd = g.L[0] * X * tpr;
    const int k = tile / per_xcd, t = tile - k * per_xcd;
    const int qd = t % tpr, rest = t / tpr;
    const int x1l = rest % X, x0 = rest / X;
    tile = (x0 * g.L[1] + k * X + x1l) * tpr + qd;
  }
}

// lane -> (site i, first rhs r0): sb sites x G = blockDim / sb rhs groups of NR;
// site fastest for the blocked field layout, rhs group fastest (rf) for the
// interleaved one, so that a wavefront reads contiguous memory in both
template <int NR>
__device__ inline bool lane_site(const Geo& g, int tile, int rg, int sb, int nrhs, int rf, int& i, int& r0) {
  const int G = (int)(blockDim.x / sb), t = (int)threadIdx.x;
  const int sl = rf ? t / G : t % sb, gl = rf ? t % G : t / sb;
  i = tile * sb + sl;
  r0 = (rg * G + gl) * NR;
  return i < g.Vh && r0 < nrhs;
}

// NTM: streaming (non-temporal) access for what the pass touches once; bit 0
// the links and clover blocks, bit 1 the site's own spinor and the output.  The
// neighbour spinors, which eight sites read, always take ordinary loads.  Bit 2:
// compressed links (two rows read, the third rebuilt).
template <class S, int NR, bool O32, int NTM>
__global__ void __launch_bounds__(256, NR == 1 ? (sizeof(S) == 8 ? 2 : 4) : 1) k_dhat_a(Geo g, LinkV<S> U, CloverV<S> Ai, FieldV<S> in_e, FieldV<S> t_o,
                                                int nrhs, int nrg, int order, int sb, int rf) {
  typedef typename St<S>::T T;
  int tile, rg, i, r0;
  map_block(g, blockIdx.x, gridDim.x, nrg, sb, order, tile, rg);
  if (!lane_site<NR>(g, tile, rg, sb, nrhs, rf, i, r0)) return;
  int nr = min(NR, nrhs - r0);
  int x[4];
  site_coords(g, 1, i, x);
  cx<T> acc[NR][12];
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {T(0), T(0)};
  hop_all<S, NR, O32, (NTM & 1) != 0, (NTM & 4) != 0>(g, U, in_e, r0, nr, 1, i, x, T(1), acc);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      cx<T> o[12];
      clover_apply_u<S, (NTM & 1) != 0>(Ai, 1, i, acc[q], o);
      st_spinor<S, O32, (NTM & 2) != 0>(t_o, r0 + q, i, o);
    }
  }
}

template <class S, int NR, bool O32, int NTM>
__global__ void __launch_bounds__(256, NR == 1 ? (sizeof(S) == 8 ? 2 : 4) : 1) k_dhat_b(Geo g, LinkV<S> U, CloverV<S> A, FieldV<S> in_e, FieldV<S> t_o,
                                                FieldV<S> out_e, int nrhs, int nrg, int order, int sb, int rf) {
  typedef typename St<S>::T T;
  int tile, rg, i, r0;
  map_block(g, blockIdx.x, gridDim.x, nrg, sb, order, tile, rg);
  if (!lane_site<NR>(g, tile, rg, sb, nrhs, rf, i, r0)) return;
  int nr = min(NR, nrhs - r0);
  int x[4];
  site_coords(g, 0, i, x);
  // acc = -1/4 H t_o, then out = A_e psi_e + acc
  cx<T> acc[NR][12];
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {T(0), T(0)};
  hop_all<S, NR, O32, (NTM & 1) != 0, (NTM & 4) != 0>(g, U, t_o, r0, nr, 0, i, x, T(-0.25), acc);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      cx<T> s[12], o[12];
      T sc = ld_spinor_raw<S, O32, (NTM & 2) != 0>(in_e, r0 + q, i, s);
      clover_apply_u<S, (NTM & 1) != 0>(A, 0, i, s, o);
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = cacc(acc[q][k], sc, o[k]);
      st_spinor<S, O32, (NTM & 2) != 0>(out_e, r0 + q, i, o);
    }
  }
}

// --------------------------------------------- rhs-vector variant of the passes
// For batches in the interleaved layout (rhs stride one element) a lane takes
// one site and V consecutive right-hand sides: each spinor component of the V
// is one V*sizeof(E)-byte load (16 bytes for V = 4 in FP16), their FP16 scales
// one more, and every link and clover element is loaded once per lane for all
// V.  Lanes are (site, rhs group) with the group fastest, so each load of a
// wavefront covers one contiguous run of memory.  The per-rhs arithmetic is
// that of the kernels above, in the same order.  The host guarantees rhs
// stride 1 (elements and scales), nrhs % V == 0, site strides and component
// strides that are multiples of V, V*sizeof(E)-aligned bases and 32-bit offsets.
template <class S, int V>
struct alignas(V * sizeof(typename St<S>::E)) VecE {
  typename St<S>::E e[V];
};
template <int V>
struct alignas(4 * V) VecF {
  float e[V];
};

template <class S, int V, bool NT>
__device__ inline void ld_spinor_v(const FieldV<S>& f, uint32_t eo, uint32_t so, VecE<S, V> (&raw)[12],
                                   typename St<S>::T (&sc)[V]) {
  typedef VecE<S, V> W;
  const uint32_t vo = eo * (uint32_t)sizeof(typename St<S>::E);
#pragma unroll
  for (int k = 0; k < 12; ++k) raw[k] = ld_off<W, NT>(reinterpret_cast<const W*>(f.p + (int64_t)k * f.n), vo);
  if constexpr (sizeof(S) == 2) {
    VecF<V> w = ld_off<VecF<V>, NT>(reinterpret_cast<const VecF<V>*>(f.scale), so * 4u);
#pragma unroll
    for (int q = 0; q < V; ++q) sc[q] = w.e[q];
  } else {
#pragma unroll
    for (int q = 0; q < V; ++q) sc[q] = typename St<S>::T(1);
  }
}

template <class S, int V, bool NT>
__device__ inline void st_spinor_v(const FieldV<S>& f, uint32_t eo, uint32_t so,
                                   const cx<typename St<S>::T> (&o)[V][12]) {
  typedef VecE<S, V> W;
  const uint32_t vo = eo * (uint32_t)sizeof(typename St<S>::E);
  W w[12];
  if constexpr (sizeof(S) == 2) {
    VecF<V> scs;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      float m = 0.f;
#pragma unroll
      for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(o[q][k].re), fabsf(o[q][k].im)));
      const float sc = m > 0.f ? m : 1.f;
      const float inv = 1.f / sc;
      scs.e[q] = sc;
#pragma unroll
      for (int k = 0; k < 12; ++k) w[k].e[q] = St<S>::to(cx<float>{o[q][k].re * inv, o[q][k].im * inv});
    }
    st_off<VecF<V>, NT>(reinterpret_cast<VecF<V>*>(f.scale), so * 4u, scs);
  } else {
#pragma unroll
    for (int q = 0; q < V; ++q)
#pragma unroll
      for (int k = 0; k < 12; ++k) w[k].e[q] = St<S>::to(o[q][k]);
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) st_off<W, NT>(reinterpret_cast<W*>(f.p + (int64_t)k * f.n), vo, w[k]);
}

// one neighbour (direction MU, SG = +1 forward, -1 backward) for all V
template <class S, int V, int MU, int SG, bool NTL, bool COMP>
__device__ inline void hop_one_v(const Geo& g, const LinkV<S>& U, const FieldV<S>& in, int r0, int p, int i,
                                 const int x[4], typename St<S>::T c0, cx<typename St<S>::T> (&acc)[V][12]) {
  typedef typename St<S>::T T;
  cx<T> u[9];
  VecE<S, V> raw[12];
  T sc[V];
  const int j = nbr_idx(g, x, MU, SG);
  const int par = SG > 0 ? p : 1 - p, li = SG > 0 ? i : j;
  if constexpr (COMP) {
    const bool edge = MU == 0 && x[0] == (SG > 0 ? g.L[0] - 1 : 0);
    ld_link_u12<S, NTL>(U, par, MU, li, T(edge ? g.bc : 1), u);
  } else {
    ld_link_u<S, NTL>(U, par, MU, li, u);
  }
  ld_spinor_v<S, V, false>(in, (uint32_t)((int64_t)j * in.ss + r0), (uint32_t)((int64_t)j * in.sss + r0), raw, sc);
#pragma unroll
  for (int q = 0; q < V; ++q) {
    cx<T> s[12], h[6], gg[6];
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = St<S>::from_reg(raw[k].e[q]);
    project<T, MU, SG>(s, h);
    su3_mul_half<T, (SG < 0)>(u, h, gg);
    reconstruct_add<T, MU, SG>(gg, acc[q], c0 * sc[q]);
  }
}

template <class S, int V, bool NTL, bool COMP>
__device__ inline void hop_all_v(const Geo& g, const LinkV<S>& U, const FieldV<S>& in, int r0, int p, int i,
                                 const int x[4], typename St<S>::T c0, cx<typename St<S>::T> (&acc)[V][12]) {
  hop_one_v<S, V, 0, +1, NTL, COMP>(g, U, in, r0, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_one_v<S, V, 0, -1, NTL, COMP>(g, U, in, r0, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_one_v<S, V, 1, +1, NTL, COMP>(g, U, in, r0, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_one_v<S, V, 1, -1, NTL, COMP>(g, U, in, r0, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_one_v<S, V, 2, +1, NTL, COMP>(g, U, in, r0, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_one_v<S, V, 2, -1, NTL, COMP>(g, U, in, r0, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_one_v<S, V, 3, +1, NTL, COMP>(g, U, in, r0, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_one_v<S, V, 3, -1, NTL, COMP>(g, U, in, r0, p, i, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
}

// The raw operands of one neighbour (link rows and the V spinors with their
// scales), loaded one neighbour ahead of their use: the loads of the next
// neighbour are in flight while the current one is computed.  Same arithmetic
// as hop_one_v.
template <class S, int V>
struct HopRaw {
  typename St<S>::E u[9];
  VecE<S, V> s[12];
  VecF<V> sc;
};

template <class S, int V, int MU, int SG, bool NTL, bool COMP>
__device__ inline void hop_load_v(const Geo& g, const LinkV<S>& U, const FieldV<S>& in, int r0, int p, int i,
                                  const int x[4], HopRaw<S, V>& h) {
  typedef typename St<S>::E E;
  typedef VecE<S, V> W;
  const int j = nbr_idx(g, x, MU, SG);
  const int par = SG > 0 ? p : 1 - p, li = SG > 0 ? i : j;
  const E* b = U.p + ((int64_t)(par * 4 + MU) * 9) * U.n;
  const uint32_t lo = (uint32_t)li * (uint32_t)sizeof(E);
#pragma unroll
  for (int k = 0; k < (COMP ? 6 : 9); ++k) h.u[k] = ld_off<E, NTL>(b + (int64_t)k * U.n, lo);
  const uint32_t eo = (uint32_t)((int64_t)j * in.ss + r0), so = (uint32_t)((int64_t)j * in.sss + r0);
  const uint32_t vo = eo * (uint32_t)sizeof(E);
#pragma unroll
  for (int k = 0; k < 12; ++k) h.s[k] = ld_off<W, false>(reinterpret_cast<const W*>(in.p + (int64_t)k * in.n), vo);
  if constexpr (sizeof(S) == 2) h.sc = ld_off<VecF<V>, false>(reinterpret_cast<const VecF<V>*>(in.scale), so * 4u);
}

template <class S, int V, int MU, int SG, bool COMP>
__device__ inline void hop_use_v(const Geo& g, const HopRaw<S, V>& h, const int x[4], typename St<S>::T c0,
                                 cx<typename St<S>::T> (&acc)[V][12]) {
  typedef typename St<S>::T T;
  cx<T> u[9];
#pragma unroll
  for (int k = 0; k < (COMP ? 6 : 9); ++k) u[k] = St<S>::from(h.u[k]);
  if constexpr (COMP) {
    const bool edge = MU == 0 && x[0] == (SG > 0 ? g.L[0] - 1 : 0);
    link_row3<T>(T(edge ? g.bc : 1), u);
  }
#pragma unroll
  for (int q = 0; q < V; ++q) {
    cx<T> s[12], hh[6], gg[6];
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = St<S>::from_reg(h.s[k].e[q]);
    T sc;
    if constexpr (sizeof(S) == 2) sc = h.sc.e[q];
    else sc = T(1);
    project<T, MU, SG>(s, hh);
    su3_mul_half<T, (SG < 0)>(u, hh, gg);
    reconstruct_add<T, MU, SG>(gg, acc[q], c0 * sc);
  }
}

template <class S, int V, bool NTL, bool COMP>
__device__ inline void hop_all_vp(const Geo& g, const LinkV<S>& U, const FieldV<S>& in, int r0, int p, int i,
                                  const int x[4], typename St<S>::T c0, cx<typename St<S>::T> (&acc)[V][12]) {
  HopRaw<S, V> a, b;
  hop_load_v<S, V, 0, +1, NTL, COMP>(g, U, in, r0, p, i, x, a);
  __builtin_amdgcn_sched_barrier(0);
  hop_load_v<S, V, 0, -1, NTL, COMP>(g, U, in, r0, p, i, x, b);
  __builtin_amdgcn_sched_barrier(0);
  hop_use_v<S, V, 0, +1, COMP>(g, a, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_load_v<S, V, 1, +1, NTL, COMP>(g, U, in, r0, p, i, x, a);
  __builtin_amdgcn_sched_barrier(0);
  hop_use_v<S, V, 0, -1, COMP>(g, b, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_load_v<S, V, 1, -1, NTL, COMP>(g, U, in, r0, p, i, x, b);
  __builtin_amdgcn_sched_barrier(0);
  hop_use_v<S, V, 1, +1, COMP>(g, a, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_load_v<S, V, 2, +1, NTL, COMP>(g, U, in, r0, p, i, x, a);
  __builtin_amdgcn_sched_barrier(0);
  hop_use_v<S, V, 1, -1, COMP>(g, b, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_load_v<S, V, 2, -1, NTL, COMP>(g, U, in, r0, p, i, x, b);
  __builtin_amdgcn_sched_barrier(0);
  hop_use_v<S, V, 2, +1, COMP>(g, a, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_load_v<S, V, 3, +1, NTL, COMP>(g, U, in, r0, p, i, x, a);
  __builtin_amdgcn_sched_barrier(0);
  hop_use_v<S, V, 2, -1, COMP>(g, b, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_load_v<S, V, 3, -1, NTL, COMP>(g, U, in, r0, p, i, x, b);
  __builtin_amdgcn_sched_barrier(0);
  hop_use_v<S, V, 3, +1, COMP>(g, a, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
  hop_use_v<S, V, 3, -1, COMP>(g, b, x, c0, acc);
  __builtin_amdgcn_sched_barrier(0);
}

// waves per SIMD the register budget is sized for
template <int V>
constexpr int vec_waves() { return V >= 4 ? 2 : 3; }

// pass A: t_o = A_o^{-1} H_oe psi_e for V right-hand sides per lane
template <class S, int V, int NTM>
__global__ void __launch_bounds__(256, vec_waves<V>()) k_dhat_va(Geo g, LinkV<S> U, CloverV<S> Ai, FieldV<S> in_e,
                                                                 FieldV<S> t_o, int nrhs, int nrg, int order, int sb) {
  typedef typename St<S>::T T;
  typedef typename St<S>::E E;
  int tile, rg, i, r0;
  map_block(g, blockIdx.x, gridDim.x, nrg, sb, order, tile, rg);
  if (!lane_site<V>(g, tile, rg, sb, nrhs, 1, i, r0)) return;
  int x[4];
  site_coords(g, 1, i, x);
  cx<T> acc[V][12];
#pragma unroll
  for (int q = 0; q < V; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {T(0), T(0)};
  if constexpr (sizeof(S) == 2)
    hop_all_vp<S, V, (NTM & 1) != 0, (NTM & 4) != 0>(g, U, in_e, r0, 1, i, x, T(1), acc);
  else
    hop_all_v<S, V, (NTM & 1) != 0, (NTM & 4) != 0>(g, U, in_e, r0, 1, i, x, T(1), acc);
  // acc <- A_o^{-1} acc, one 6x6 block at a time for all V
  const E* b = Ai.p + (int64_t)36 * Ai.n;
  const uint32_t vo = (uint32_t)i * (uint32_t)sizeof(E);
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    cx<T> a[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) a[k] = St<S>::from(ld_off<E, (NTM & 1) != 0>(b + (int64_t)(blk * 18 + k) * Ai.n, vo));
#pragma unroll
    for (int q = 0; q < V; ++q) {
      cx<T> y[6];
      herm6_mul<T>(a, acc[q] + 6 * blk, y);
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[q][6 * blk + k] = y[k];
    }
  }
  st_spinor_v<S, V, (NTM & 2) != 0>(t_o, (uint32_t)((int64_t)i * t_o.ss + r0), (uint32_t)((int64_t)i * t_o.sss + r0),
                                    acc);
}

// pass B: out_e = A_e psi_e - 1/4 H_eo t_o for V right-hand sides per lane
template <class S, int V, int NTM>
__global__ void __launch_bounds__(256, vec_waves<V>()) k_dhat_vb(Geo g, LinkV<S> U, CloverV<S> A, FieldV<S> in_e,
                                                                 FieldV<S> t_o, FieldV<S> out_e, int nrhs, int nrg,
                                                                 int order, int sb) {
  typedef typename St<S>::T T;
  typedef typename St<S>::E E;
  int tile, rg, i, r0;
  map_block(g, blockIdx.x, gridDim.x, nrg, sb, order, tile, rg);
  if (!lane_site<V>(g, tile, rg, sb, nrhs, 1, i, r0)) return;
  int x[4];
  site_coords(g, 0, i, x);
  cx<T> acc[V][12];
#pragma unroll
  for (int q = 0; q < V; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {T(0), T(0)};
  if constexpr (sizeof(S) == 2)
    hop_all_vp<S, V, (NTM & 1) != 0, (NTM & 4) != 0>(g, U, t_o, r0, 0, i, x, T(-0.25), acc);
  else
    hop_all_v<S, V, (NTM & 1) != 0, (NTM & 4) != 0>(g, U, t_o, r0, 0, i, x, T(-0.25), acc);
  VecE<S, V> raw[12];
  T sc[V];
  ld_spinor_v<S, V, (NTM & 2) != 0>(in_e, (uint32_t)((int64_t)i * in_e.ss + r0),
                                    (uint32_t)((int64_t)i * in_e.sss + r0), raw, sc);
  const E* b = A.p;
  const uint32_t vo = (uint32_t)i * (uint32_t)sizeof(E);
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    cx<T> a[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) a[k] = St<S>::from(ld_off<E, (NTM & 1) != 0>(b + (int64_t)(blk * 18 + k) * A.n, vo));
#pragma unroll
    for (int q = 0; q < V; ++q) {
      cx<T> v[6], y[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] = St<S>::from_reg(raw[6 * blk + k].e[q]);
      herm6_mul<T>(a, v, y);
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[q][6 * blk + k] = cacc(acc[q][6 * blk + k], sc[q], y[k]);
    }
  }
  st_spinor_v<S, V, (NTM & 2) != 0>(out_e, (uint32_t)((int64_t)i * out_e.ss + r0),
                                    (uint32_t)((int64_t)i * out_e.sss + r0), acc);
}

// full D on both parities; in/out: full fields (parity p at offset p*poff
// elements); the two halves of the grid are walked like two Dhat passes.
// The per-rhs array `shift` holds, with SH, a diagonal shift (out += shift[r]
// psi) and, with CE, a factor on the even sites' clover term (out_e =
// shift[r] A_e psi_e - 1/2 H psi_o: with shift[r] = 1 + dm the operator whose
// Schur complement is Dhat + dm A_e)
template <class S, int NR, bool O32, bool SH, bool CE>
__device__ __forceinline__ void dw_body(const Geo& g, const LinkV<S>& U, const CloverV<S>& A, const FieldV<S>& in,
                                        const FieldV<S>& out, int64_t poff, int64_t spoff, int nrhs, int nrg,
                                        int order, int sb, const double* shift, int bid, int nbid) {
  typedef typename St<S>::T T;
  const int rf = 0;  // full fields are always in the blocked layout
  int nh = nbid >> 1;
  int p = bid >= nh;
  int tile, rg, i, r0;
  map_block(g, bid - p * nh, nh, nrg, sb, order, tile, rg);
  if (!lane_site<NR>(g, tile, rg, sb, nrhs, rf, i, r0)) return;
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
  // acc = -1/2 H psi_{1-p}, then out = A_p psi_p + acc
  cx<T> acc[NR][12];
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[q][k] = {T(0), T(0)};
  hop_all<S, NR, O32>(g, U, src, r0, nr, p, i, x, T(-0.5), acc);
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      cx<T> s[12], o[12];
      T sc = ld_spinor_raw<S, O32>(self, r0 + q, i, s);
      clover_apply_u<S>(A, p, i, s, o);
      if constexpr (SH) {
        const T dl = (T)shift[r0 + q];
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] = cacc(o[k], dl, s[k]);
      }
      // the even clover factor rides on the spinor's scale (SH and CE never meet)
      if constexpr (CE) {
        const T f = (T)shift[r0 + q];
        sc = p ? sc : sc * f;
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = cacc(acc[q][k], sc, o[k]);
      st_spinor<S, O32>(dst, r0 + q, i, o);
    }
  }
}

template <class S, int NR, bool O32, bool SH, bool CE = false>
__global__ void __launch_bounds__(256, NR == 1 ? (sizeof(S) == 8 ? 2 : 4) : 1) k_dw(Geo g, LinkV<S> U, CloverV<S> A, FieldV<S> in, FieldV<S> out,
                                            int64_t poff, int64_t spoff, int nrhs, int nrg, int order, int sb,
                                            const double* shift) {
  dw_body<S, NR, O32, SH, CE>(g, U, A, in, out, poff, spoff, nrhs, nrg, order, sb, shift, blockIdx.x, gridDim.x);
}

// the full D of several systems in one launch (no shifts)
template <class S, int NR, bool O32>
__global__ void __launch_bounds__(256, NR == 1 ? (sizeof(S) == 8 ? 2 : 4) : 1) k_dw_grp(Grp<DwArgs<S>> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  const DwArgs<S>& a = G.a[s];
  dw_body<S, NR, O32, false, false>(a.g, a.U, a.A, a.in, a.out, a.poff, a.spoff, a.nrhs, a.nrg, a.order, a.sb,
                                    nullptr, blockIdx.x - G.start[s], G.start[s + 1] - G.start[s]);
}

// ------------------------------------------------- LDS-staged batched variant
// A workgroup owns a tile of sb consecutive sites of one parity and all
// right-hand sides: blockDim = sb x R lanes, lane (s, rl) takes site s and the
// right-hand sides rl, rl + R, ...  The tile's 8 links per site (4 forward of its
// own parity, 4 backward stored at the neighbours of the other parity) and its
// clover block are read from HBM once, coalesced, into LDS as [slot][site]; every
// lane then loops over its right-hand sides with the links and the clover taken
// from LDS and only the spinors from global memory.  Slots: 0..35 forward links
// (9 per direction), 36..71 backward links, 72..107 clover (2 x 18).
constexpr int kStageSlots = 108;

template <class S>
__device__ inline typename St<S>::E stage_elem(const LinkV<S>& U, const CloverV<S>& C, int p, int i, const int nb[4],
                                               int slot) {
  if (slot < 36) {
    int mu = slot / 9, k = slot - 9 * mu;
    return U.p[((int64_t)(p * 4 + mu) * 9 + k) * U.n + i];
  }
  if (slot < 72) {
    int mu = (slot - 36) / 9, k = slot - 36 - 9 * mu;
    return U.p[((int64_t)((1 - p) * 4 + mu) * 9 + k) * U.n + nb[mu]];
  }
  return C.p[((int64_t)p * 36 + (slot - 72)) * C.n + i];
}

// lane (s, rl) moves slots rl, rl + R, ... of site s; the loads of a chunk are
// all issued before the first LDS write so their latencies overlap
template <class S>
__device__ inline void stage_tile(const Geo& g, const LinkV<S>& U, const CloverV<S>& C, int p, int i, bool valid,
                                  int s, int sb, int rl, int R, const int nb[4], typename St<S>::E* lds) {
  typedef typename St<S>::E E;
  constexpr int CH = 12;
  for (int base = rl; base < kStageSlots; base += CH * R) {
    E v[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      int slot = base + c * R;
      v[c] = (valid && slot < kStageSlots) ? stage_elem<S>(U, C, p, i, nb, slot) : E{};
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      int slot = base + c * R;
      if (slot < kStageSlots) lds[slot * sb + s] = v[c];
    }
  }
}

template <class S, int MU, bool O32>
__device__ inline void hop_dir_lds(const typename St<S>::E* lds, int sb, int s, const FieldV<S>& in, int r, int jf,
                                   int jb, typename St<S>::T c0, cx<typename St<S>::T> (&acc)[12]) {
  typedef typename St<S>::T T;
  cx<T> u[9], sp[12], h[6], gg[6];
#pragma unroll
  for (int k = 0; k < 9; ++k) u[k] = St<S>::ldc(lds + (MU * 9 + k) * sb + s);
  T sc = ld_spinor_raw<S, O32>(in, r, jf, sp);
  project<T, MU, +1>(sp, h);
  su3_mul_half<T, false>(u, h, gg);
  reconstruct_add<T, MU, +1>(gg, acc, c0 * sc);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) u[k] = St<S>::ldc(lds + (36 + MU * 9 + k) * sb + s);
  sc = ld_spinor_raw<S, O32>(in, r, jb, sp);
  project<T, MU, -1>(sp, h);
  su3_mul_half<T, true>(u, h, gg);
  reconstruct_add<T, MU, -1>(gg, acc, c0 * sc);
}

template <class S>
__device__ inline void clover_lds(const typename St<S>::E* lds, int sb, int s, const cx<typename St<S>::T> in[12],
                                  cx<typename St<S>::T> out[12]) {
  typedef typename St<S>::T T;
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    cx<T> a[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) a[k] = St<S>::ldc(lds + (72 + blk * 18 + k) * sb + s);
    herm6_mul<T>(a, in + 6 * blk, out + 6 * blk);
  }
}

// PASS 0 (pass A, odd sites):  out = A_o^{-1} H in      (in: even field)
// PASS 1 (pass B, even sites): out = A_e self - 1/4 H in (in: odd field t_o)
template <class S, int PASS, bool O32>
__global__ void __launch_bounds__(256, sizeof(S) == 8 ? 2 : 4) k_dhat_staged(Geo g, LinkV<S> U, CloverV<S> C, FieldV<S> in, FieldV<S> self,
                                                     FieldV<S> out, int nrhs, int order, int sb, int rf) {
  typedef typename St<S>::T T;
  typedef typename St<S>::E E;
  extern __shared__ unsigned char smem[];
  E* lds = reinterpret_cast<E*>(smem);
  const int p = PASS == 0 ? 1 : 0;
  int tile, rg;
  map_block(g, blockIdx.x, gridDim.x, 1, sb, order, tile, rg);
  const int R = (int)blockDim.x / sb;
  const int s = rf ? (int)threadIdx.x / R : (int)threadIdx.x % sb;
  const int rl = rf ? (int)threadIdx.x % R : (int)threadIdx.x / sb;
  const int i = tile * sb + s;
  const bool valid = i < g.Vh;
  int jf[4], jb[4];
  if (valid) {
    int x[4];
    site_coords(g, p, i, x);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      jf[mu] = nbr_idx(g, x, mu, +1);
      jb[mu] = nbr_idx(g, x, mu, -1);
    }
  }
  stage_tile<S>(g, U, C, p, i, valid, s, sb, rl, R, jb, lds);
  __syncthreads();
  if (!valid) return;
  for (int r = rl; r < nrhs; r += R) {
    // the LDS reads are the same for every right-hand side; an opaque copy of
    // the site offset keeps the compiler from hoisting all 108 of them out of
    // the loop into registers (which would cut the occupancy to one wave)
    int so = s;
    asm volatile("" : "+v"(so));
    cx<T> acc[12], o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
    const T c0 = PASS == 0 ? T(1) : T(-0.25);
    hop_dir_lds<S, 0, O32>(lds, sb, so, in, r, jf[0], jb[0], c0, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop_dir_lds<S, 1, O32>(lds, sb, so, in, r, jf[1], jb[1], c0, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop_dir_lds<S, 2, O32>(lds, sb, so, in, r, jf[2], jb[2], c0, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop_dir_lds<S, 3, O32>(lds, sb, so, in, r, jf[3], jb[3], c0, acc);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (PASS == 0) {
      clover_lds<S>(lds, sb, so, acc, o);
    } else {
      cx<T> v[12];
      T sc = ld_spinor_raw<S, O32>(self, r, i, v);
      clover_lds<S>(lds, sb, so, v, o);
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = cacc(acc[k], sc, o[k]);
    }
    st_spinor<S, O32>(out, r, i, o);
  }
}

// ----------------------------------------------------------------- launchers
static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// true if every element offset (r * rs + i, r < nrhs, i < n, plus the parity
// offset poff of a full field) of f, in bytes, and of its scale array, stays
// below 2^32: the kernels may then form the offsets in 32 bits
template <class S>
static bool fits32(const Geo& g, const FieldV<S>& f, int nrhs, int64_t poff = 0, int64_t spoff = 0) {
  const int64_t lim = (int64_t)1 << 32;
  // largest per-lane offset (r * rs + i * ss; the component offset is scalar) plus the parity offset
  int64_t e = ((int64_t)(nrhs - 1) * f.rs + (int64_t)(g.Vh - 1) * f.ss + poff + 1) * (int64_t)sizeof(typename St<S>::E);
  int64_t sc = f.scale ? ((int64_t)(nrhs - 1) * f.srs + (int64_t)(g.Vh - 1) * f.sss + spoff + 1) * 4 : 0;
  return e < lim && sc < lim;
}

template <class S>
static hipError_t launch_dhat_staged(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> tmp, FieldV<S> out,
                                     int nrhs, const LaunchCfg& c, hipStream_t st, int pass, hipEvent_t ev) {
  int sb = c.sb > 0 ? c.sb : c.block;
  dim3 grid(ceil_div(g.Vh, sb)), blk(c.block);
  size_t lds = (size_t)kStageSlots * sb * sizeof(typename St<S>::E);
  const bool o32 = fits32(g, in, nrhs) && fits32(g, tmp, nrhs) && fits32(g, out, nrhs);
  const int rf = in.ss > 1;  // interleaved operands: rhs fastest across the lanes
  if (pass & 1) {
    if (o32)
      hipLaunchKernelGGL((k_dhat_staged<S, 0, true>), grid, blk, lds, st, g, op.U, op.Ainv, in, in, tmp, nrhs, c.xcd,
                         sb, rf);
    else
      hipLaunchKernelGGL((k_dhat_staged<S, 0, false>), grid, blk, lds, st, g, op.U, op.Ainv, in, in, tmp, nrhs, c.xcd,
                         sb, rf);
  }
  if (ev) (void)hipEventRecord(ev, st);
  if (pass & 2) {
    if (o32)
      hipLaunchKernelGGL((k_dhat_staged<S, 1, true>), grid, blk, lds, st, g, op.U, op.A, tmp, in, out, nrhs, c.xcd, sb, rf);
    else
      hipLaunchKernelGGL((k_dhat_staged<S, 1, false>), grid, blk, lds, st, g, op.U, op.A, tmp, in, out, nrhs, c.xcd,
                         sb, rf);
  }
  return hipGetLastError();
}

// the rhs-vector kernels apply to an operand that keeps V consecutive right-hand
// sides of a site in one aligned V*sizeof(E)-byte word (and their FP16 scales
// in one 4V-byte word)
template <class S, int V>
static bool vec_ok(const FieldV<S>& f, int nrhs) {
  constexpr size_t W = V * sizeof(typename St<S>::E);
  bool ok = f.rs == 1 && f.ss % V == 0 && f.n % V == 0 && nrhs % V == 0 && ((uintptr_t)f.p % W) == 0;
  if constexpr (sizeof(S) == 2) ok = ok && f.scale && f.srs == 1 && f.sss % V == 0 && ((uintptr_t)f.scale % (4 * V)) == 0;
  return ok;
}

template <class S, int V>
static hipError_t launch_dhat_vec(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> tmp, FieldV<S> out,
                                  int nrhs, const LaunchCfg& c, hipStream_t st, int pass, hipEvent_t ev) {
  int sb = c.sb > 0 ? c.sb : c.block;
  int nrg = ceil_div(nrhs, V * (c.block / sb));
  dim3 grid(ceil_div(g.Vh, sb) * nrg), blk(c.block);
  const int ntm = (c.xcd >> 2) & 7, order = c.xcd & 3, order_b = order | ((c.xcd & 64) ? 4 : 0);
#define QDD_VEC(KER, ...)                                                                  \
  switch (ntm) {                                                                           \
    case 0: hipLaunchKernelGGL((KER<S, V, 0>), grid, blk, 0, st, __VA_ARGS__); break;      \
    case 1: hipLaunchKernelGGL((KER<S, V, 1>), grid, blk, 0, st, __VA_ARGS__); break;      \
    case 2: hipLaunchKernelGGL((KER<S, V, 2>), grid, blk, 0, st, __VA_ARGS__); break;      \
    case 3: hipLaunchKernelGGL((KER<S, V, 3>), grid, blk, 0, st, __VA_ARGS__); break;      \
    case 4: hipLaunchKernelGGL((KER<S, V, 4>), grid, blk, 0, st, __VA_ARGS__); break;      \
    case 5: hipLaunchKernelGGL((KER<S, V, 5>), grid, blk, 0, st, __VA_ARGS__); break;      \
    case 6: hipLaunchKernelGGL((KER<S, V, 6>), grid, blk, 0, st, __VA_ARGS__); break;      \
    default: hipLaunchKernelGGL((KER<S, V, 7>), grid, blk, 0, st, __VA_ARGS__); break;     \
  }
  if (pass & 1) QDD_VEC(k_dhat_va, g, op.U, op.Ainv, in, tmp, nrhs, nrg, order, sb)
  if (ev) (void)hipEventRecord(ev, st);
  if (pass & 2) QDD_VEC(k_dhat_vb, g, op.U, op.A, in, tmp, out, nrhs, nrg, order_b, sb)
#undef QDD_VEC
  return hipGetLastError();
}

template <class S, int NR>
static hipError_t launch_dhat_nr(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> tmp, FieldV<S> out,
                                 int nrhs, const LaunchCfg& c, hipStream_t st, int pass, hipEvent_t ev) {
  int sb = c.sb > 0 ? c.sb : c.block;
  int nrg = ceil_div(nrhs, NR * (c.block / sb));
  int tiles = ceil_div(g.Vh, sb);
  dim3 grid(tiles * nrg), blk(c.block);
  const bool o32 = fits32(g, in, nrhs) && fits32(g, tmp, nrhs) && fits32(g, out, nrhs);
  // rhs-vector loads (bit 5 of the walk field) where the operands allow them
  if constexpr (NR > 1 && NR * sizeof(typename St<S>::E) <= 16)
    if ((c.xcd & 32) && o32 && vec_ok<S, NR>(in, nrhs) && vec_ok<S, NR>(tmp, nrhs) && vec_ok<S, NR>(out, nrhs))
      return launch_dhat_vec<S, NR>(g, op, in, tmp, out, nrhs, c, st, pass, ev);
  // streaming access to single-use data (bits 0, 1) and compressed links (bit 2)
  const int ntm = o32 && NR == 1 ? (c.xcd >> 2) & 7 : 0;
  const int order = c.xcd & 3, order_b = order | ((c.xcd & 64) ? 4 : 0);
  const int rf = in.ss > 1;  // interleaved operands: rhs fastest across the lanes
#define QDD_DHAT_V(KER, M, ...) \
  hipLaunchKernelGGL((KER<S, NR, true, NR == 1 ? M : 0>), grid, blk, 0, st, __VA_ARGS__)
#define QDD_DHAT_PASS(KER, ...)                                                                  \
  switch (o32 ? 1 + ntm : 0) {                                                                   \
    case 0: hipLaunchKernelGGL((KER<S, NR, false, 0>), grid, blk, 0, st, __VA_ARGS__); break;    \
    case 1: QDD_DHAT_V(KER, 0, __VA_ARGS__); break;                                              \
    case 2: QDD_DHAT_V(KER, 1, __VA_ARGS__); break;                                              \
    case 3: QDD_DHAT_V(KER, 2, __VA_ARGS__); break;                                              \
    case 4: QDD_DHAT_V(KER, 3, __VA_ARGS__); break;                                              \
    case 5: QDD_DHAT_V(KER, 4, __VA_ARGS__); break;                                              \
    case 6: QDD_DHAT_V(KER, 5, __VA_ARGS__); break;                                              \
    case 7: QDD_DHAT_V(KER, 6, __VA_ARGS__); break;                                              \
    default: QDD_DHAT_V(KER, 7, __VA_ARGS__); break;                                             \
  }
  if (pass & 1) QDD_DHAT_PASS(k_dhat_a, g, op.U, op.Ainv, in, tmp, nrhs, nrg, order, sb, rf)
  if (ev) (void)hipEventRecord(ev, st);
  if (pass & 2) QDD_DHAT_PASS(k_dhat_b, g, op.U, op.A, in, tmp, out, nrhs, nrg, order_b, sb, rf)
#undef QDD_DHAT_PASS
#undef QDD_DHAT_V
  return hipGetLastError();
}

template <class S>
hipError_t launch_dhat(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> tmp, FieldV<S> out, int nrhs,
                       const LaunchCfg& c, hipStream_t st, int pass, hipEvent_t ev) {
  switch (c.nr) {
    case 0: return launch_dhat_staged<S>(g, op, in, tmp, out, nrhs, c, st, pass, ev);
    case 1: return launch_dhat_nr<S, 1>(g, op, in, tmp, out, nrhs, c, st, pass, ev);
    case 2: return launch_dhat_nr<S, 2>(g, op, in, tmp, out, nrhs, c, st, pass, ev);
    case 4: return launch_dhat_nr<S, 4>(g, op, in, tmp, out, nrhs, c, st, pass, ev);
    default: return hipErrorInvalidValue;
  }
}

template <class S, int NR>
static hipError_t launch_dw_nr(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> out, int64_t poff,
                               int64_t spoff, int nrhs, const LaunchCfg& c, hipStream_t st, const double* sh,
                               const double* ce) {
  int sb = c.sb > 0 ? c.sb : c.block;
  int nrg = ceil_div(nrhs, NR * (c.block / sb));
  int tiles = 2 * ceil_div(g.Vh, sb);
  const dim3 grid(tiles * nrg), blk(c.block);
  const bool o32 = fits32(g, in, nrhs, poff, spoff) && fits32(g, out, nrhs, poff, spoff);
#define DW(O, H, E, P) \
  hipLaunchKernelGGL((k_dw<S, NR, O, H, E>), grid, blk, 0, st, g, op.U, op.A, in, out, poff, spoff, nrhs, nrg, c.xcd, \
                     sb, P)
  if (ce) {
    if (o32) DW(true, false, true, ce);
    else DW(false, false, true, ce);
  } else if (o32) {
    if (sh) DW(true, true, false, sh);
    else DW(true, false, false, sh);
  } else {
    if (sh) DW(false, true, false, sh);
    else DW(false, false, false, sh);
  }
#undef DW
  return hipGetLastError();
}

template <class S, int NR>
static hipError_t launch_dw_grp_nr(const DwArgs<S>* a, int ns, const LaunchCfg& c, hipStream_t st) {
  Grp<DwArgs<S>> G = grp_new<DwArgs<S>>();
  bool o32 = true;
  for (int s = 0; s < ns; ++s) {
    DwArgs<S> b = a[s];
    b.sb = c.sb > 0 ? c.sb : c.block;
    b.nrg = ceil_div(b.nrhs, NR * (c.block / b.sb));
    b.order = c.xcd;
    o32 = o32 && fits32(b.g, b.in, b.nrhs, b.poff, b.spoff) && fits32(b.g, b.out, b.nrhs, b.poff, b.spoff);
    grp_add(G, b, 2 * ceil_div(b.g.Vh, b.sb) * b.nrg);
  }
  const dim3 grid(G.start[ns]), blk(c.block);
  if (o32) hipLaunchKernelGGL((k_dw_grp<S, NR, true>), grid, blk, 0, st, G);
  else hipLaunchKernelGGL((k_dw_grp<S, NR, false>), grid, blk, 0, st, G);
  return hipGetLastError();
}

template <class S>
hipError_t launch_dw_grp(const DwArgs<S>* a, int ns, const LaunchCfg& c, hipStream_t st) {
  if (ns < 1 || ns > kGrpMax) return hipErrorInvalidValue;
  switch (c.nr) {
    case 1: return launch_dw_grp_nr<S, 1>(a, ns, c, st);
    case 2: return launch_dw_grp_nr<S, 2>(a, ns, c, st);
    case 4: return launch_dw_grp_nr<S, 4>(a, ns, c, st);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_dw_grp<double>(const DwArgs<double>*, int, const LaunchCfg&, hipStream_t);

template <class S>
hipError_t launch_dw(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> out, int64_t poff, int64_t spoff,
                     int nrhs, const LaunchCfg& c, hipStream_t st, const double* shift, const double* ce) {
  if (shift && ce) return hipErrorInvalidValue;
  switch (c.nr) {
    case 1: return launch_dw_nr<S, 1>(g, op, in, out, poff, spoff, nrhs, c, st, shift, ce);
    case 2: return launch_dw_nr<S, 2>(g, op, in, out, poff, spoff, nrhs, c, st, shift, ce);
    case 4: return launch_dw_nr<S, 4>(g, op, in, out, poff, spoff, nrhs, c, st, shift, ce);
    default: return hipErrorInvalidValue;
  }
}

#define INST(S)                                                                                                     \
  template hipError_t launch_dhat<S>(const Geo&, const DevOp<S>&, FieldV<S>, FieldV<S>, FieldV<S>, int,             \
                                     const LaunchCfg&, hipStream_t, int, hipEvent_t);                               \
  template hipError_t launch_dw<S>(const Geo&, const DevOp<S>&, FieldV<S>, FieldV<S>, int64_t, int64_t, int,        \
                                   const LaunchCfg&, hipStream_t, const double*, const double*);
INST(double)
INST(float)
INST(__half)
#undef INST

}  // namespace qdd
