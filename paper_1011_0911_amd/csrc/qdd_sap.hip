// Schwarz alternating procedure (the "Schwarz-preconditioned" part of the
// paper's solver, Sect. 3): multiplicative two-colour SAP with minimal-residual
// block solves on the even-odd block operator.
//
// A half-sweep over the blocks of one colour does, for every block Lambda and
// every right-hand side:
//   rho_L += 1/2 H_face V        (corrections V of the neighbouring blocks of the
//                                 other colour, made in the previous half-sweep)
//   b      = rho_e + 1/2 H_L A_o^{-1} rho_o
//   x = 0, r = b; nmr times: p = Dhat_L r, alpha = <p,r>/<p,p>, x += alpha r, r -= alpha p
//   v_e = x, v_o = A_o^{-1} (rho_o + 1/2 H_L v_e)
//   psi_L += v, V_L = v, rho_L = (r on even sites, 0 on odd sites)
// (D = A - H/2; H_L the hops inside the block, H_face those across its faces.)
// The new block residual needs no extra operator application: on odd sites it is
// zero by construction and on even sites it is the MR residual r.
//
// Two kernels, both with one lane per even/odd site pair of the block (every
// lane busy in both halves of a hop): for FP32 and FP16 storage one workgroup per
// (block, right-hand side), hop sources exchanged as whole spinors in LDS; for
// FP64 one workgroup per block looping over the right-hand sides, with projected
// half-spinors exchanged in LDS.  Links and clover blocks are read where they
// are used.
#include "qdd_kernels.h"
#include "qdd_sap.h"

namespace qdd {

template <class S>
__device__ inline cx<typename St<S>::T> cvt(typename St<S>::E e);
template <>
__device__ inline cx<double> cvt<double>(double2 e) { return {e.x, e.y}; }
template <>
__device__ inline cx<float> cvt<float>(float2 e) { return {e.x, e.y}; }
// FP16 operands held in registers are converted where used: the opaque move
// keeps the compiler from hoisting FP32 copies of all links and clover entries
// out of the solver loops (which would not fit the register file)
template <>
__device__ inline cx<float> cvt<__half>(__half2 e) {
  asm volatile("" : "+v"(e));
  float2 f = __half22float2(e);
  return {f.x, f.y};
}

template <class T>
__device__ inline T wsum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// half-spinor exchange buffer: [slot][component][source site]
template <class T, int NSLOT>
struct Exch {
  cx<T> v[NSLOT][6][kSapMaxHalf];
};

// Per-site variant for FP32 and FP16 storage: one workgroup per block, one lane
// per site (even sites in the low lanes, odd sites in the high lanes), the
// site's own links and clover block held in registers for the whole half-sweep
// and reused across all MR steps and right-hand sides, which are solved one
// after the other; hops exchange projected half-spinors (the forward
// projection, and the U^dag-transported backward one) through LDS, so every lane
// multiplies only with its own forward links.
// block of one colour taken by a workgroup: hardware workgroup ids go round-robin
// over the 8 XCDs, so every XCD gets a contiguous range of blocks.  With 4^4
// blocks a block row holds 2 sites of a parity, and the blocks of one x3 row
// share the cache lines of the parity-split fields and links: walked on one XCD
// they are fetched into its L2 once instead of once per XCD.
__device__ inline int sap_xcd_block(int id, int nbc) {
  return (nbc & 7) == 0 ? (id & 7) * (nbc >> 3) + (id >> 3) : id;
}

template <class S, class P, int DR>
__device__ __forceinline__ void sap_half_body(const SapArgs<S, P>& a, int bid, int nbid) {
  typedef typename St<S>::T T;
  typedef typename St<S>::E E;
  constexpr bool REG = sizeof(S) <= 4;  // FP32 / FP16: own links + clover in registers
  __shared__ Exch<T, 2 * DR> ex;
  __shared__ T red[8][4];
  const Geo& g = a.g;
  const int nsb = a.bs[0] * a.bs[1] * a.bs[2] * a.bs[3], nsh = nsb >> 1;
  const int t = threadIdx.x;
  const int q = t >= nsh;  // parity of this lane's site
  const int j = t - q * nsh;
  // this block: the sap_xcd_block(blockIdx.x)-th block of colour a.col
  int bc[4];
  {
    int bl = 2 * sap_xcd_block(bid, nbid);
    int nbh3 = a.nb[3];
    bc[3] = bl % nbh3;
    int rr = bl / nbh3;
    bc[2] = rr % a.nb[2];
    rr /= a.nb[2];
    bc[1] = rr % a.nb[1];
    bc[0] = rr / a.nb[1];
    bc[3] += (a.col + bc[0] + bc[1] + bc[2] + bc[3]) & 1;
  }
  // local coordinates of the site
  int y[4];
  {
    int l = 2 * j;
    y[3] = l % a.bs[3];
    int rr = l / a.bs[3];
    y[2] = rr % a.bs[2];
    rr /= a.bs[2];
    y[1] = rr % a.bs[1];
    y[0] = rr / a.bs[1];
    y[3] += (q + y[0] + y[1] + y[2] + y[3]) & 1;
  }
  int x[4];
  for (int m = 0; m < 4; ++m) x[m] = bc[m] * a.bs[m] + y[m];
  const int i = lex_of(g, x) >> 1;
  // neighbour slots inside the block (-1 if the hop crosses a face)
  int nin[4][2];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      int z[4] = {y[0], y[1], y[2], y[3]};
      z[m] += d == 0 ? 1 : -1;
      bool in = z[m] >= 0 && z[m] < a.bs[m];
      nin[m][d] = in ? ((((z[0] * a.bs[1] + z[1]) * a.bs[2] + z[2]) * a.bs[3] + z[3]) >> 1) : -1;
    }
  }
  // own forward links and clover block (A on even sites, A^{-1} on odd sites)
  E ureg[REG ? 4 : 1][9];
  E creg[REG ? 36 : 1];
  const E* ubase = a.U.p + (int64_t)(q * 4) * 9 * a.U.n + i;
  const CloverV<S> cl = q == 0 ? a.A : a.Ai;
  const E* cbase = cl.p + (int64_t)q * 36 * cl.n + i;
  if constexpr (REG) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int k = 0; k < 9; ++k) ureg[m][k] = ubase[(int64_t)(m * 9 + k) * a.U.n];
#pragma unroll
    for (int k = 0; k < 36; ++k) creg[k] = cbase[(int64_t)k * cl.n];
  }
  auto link = [&](int m, cx<T> u[9]) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if constexpr (REG) u[k] = cvt<S>(ureg[m][k]);
      else u[k] = cvt<S>(ubase[(int64_t)(m * 9 + k) * a.U.n]);
    }
  };
  auto clover = [&](const cx<T> in[12], cx<T> out[12]) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      cx<T> c[18];
#pragma unroll
      for (int k = 0; k < 18; ++k) {
        if constexpr (REG) c[k] = cvt<S>(creg[blk * 18 + k]);
        else c[k] = cvt<S>(cbase[(int64_t)(blk * 18 + k) * cl.n]);
      }
      herm6_mul<T>(c, in + 6 * blk, out + 6 * blk);
    }
  };

  // acc (on target lanes of parity 1-sp) = H_L src (sources: lanes of parity sp)
  auto hop_block = [&](int sp, const cx<T> src[12], cx<T> acc[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
#pragma unroll
    for (int r0 = 0; r0 < 4; r0 += DR) {
      if (q == sp) {
#pragma unroll
        for (int m = r0; m < r0 + DR; ++m) {
          cx<T> h[6], gg[6], u[9];
          // for the backward neighbour's forward hop: (1 - g_m) projection
          if (m == 0) project<T, 0, +1>(src, h);
          else if (m == 1) project<T, 1, +1>(src, h);
          else if (m == 2) project<T, 2, +1>(src, h);
          else project<T, 3, +1>(src, h);
#pragma unroll
          for (int k = 0; k < 6; ++k) ex.v[2 * (m - r0)][k][j] = h[k];
          // for the forward neighbour's backward hop: U^dag (1 + g_m) projection
          if (m == 0) project<T, 0, -1>(src, h);
          else if (m == 1) project<T, 1, -1>(src, h);
          else if (m == 2) project<T, 2, -1>(src, h);
          else project<T, 3, -1>(src, h);
          link(m, u);
          su3_mul_half<T, true>(u, h, gg);
#pragma unroll
          for (int k = 0; k < 6; ++k) ex.v[2 * (m - r0) + 1][k][j] = gg[k];
        }
      }
      __syncthreads();
      if (q != sp) {
#pragma unroll
        for (int m = r0; m < r0 + DR; ++m) {
          int jf = nin[m][0], jb = nin[m][1];
          cx<T> h[6], gg[6], u[9];
          if (jf >= 0) {
#pragma unroll
            for (int k = 0; k < 6; ++k) h[k] = ex.v[2 * (m - r0)][k][jf];
            link(m, u);
            su3_mul_half<T, false>(u, h, gg);
            if (m == 0) reconstruct_add<T, 0, +1>(gg, acc);
            else if (m == 1) reconstruct_add<T, 1, +1>(gg, acc);
            else if (m == 2) reconstruct_add<T, 2, +1>(gg, acc);
            else reconstruct_add<T, 3, +1>(gg, acc);
          }
          if (jb >= 0) {
#pragma unroll
            for (int k = 0; k < 6; ++k) gg[k] = ex.v[2 * (m - r0) + 1][k][jb];
            if (m == 0) reconstruct_add<T, 0, -1>(gg, acc);
            else if (m == 1) reconstruct_add<T, 1, -1>(gg, acc);
            else if (m == 2) reconstruct_add<T, 2, -1>(gg, acc);
            else reconstruct_add<T, 3, -1>(gg, acc);
          }
        }
      }
      __syncthreads();
    }
  };

  auto block_sum2 = [&](T v0, T v1, T v2, T& s0, T& s1, T& s2) {
    v0 = wsum(v0);
    v1 = wsum(v1);
    v2 = wsum(v2);
    int w = t >> 6, nw = (blockDim.x + 63) >> 6;
    if ((t & 63) == 0) {
      red[w][0] = v0;
      red[w][1] = v1;
      red[w][2] = v2;
    }
    __syncthreads();
    s0 = s1 = s2 = T(0);
    for (int k = 0; k < nw; ++k) {
      s0 += red[k][0];
      s1 += red[k][1];
      s2 += red[k][2];
    }
    __syncthreads();
  };

  // field views shifted to this lane's parity
  FieldV<S> rho = a.rho, vf = a.V, vn = a.V;
  FieldV<P> psi = a.psi;
  rho.p += q * a.poff;
  vf.p += q * a.poff;
  vn.p += (1 - q) * a.poff;
  psi.p += q * a.poff;
  if (rho.scale) {
    rho.scale += q * a.spoff;
    vf.scale += q * a.spoff;
    vn.scale += (1 - q) * a.spoff;
  }
  if (psi.scale) psi.scale += q * a.spoff;

  for (int r = 0; r < a.nrhs; ++r) {
    cx<T> rh[12];
    ld_spinor(rho, r, i, rh);
    // boundary: rho += 1/2 H_face V (the neighbours across the faces are of the other parity)
    if (a.do_bnd) {
      cx<T> acc[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
      cx<T> s[12], h[6], gg[6], u[9];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (nin[m][0] < 0) {
          int jn = nbr_idx(g, x, m, +1);
          ld_spinor(vn, r, jn, s);
          link(m, u);
          if (m == 0) { project<T, 0, +1>(s, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 0, +1>(gg, acc); }
          else if (m == 1) { project<T, 1, +1>(s, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 1, +1>(gg, acc); }
          else if (m == 2) { project<T, 2, +1>(s, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 2, +1>(gg, acc); }
          else { project<T, 3, +1>(s, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 3, +1>(gg, acc); }
        }
        if (nin[m][1] < 0) {
          int jn = nbr_idx(g, x, m, -1);
          ld_spinor(vn, r, jn, s);
          ld_link(a.U, 1 - q, m, jn, u);
          if (m == 0) { project<T, 0, -1>(s, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 0, -1>(gg, acc); }
          else if (m == 1) { project<T, 1, -1>(s, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 1, -1>(gg, acc); }
          else if (m == 2) { project<T, 2, -1>(s, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 2, -1>(gg, acc); }
          else { project<T, 3, -1>(s, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 3, -1>(gg, acc); }
        }
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) rh[k] = rh[k] + T(0.5) * acc[k];
    }
    // source reduction: w = A_o^{-1} rho_o (odd lanes); b = rho_e + 1/2 H_L w (even lanes)
    cx<T> w[12], acc[12], xs[12], rr[12];
    if (q == 1) clover(rh, w);
    hop_block(1, w, acc);
    if (q == 0) {
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        rr[k] = rh[k] + T(0.5) * acc[k];
        xs[k] = {T(0), T(0)};
      }
    }
    // minimal-residual steps on Dhat_L
    for (int it = 0; it < a.nmr; ++it) {
      hop_block(0, rr, acc);  // odd lanes: acc = H_L r
      if (q == 1) {
        cx<T> hh[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) hh[k] = T(-0.5) * acc[k];
        clover(hh, w);  // w = A_o^{-1} (-1/2 H r)
      }
      hop_block(1, w, acc);  // even lanes: acc = H_L w
      T pr_re = 0, pr_im = 0, pp = 0;
      cx<T> p[12];
      if (q == 0) {
        clover(rr, p);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          p[k] = p[k] + T(0.5) * acc[k];
          cx<T> z = cmulc(p[k], rr[k]);
          pr_re += z.re;
          pr_im += z.im;
          pp += p[k].re * p[k].re + p[k].im * p[k].im;
        }
      }
      T s0, s1, s2;
      block_sum2(pr_re, pr_im, pp, s0, s1, s2);
      cx<T> al = s2 > T(0) ? cx<T>{s0 / s2, s1 / s2} : cx<T>{T(0), T(0)};
      if (q == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          xs[k] = fma_c(al, rr[k], xs[k]);
          rr[k] = rr[k] - al * p[k];
        }
      }
    }
    // odd reconstruction: v_o = A_o^{-1} (rho_o + 1/2 H_L v_e)
    hop_block(0, xs, acc);
    cx<T> v[12], rnew[12];
    if (q == 1) {
      cx<T> hh[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) hh[k] = rh[k] + T(0.5) * acc[k];
      clover(hh, v);
#pragma unroll
      for (int k = 0; k < 12; ++k) rnew[k] = {T(0), T(0)};
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        v[k] = xs[k];
        rnew[k] = rr[k];
      }
    }
    // write back: psi += v, V = v, rho = new block residual
    typedef typename St<P>::T TP;
    cx<TP> pv[12];
    if (a.first) {
#pragma unroll
      for (int k = 0; k < 12; ++k) pv[k] = {(TP)v[k].re, (TP)v[k].im};
    } else {
      ld_spinor(psi, r, i, pv);
#pragma unroll
      for (int k = 0; k < 12; ++k) pv[k] = pv[k] + cx<TP>{(TP)v[k].re, (TP)v[k].im};
    }
    st_spinor(psi, r, i, pv);
    if (a.write_v) st_spinor(vf, r, i, v);
    st_spinor(rho, r, i, rnew);
  }
}

template <class S, class P, int DR>
__global__ void __launch_bounds__(256) k_sap_half(SapArgs<S, P> a) {
  sap_half_body<S, P, DR>(a, blockIdx.x, gridDim.x);
}
// the same half-sweep for several systems in one launch
template <class S, class P, int DR>
__global__ void __launch_bounds__(256) k_sap_half_grp(Grp<SapArgs<S, P>> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  sap_half_body<S, P, DR>(G.a[s], blockIdx.x - G.start[s], G.start[s + 1] - G.start[s]);
}

// One workgroup per (block, right-hand side): the right-hand sides of a block
// are solved by concurrent workgroups instead of one after the other, and the
// workgroup ids are ordered so that all of them land on the same XCD at about
// the same time (hardware ids go round-robin over the 8 XCDs), where the block's
// links and clover blocks are then fetched from HBM once and served from the L2.
// Lane j owns the j-th even and the j-th odd site of the block (block-local
// order), so every lane works in both halves of a hop.  A hop onto parity tp
// reads the source spinors of parity 1 - tp that all lanes wrote to LDS (one
// 12-component spinor per site, the smallest exchange) and applies the
// projection, the link and the reconstruction for each in-block neighbour of its
// own site (target side).  Links and clover blocks are read where they are used
// (L1/L2 hits), behind an opaque per-lane zero so that the compiler does not
// hoist them out of the MR loop into registers.
template <class S, class P, bool O32>
__device__ __forceinline__ void sap_rhs_body(const SapArgs<S, P>& a, int bid, int nbid) {
  typedef typename St<S>::T T;
  __shared__ cx<T> ex[12][kSapMaxHalf];    // hop sources (one parity of the block)
  __shared__ cx<T> ro_l[12][kSapMaxHalf];  // the odd-site source, own column only
  __shared__ int ig_l[2][kSapMaxHalf];     // index within its parity of every block site
  __shared__ T red[2][3][kSapMaxHalf / 64];  // per-wave partial sums, by MR-step parity
  const Geo& g = a.g;
  const int j = threadIdx.x;
  const int nw = (blockDim.x + 63) >> 6;
  // workgroup -> (block of colour a.col, right-hand side)
  int bi, r;
  {
    const int id = bid, nbc = nbid / a.nrhs;
    if ((nbc & 7) == 0) {  // every XCD a contiguous range of blocks (see sap_xcd_block)
      const int rest = id >> 3;
      r = rest % a.nrhs;
      bi = (id & 7) * (nbc >> 3) + rest / a.nrhs;
    } else {
      r = id % a.nrhs;
      bi = id / a.nrhs;
    }
  }
  int bc[4];
  {
    int bl = 2 * bi;
    bc[3] = bl % a.nb[3];
    int rr = bl / a.nb[3];
    bc[2] = rr % a.nb[2];
    rr /= a.nb[2];
    bc[1] = rr % a.nb[1];
    bc[0] = rr / a.nb[1];
    bc[3] += (a.col + bc[0] + bc[1] + bc[2] + bc[3]) & 1;
  }
  // the lane's two sites (q = 0 even, 1 odd): global coordinates, index within
  // the parity, and neighbour slots inside the block (-1: the hop crosses a face)
  int x[2][4], ig[2], nin[2][4][2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    int y[4];
    int l = 2 * j;
    y[3] = l % a.bs[3];
    int rr = l / a.bs[3];
    y[2] = rr % a.bs[2];
    rr /= a.bs[2];
    y[1] = rr % a.bs[1];
    y[0] = rr / a.bs[1];
    y[3] += (q + y[0] + y[1] + y[2] + y[3]) & 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) x[q][m] = bc[m] * a.bs[m] + y[m];
    ig[q] = lex_of(g, x[q]) >> 1;
    ig_l[q][j] = ig[q];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        int z[4] = {y[0], y[1], y[2], y[3]};
        z[m] += d == 0 ? 1 : -1;
        bool in = z[m] >= 0 && z[m] < a.bs[m];
        nin[q][m][d] = in ? ((((z[0] * a.bs[1] + z[1]) * a.bs[2] + z[2]) * a.bs[3] + z[3]) >> 1) : -1;
      }
    }
  }
  auto vsalt = []() {
    int z = 0;
    asm volatile("" : "+v"(z));
    return z;
  };
  // clover: A on even sites, A^{-1} on odd sites
  auto clover = [&](int q, const cx<T> in[12], cx<T> out[12]) __attribute__((always_inline)) {
    clover_apply_u<S>(q == 0 ? a.A : a.Ai, q, ig[q] + vsalt(), in, out);
  };
  // all lanes: src (the lane's site of parity 1 - tp) -> LDS; then acc (at the
  // lane's site of parity tp) = H_L src.  The barrier before the writes keeps
  // them from overtaking the reads of the previous hop.
  auto hop = [&](const int tp, const cx<T> src[12], cx<T> acc[12]) __attribute__((always_inline)) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 12; ++k) ex[k][j] = src[k];
    __syncthreads();
    const int zv = vsalt();
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int jf = nin[tp][m][0], jb = nin[tp][m][1];
      cx<T> sv[12], h[6], gg[6], u[9];
      if (jf >= 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) sv[k] = ex[k][jf];
        ld_link_u<S>(a.U, tp, m, ig[tp] + zv, u);
        if (m == 0) { project<T, 0, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 0, +1>(gg, acc); }
        else if (m == 1) { project<T, 1, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 1, +1>(gg, acc); }
        else if (m == 2) { project<T, 2, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 2, +1>(gg, acc); }
        else { project<T, 3, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 3, +1>(gg, acc); }
      }
      if (jb >= 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) sv[k] = ex[k][jb];
        ld_link_u<S>(a.U, 1 - tp, m, ig_l[1 - tp][jb] + zv, u);
        if (m == 0) { project<T, 0, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 0, -1>(gg, acc); }
        else if (m == 1) { project<T, 1, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 1, -1>(gg, acc); }
        else if (m == 2) { project<T, 2, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 2, -1>(gg, acc); }
        else { project<T, 3, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 3, -1>(gg, acc); }
      }
    }
  };
  // parity views of the fields
  FieldV<S> rho[2] = {a.rho, a.rho}, vf[2] = {a.V, a.V};
  FieldV<P> psi[2] = {a.psi, a.psi};
  rho[1].p += a.poff;
  vf[1].p += a.poff;
  psi[1].p += a.poff;
  if (a.rho.scale) {
    rho[1].scale += a.spoff;
    vf[1].scale += a.spoff;
  }
  if (a.psi.scale) psi[1].scale += a.spoff;
  // rq += 1/2 H_face V at the lane's site of parity q (the sites across the faces
  // belong to blocks of the other colour, whose corrections V the previous
  // half-sweep stored)
  auto bnd = [&](const int q, cx<T> (&rq)[12]) __attribute__((always_inline)) {
    const int zv = vsalt();
    cx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
    const FieldV<S>& vn = vf[1 - q];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      cx<T> sv[12], h[6], gg[6], u[9];
      if (nin[q][m][0] < 0) {
        int jn = nbr_idx(g, x[q], m, +1) + zv;
        ld_spinor<S, O32>(vn, r, jn, sv);
        ld_link_u<S>(a.U, q, m, ig[q] + zv, u);
        if (m == 0) { project<T, 0, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 0, +1>(gg, acc); }
        else if (m == 1) { project<T, 1, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 1, +1>(gg, acc); }
        else if (m == 2) { project<T, 2, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 2, +1>(gg, acc); }
        else { project<T, 3, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 3, +1>(gg, acc); }
      }
      if (nin[q][m][1] < 0) {
        int jn = nbr_idx(g, x[q], m, -1) + zv;
        ld_spinor<S, O32>(vn, r, jn, sv);
        ld_link_u<S>(a.U, 1 - q, m, jn, u);
        if (m == 0) { project<T, 0, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 0, -1>(gg, acc); }
        else if (m == 1) { project<T, 1, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 1, -1>(gg, acc); }
        else if (m == 2) { project<T, 2, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 2, -1>(gg, acc); }
        else { project<T, 3, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 3, -1>(gg, acc); }
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) rq[k] = cacc(rq[k], T(0.5), acc[k]);
  };
  // psi += v, V = v at the lane's site of parity q
  auto put = [&](const int q, const cx<T> (&v)[12]) __attribute__((always_inline)) {
    typedef typename St<P>::T TP;
    cx<TP> pv[12];
    if (a.first) {
#pragma unroll
      for (int k = 0; k < 12; ++k) pv[k] = {(TP)v[k].re, (TP)v[k].im};
    } else {
      ld_spinor<P, O32>(psi[q], r, ig[q], pv);
#pragma unroll
      for (int k = 0; k < 12; ++k) pv[k] = pv[k] + cx<TP>{(TP)v[k].re, (TP)v[k].im};
    }
    st_spinor<P, O32>(psi[q], r, ig[q], pv);
    if (a.write_v) st_spinor<S, O32>(vf[q], r, ig[q], v);
  };

  cx<T> re[12], ro[12], rr[12], xs[12], w[12], acc[12];
  ld_spinor<S, O32>(rho[0], r, ig[0], re);
  ld_spinor<S, O32>(rho[1], r, ig[1], ro);
  if (a.do_bnd) {
    bnd(0, re);
    bnd(1, ro);
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) ro_l[k][j] = ro[k];
  // source reduction: w = A_o^{-1} rho_o (odd sites); b = rho_e + 1/2 H_L w
  clover(1, ro, w);
  hop(0, w, acc);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    rr[k] = cacc(re[k], T(0.5), acc[k]);
    xs[k] = {T(0), T(0)};
  }
  // minimal-residual steps on Dhat_L: p = A_e r + 1/2 H_L A_o^{-1} (-1/2 H_L r),
  // alpha = <p, r> / <p, p>, x += alpha r, r -= alpha p
  for (int it = 0; it < a.nmr; ++it) {
    hop(1, rr, acc);  // odd sites: acc = H_L r
    {
      cx<T> hh[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) hh[k] = T(-0.5) * acc[k];
      clover(1, hh, w);  // w = A_o^{-1} (-1/2 H_L r)
    }
    hop(0, w, acc);  // even sites: acc = H_L w
    cx<T> pe[12];
    clover(0, rr, pe);
    T pr_re = 0, pr_im = 0, pp = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      pe[k] = cacc(pe[k], T(0.5), acc[k]);
      pr_re = fmar(pe[k].re, rr[k].re, fmar(pe[k].im, rr[k].im, pr_re));
      pr_im = fmar(pe[k].re, rr[k].im, fmar(-pe[k].im, rr[k].re, pr_im));
      pp = fmar(pe[k].re, pe[k].re, fmar(pe[k].im, pe[k].im, pp));
    }
    pr_re = wsum(pr_re);
    pr_im = wsum(pr_im);
    pp = wsum(pp);
    // per-wave partials in alternating slots, so that one barrier per step
    // suffices: a slot is rewritten two steps later, after the hops' barriers
    const int sl = it & 1;
    if ((j & 63) == 0) {
      red[sl][0][j >> 6] = pr_re;
      red[sl][1][j >> 6] = pr_im;
      red[sl][2][j >> 6] = pp;
    }
    __syncthreads();
    T s0 = 0, s1 = 0, s2 = 0;
    for (int k = 0; k < nw; ++k) {
      s0 += red[sl][0][k];
      s1 += red[sl][1][k];
      s2 += red[sl][2][k];
    }
    const cx<T> al = s2 > T(0) ? cx<T>{s0 / s2, s1 / s2} : cx<T>{T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      xs[k] = fma_c(al, rr[k], xs[k]);
      rr[k] = fma_c(cx<T>{-al.re, -al.im}, pe[k], rr[k]);
    }
  }
  // odd reconstruction: v_o = A_o^{-1} (rho_o + 1/2 H_L v_e)
  hop(1, xs, acc);
  cx<T> vo[12];
  {
    cx<T> hh[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) hh[k] = cacc(ro_l[k][j], T(0.5), acc[k]);
    clover(1, hh, vo);
  }
  // write back: psi += v, V = v, rho = new block residual (r even, 0 odd)
  put(0, xs);
  put(1, vo);
  cx<T> zero[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) zero[k] = {T(0), T(0)};
  st_spinor<S, O32>(rho[0], r, ig[0], rr);
  st_spinor<S, O32>(rho[1], r, ig[1], zero);
}

template <class S, class P, bool O32>
__global__ void __launch_bounds__(kSapMaxHalf, 2) k_sap_rhs(SapArgs<S, P> a) {
  sap_rhs_body<S, P, O32>(a, blockIdx.x, gridDim.x);
}
template <class S, class P, bool O32>
__global__ void __launch_bounds__(kSapMaxHalf, 2) k_sap_rhs_grp(Grp<SapArgs<S, P>> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  sap_rhs_body<S, P, O32>(G.a[s], blockIdx.x - G.start[s], G.start[s + 1] - G.start[s]);
}

// LDS-staged variants for FP16 storage: one workgroup per (block, group of R
// right-hand sides).  The block's forward links (4 x 9 per site) and, with CL,
// its clover blocks (A_e on the even, A_o^{-1} on the odd sites, 36 slots each)
// are copied into LDS once and shared by the R right-hand sides the workgroup
// solves side by side, so the hops of the MR loop read only LDS and registers.
// With CL (R = 4, 124 KB of LDS) one workgroup fills a CU; without it (R = 2,
// the clover read from memory at its ten uses per half-sweep, 62 KB) two
// workgroups share a CU and overlap each other's barriers and staging.  Lane (q, j): right-hand side g0 + q of the group, site pair j (the j-th
// even and the j-th odd site of the block); each right-hand side takes whole
// wavefronts (nh rounded up to a multiple of 64 lanes), so its inner products
// are wavefront sums plus one LDS step.  Hops are taken on the target side:
// every lane writes its source spinor to the LDS exchange of its right-hand side,
// then applies projection, link (its own forward link, or the neighbour's for a
// backward hop, both in LDS) and reconstruction for each in-block neighbour.
// FP32 storage (R = 4, links staged, clover from memory): the links alone take
// 72 KB, so one workgroup fills a CU as with CL.
template <class S, class P, int R, bool CL>
constexpr int sap_lds_wgs() { return (CL || sizeof(S) == 4) ? 1 : 2; }

template <class S, class P, int R, bool CL, bool O32>
__device__ __forceinline__ void sap_lds_body(const SapArgs<S, P>& a, int bid, int nbid) {
  typedef typename St<S>::T T;
  typedef typename St<S>::E E;
  constexpr int H = kSapMaxHalf;
  __shared__ E su[36][2 * H];           // forward links, [mu * 9 + k][parity * H + pair]
  __shared__ E sc[CL ? 36 : 1][CL ? 2 * H : 1];  // clover slots, [slot][parity * H + pair] (CL)
  __shared__ cx<T> ex[R][12][H];        // hop sources, per right-hand side
  __shared__ int ig_l[2][H];            // index within its parity of every block site
  __shared__ T red[2][3][R * H / 64];   // per-wave partial sums, by MR-step parity
  const Geo& g = a.g;
  const int nh = (a.bs[0] * a.bs[1] * a.bs[2] * a.bs[3]) >> 1;
  const int nhp = (nh + 63) & ~63;  // lanes per right-hand side
  const int t = threadIdx.x, q = t / nhp, j = t - q * nhp;
  const bool on = j < nh;
  const int nrg = (a.nrhs + R - 1) / R;
  // workgroup -> (block of colour a.col, group of right-hand sides); the groups
  // of a block go to the same XCD one after the other
  int bi, rg;
  {
    const int id = bid, nbc = nbid / nrg;
    if ((nbc & 7) == 0) {  // every XCD a contiguous range of blocks (see sap_xcd_block)
      const int rest = id >> 3;
      rg = rest % nrg;
      bi = (id & 7) * (nbc >> 3) + rest / nrg;
    } else {
      rg = id % nrg;
      bi = id / nrg;
    }
  }
  const int r = rg * R + q;
  const bool act = on && r < a.nrhs;
  const int rs = act ? r : 0;
  int bc[4];
  {
    int bl = 2 * bi;
    bc[3] = bl % a.nb[3];
    int rr = bl / a.nb[3];
    bc[2] = rr % a.nb[2];
    rr /= a.nb[2];
    bc[1] = rr % a.nb[1];
    bc[0] = rr / a.nb[1];
    bc[3] += (a.col + bc[0] + bc[1] + bc[2] + bc[3]) & 1;
  }
  // the lane's two sites (pair jj; lanes beyond the block take pair 0 and only
  // feed barriers): coordinates, index within the parity, in-block neighbour slots
  const int jj = on ? j : 0;
  int x[2][4], ig[2], nin[2][4][2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    int y[4];
    int l = 2 * jj;
    y[3] = l % a.bs[3];
    int rr = l / a.bs[3];
    y[2] = rr % a.bs[2];
    rr /= a.bs[2];
    y[1] = rr % a.bs[1];
    y[0] = rr / a.bs[1];
    y[3] += (p + y[0] + y[1] + y[2] + y[3]) & 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) x[p][m] = bc[m] * a.bs[m] + y[m];
    ig[p] = lex_of(g, x[p]) >> 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        int z[4] = {y[0], y[1], y[2], y[3]};
        z[m] += d == 0 ? 1 : -1;
        bool in = z[m] >= 0 && z[m] < a.bs[m];
        nin[p][m][d] = in ? ((((z[0] * a.bs[1] + z[1]) * a.bs[2] + z[2]) * a.bs[3] + z[3]) >> 1) : -1;
      }
    }
  }
  if (q == 0 && on) {
    ig_l[0][j] = ig[0];
    ig_l[1][j] = ig[1];
  }
  __syncthreads();
  // stage the block's links and clover blocks (once for the R right-hand sides):
  // element (slot, site) of (CL ? 72 : 36) x 2 nh; when the workgroup size is a
  // multiple of 2 nh every lane keeps one site and steps through the slots
  constexpr int NSLOT = CL ? 72 : 36;
  auto stage = [&](int slot, int par, int js, int gi) __attribute__((always_inline)) {
    if (slot < 36) {
      su[slot][par * H + js] = a.U.p[((int64_t)par * 36 + slot) * a.U.n + gi];
    } else if constexpr (CL) {
      const CloverV<S>& c = par == 0 ? a.A : a.Ai;
      sc[slot - 36][par * H + js] = c.p[((int64_t)par * 36 + (slot - 36)) * c.n + gi];
    }
  };
  const int ns2 = 2 * nh;
  if ((int)blockDim.x % ns2 == 0) {
    const int site = t % ns2, par = site >= nh, js = site - par * nh, gi = ig_l[par][js];
    const int step = (int)blockDim.x / ns2;
    for (int slot = t / ns2; slot < NSLOT; slot += step) stage(slot, par, js, gi);
  } else {
    for (int e = t; e < NSLOT * ns2; e += blockDim.x) {
      const int site = e % ns2, slot = e / ns2;
      const int par = site >= nh, js = site - par * nh;
      stage(slot, par, js, ig_l[par][js]);
    }
  }
  auto link = [&](int par, int m, int js, cx<T> u[9]) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = St<S>::from(su[m * 9 + k][par * H + js]);
  };
  auto clover = [&](int par, const cx<T> in[12], cx<T> out[12]) __attribute__((always_inline)) {
    if constexpr (CL) {
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        cx<T> c[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) c[k] = St<S>::from(sc[blk * 18 + k][par * H + jj]);
        herm6_mul<T>(c, in + 6 * blk, out + 6 * blk);
      }
    } else {
      // from memory (L2), behind an opaque zero so that the loads stay at their use
      int z = 0;
      asm volatile("" : "+v"(z));
      clover_apply_u<S>(par == 0 ? a.A : a.Ai, par, ig[par] + z, in, out);
    }
  };
  // src (the lane's site of parity 1 - tp) -> LDS; acc (its site of parity tp) = H_L src
  auto hop = [&](const int tp, const cx<T> src[12], cx<T> acc[12]) __attribute__((always_inline)) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 12; ++k) ex[q][k][j] = src[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int jf = nin[tp][m][0], jb = nin[tp][m][1];
      cx<T> sv[12], h[6], gg[6], u[9];
      if (jf >= 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) sv[k] = ex[q][k][jf];
        link(tp, m, jj, u);
        if (m == 0) { project<T, 0, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 0, +1>(gg, acc); }
        else if (m == 1) { project<T, 1, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 1, +1>(gg, acc); }
        else if (m == 2) { project<T, 2, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 2, +1>(gg, acc); }
        else { project<T, 3, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 3, +1>(gg, acc); }
      }
      if (jb >= 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) sv[k] = ex[q][k][jb];
        link(1 - tp, m, jb, u);
        if (m == 0) { project<T, 0, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 0, -1>(gg, acc); }
        else if (m == 1) { project<T, 1, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 1, -1>(gg, acc); }
        else if (m == 2) { project<T, 2, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 2, -1>(gg, acc); }
        else { project<T, 3, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 3, -1>(gg, acc); }
      }
    }
  };
  FieldV<S> rho[2] = {a.rho, a.rho}, vf[2] = {a.V, a.V};
  FieldV<P> psi[2] = {a.psi, a.psi};
  rho[1].p += a.poff;
  vf[1].p += a.poff;
  psi[1].p += a.poff;
  if (a.rho.scale) {
    rho[1].scale += a.spoff;
    vf[1].scale += a.spoff;
  }
  if (a.psi.scale) psi[1].scale += a.spoff;
  // rp += 1/2 H_face V at the lane's site of parity p (the sites across the faces
  // belong to blocks of the other colour, whose corrections V the previous
  // half-sweep stored).  Both links across a face come from memory: this runs
  // before the barrier that completes the staging, so the staged links, which
  // other wavefronts write, are not read here.
  auto bnd = [&](const int p, cx<T> (&rp)[12]) __attribute__((always_inline)) {
    cx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
    const FieldV<S>& vn = vf[1 - p];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      cx<T> sv[12], h[6], gg[6], u[9];
      if (nin[p][m][0] < 0) {
        ld_spinor<S, O32>(vn, rs, nbr_idx(g, x[p], m, +1), sv);
        ld_link_u<S>(a.U, p, m, ig[p], u);
        if (m == 0) { project<T, 0, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 0, +1>(gg, acc); }
        else if (m == 1) { project<T, 1, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 1, +1>(gg, acc); }
        else if (m == 2) { project<T, 2, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 2, +1>(gg, acc); }
        else { project<T, 3, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 3, +1>(gg, acc); }
      }
      if (nin[p][m][1] < 0) {
        const int jn = nbr_idx(g, x[p], m, -1);
        ld_spinor<S, O32>(vn, rs, jn, sv);
        ld_link_u<S>(a.U, 1 - p, m, jn, u);
        if (m == 0) { project<T, 0, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 0, -1>(gg, acc); }
        else if (m == 1) { project<T, 1, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 1, -1>(gg, acc); }
        else if (m == 2) { project<T, 2, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 2, -1>(gg, acc); }
        else { project<T, 3, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 3, -1>(gg, acc); }
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) rp[k] = cacc(rp[k], T(0.5), acc[k]);
  };
  auto put = [&](const int p, const cx<T> (&v)[12]) __attribute__((always_inline)) {
    typedef typename St<P>::T TP;
    cx<TP> pv[12];
    if (a.first) {
#pragma unroll
      for (int k = 0; k < 12; ++k) pv[k] = {(TP)v[k].re, (TP)v[k].im};
    } else {
      ld_spinor<P, O32>(psi[p], r, ig[p], pv);
#pragma unroll
      for (int k = 0; k < 12; ++k) pv[k] = pv[k] + cx<TP>{(TP)v[k].re, (TP)v[k].im};
    }
    st_spinor<P, O32>(psi[p], r, ig[p], pv);
    if (a.write_v) st_spinor<S, O32>(vf[p], r, ig[p], v);
  };

  cx<T> re[12], ro[12], rr[12], xs[12], w[12], acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) re[k] = ro[k] = {T(0), T(0)};
  if (act) {
    ld_spinor<S, O32>(rho[0], r, ig[0], re);
    ld_spinor<S, O32>(rho[1], r, ig[1], ro);
    if (a.do_bnd) {
      bnd(0, re);
      bnd(1, ro);
    }
  }
  __syncthreads();  // the staged links and clover are complete
  // source reduction: w = A_o^{-1} rho_o (odd sites); b = rho_e + 1/2 H_L w
  clover(1, ro, w);
  hop(0, w, acc);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    rr[k] = cacc(re[k], T(0.5), acc[k]);
    xs[k] = {T(0), T(0)};
  }
  const int wpr = nhp >> 6;  // wavefronts per right-hand side
  for (int it = 0; it < a.nmr; ++it) {
    hop(1, rr, acc);  // odd sites: acc = H_L r
    {
      cx<T> hh[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) hh[k] = T(-0.5) * acc[k];
      clover(1, hh, w);  // w = A_o^{-1} (-1/2 H_L r)
    }
    hop(0, w, acc);  // even sites: acc = H_L w
    cx<T> pe[12];
    clover(0, rr, pe);
    T pr_re = 0, pr_im = 0, pp = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      pe[k] = cacc(pe[k], T(0.5), acc[k]);
      pr_re = fmar(pe[k].re, rr[k].re, fmar(pe[k].im, rr[k].im, pr_re));
      pr_im = fmar(pe[k].re, rr[k].im, fmar(-pe[k].im, rr[k].re, pr_im));
      pp = fmar(pe[k].re, pe[k].re, fmar(pe[k].im, pe[k].im, pp));
    }
    if (!act) pr_re = pr_im = pp = T(0);
    pr_re = wsum(pr_re);
    pr_im = wsum(pr_im);
    pp = wsum(pp);
    // per-wave partials in alternating slots: one barrier per step
    const int sl = it & 1;
    if ((t & 63) == 0) {
      red[sl][0][t >> 6] = pr_re;
      red[sl][1][t >> 6] = pr_im;
      red[sl][2][t >> 6] = pp;
    }
    __syncthreads();
    T s0 = 0, s1 = 0, s2 = 0;
    for (int k = q * wpr; k < (q + 1) * wpr; ++k) {
      s0 += red[sl][0][k];
      s1 += red[sl][1][k];
      s2 += red[sl][2][k];
    }
    const cx<T> al = s2 > T(0) ? cx<T>{s0 / s2, s1 / s2} : cx<T>{T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      xs[k] = fma_c(al, rr[k], xs[k]);
      rr[k] = fma_c(cx<T>{-al.re, -al.im}, pe[k], rr[k]);
    }
  }
  // odd reconstruction: v_o = A_o^{-1} (rho_o + 1/2 H_L v_e)
  hop(1, xs, acc);
  cx<T> vo[12];
  {
    cx<T> hh[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) hh[k] = cacc(ro[k], T(0.5), acc[k]);
    clover(1, hh, vo);
  }
  if (!act) return;
  put(0, xs);
  put(1, vo);
  cx<T> zero[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) zero[k] = {T(0), T(0)};
  st_spinor<S, O32>(rho[0], r, ig[0], rr);
  st_spinor<S, O32>(rho[1], r, ig[1], zero);
}

template <class S, class P, int R, bool CL, bool O32>
__global__ void __launch_bounds__(R * kSapMaxHalf, (sap_lds_wgs<S, P, R, CL>())) k_sap_lds(SapArgs<S, P> a) {
  sap_lds_body<S, P, R, CL, O32>(a, blockIdx.x, gridDim.x);
}
template <class S, class P, int R, bool CL, bool O32>
__global__ void __launch_bounds__(R * kSapMaxHalf, (sap_lds_wgs<S, P, R, CL>())) k_sap_lds_grp(Grp<SapArgs<S, P>> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  sap_lds_body<S, P, R, CL, O32>(G.a[s], blockIdx.x - G.start[s], G.start[s + 1] - G.start[s]);
}

// One lane per even/odd site pair of the block: lane j owns the j-th even and
// the j-th odd site (block-local order), so every lane is busy in both halves
// of a hop (source side: projections into LDS; target side: transport and
// accumulation) and in both clover applications.  Links and clover are read
// from memory (L2) where they are used, which keeps the registers for the
// block-solve vectors.
template <class S, class P, int DR, bool O32>
__global__ void __launch_bounds__(kSapMaxHalf, sizeof(S) == 8 ? 1 : 2) k_sap_pair(SapArgs<S, P> a) {
  typedef typename St<S>::T T;
  __shared__ Exch<T, 2 * DR> ex;
  __shared__ T red[2][4];
  // per-lane vectors parked in LDS (each lane touches only its own column):
  // the odd-site source rho_o (needed again for the reconstruction) and the
  // even-site MR solution x
  __shared__ cx<T> ro_l[12][kSapMaxHalf], xs_l[12][kSapMaxHalf];
  const Geo& g = a.g;
  const int j = threadIdx.x;
  // this block: the sap_xcd_block(blockIdx.x)-th block of colour a.col
  int bc[4];
  {
    int bl = 2 * sap_xcd_block(blockIdx.x, gridDim.x);
    bc[3] = bl % a.nb[3];
    int rr = bl / a.nb[3];
    bc[2] = rr % a.nb[2];
    rr /= a.nb[2];
    bc[1] = rr % a.nb[1];
    bc[0] = rr / a.nb[1];
    bc[3] += (a.col + bc[0] + bc[1] + bc[2] + bc[3]) & 1;
  }
  // the lane's two sites (q = 0 even, 1 odd): global coordinates, index within
  // the parity, and neighbour slots inside the block (-1: the hop crosses a face)
  int x[2][4], ig[2], nin[2][4][2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    int y[4];
    int l = 2 * j;
    y[3] = l % a.bs[3];
    int rr = l / a.bs[3];
    y[2] = rr % a.bs[2];
    rr /= a.bs[2];
    y[1] = rr % a.bs[1];
    y[0] = rr / a.bs[1];
    y[3] += (q + y[0] + y[1] + y[2] + y[3]) & 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) x[q][m] = bc[m] * a.bs[m] + y[m];
    ig[q] = lex_of(g, x[q]) >> 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        int z[4] = {y[0], y[1], y[2], y[3]};
        z[m] += d == 0 ? 1 : -1;
        bool in = z[m] >= 0 && z[m] < a.bs[m];
        nin[q][m][d] = in ? ((((z[0] * a.bs[1] + z[1]) * a.bs[2] + z[2]) * a.bs[3] + z[3]) >> 1) : -1;
      }
    }
  }
  // clover: A on even sites, A^{-1} on odd sites
  // Link and clover addresses are formed from the site index plus an opaque zero
  // at every use: otherwise the compiler hoists all of them (two sites x 72
  // components) out of the loops and runs out of registers.
  auto vsalt = []() {
    int z = 0;
    asm volatile("" : "+v"(z));
    return z;
  };
  auto clover = [&](int q, const cx<T> in[12], cx<T> out[12]) {
    const CloverV<S>& c = q == 0 ? a.A : a.Ai;
    clover_apply<S>(c, q, ig[q] + vsalt(), in, out);
  };
  // acc (at the lane's site of parity 1-sp) = H_L src (src: the lane's site of parity sp)
  auto hop_block = [&](const int sp, const cx<T> src[12], cx<T> acc[12]) {
    const int tp = 1 - sp;
    const LinkV<S>& U = a.U;
    const int zv = vsalt();
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
#pragma unroll
    for (int r0 = 0; r0 < 4; r0 += DR) {
#pragma unroll
      for (int m = r0; m < r0 + DR; ++m) {
        cx<T> h[6], gg[6], u[9];
        // for the backward neighbour's forward hop: (1 - g_m) projection
        if (m == 0) project<T, 0, +1>(src, h);
        else if (m == 1) project<T, 1, +1>(src, h);
        else if (m == 2) project<T, 2, +1>(src, h);
        else project<T, 3, +1>(src, h);
#pragma unroll
        for (int k = 0; k < 6; ++k) ex.v[2 * (m - r0)][k][j] = h[k];
        // for the forward neighbour's backward hop: U^dag (1 + g_m) projection
        if (m == 0) project<T, 0, -1>(src, h);
        else if (m == 1) project<T, 1, -1>(src, h);
        else if (m == 2) project<T, 2, -1>(src, h);
        else project<T, 3, -1>(src, h);
        ld_link(U, sp, m, ig[sp] + zv, u);
        su3_mul_half<T, true>(u, h, gg);
#pragma unroll
        for (int k = 0; k < 6; ++k) ex.v[2 * (m - r0) + 1][k][j] = gg[k];
      }
      __syncthreads();
#pragma unroll
      for (int m = r0; m < r0 + DR; ++m) {
        const int jf = nin[tp][m][0], jb = nin[tp][m][1];
        cx<T> h[6], gg[6], u[9];
        if (jf >= 0) {
#pragma unroll
          for (int k = 0; k < 6; ++k) h[k] = ex.v[2 * (m - r0)][k][jf];
          ld_link(U, tp, m, ig[tp] + zv, u);
          su3_mul_half<T, false>(u, h, gg);
          if (m == 0) reconstruct_add<T, 0, +1>(gg, acc);
          else if (m == 1) reconstruct_add<T, 1, +1>(gg, acc);
          else if (m == 2) reconstruct_add<T, 2, +1>(gg, acc);
          else reconstruct_add<T, 3, +1>(gg, acc);
        }
        if (jb >= 0) {
#pragma unroll
          for (int k = 0; k < 6; ++k) gg[k] = ex.v[2 * (m - r0) + 1][k][jb];
          if (m == 0) reconstruct_add<T, 0, -1>(gg, acc);
          else if (m == 1) reconstruct_add<T, 1, -1>(gg, acc);
          else if (m == 2) reconstruct_add<T, 2, -1>(gg, acc);
          else reconstruct_add<T, 3, -1>(gg, acc);
        }
      }
      __syncthreads();
    }
  };
  auto block_sum3 = [&](T v0, T v1, T v2, T& s0, T& s1, T& s2) {
    v0 = wsum(v0);
    v1 = wsum(v1);
    v2 = wsum(v2);
    const int w = j >> 6, nw = (blockDim.x + 63) >> 6;
    if ((j & 63) == 0) {
      red[w][0] = v0;
      red[w][1] = v1;
      red[w][2] = v2;
    }
    __syncthreads();
    s0 = s1 = s2 = T(0);
    for (int k = 0; k < nw; ++k) {
      s0 += red[k][0];
      s1 += red[k][1];
      s2 += red[k][2];
    }
    __syncthreads();
  };
  // parity views of the fields
  FieldV<S> rho[2] = {a.rho, a.rho}, vf[2] = {a.V, a.V};
  FieldV<P> psi[2] = {a.psi, a.psi};
  rho[1].p += a.poff;
  vf[1].p += a.poff;
  psi[1].p += a.poff;
  if (a.rho.scale) {
    rho[1].scale += a.spoff;
    vf[1].scale += a.spoff;
  }
  if (a.psi.scale) psi[1].scale += a.spoff;

  // rq += 1/2 H_face V at the lane's site of parity q (the sites across the faces
  // belong to blocks of the other colour, whose corrections V the previous
  // half-sweep stored)
  auto bnd = [&](const int q, const int r, cx<T> (&rq)[12]) {
    const LinkV<S>& U = a.U;
    const int zv = vsalt();  // opaque per-lane zero: keeps the addresses inside the loop
    cx<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {T(0), T(0)};
    const FieldV<S>& vn = vf[1 - q];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      cx<T> sv[12], h[6], gg[6], u[9];
      if (nin[q][m][0] < 0) {
        int jn = nbr_idx(g, x[q], m, +1) + zv;
        ld_spinor<S, O32>(vn, r, jn, sv);
        ld_link(U, q, m, ig[q] + zv, u);
        if (m == 0) { project<T, 0, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 0, +1>(gg, acc); }
        else if (m == 1) { project<T, 1, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 1, +1>(gg, acc); }
        else if (m == 2) { project<T, 2, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 2, +1>(gg, acc); }
        else { project<T, 3, +1>(sv, h); su3_mul_half<T, false>(u, h, gg); reconstruct_add<T, 3, +1>(gg, acc); }
      }
      if (nin[q][m][1] < 0) {
        int jn = nbr_idx(g, x[q], m, -1) + zv;
        ld_spinor<S, O32>(vn, r, jn, sv);
        ld_link(a.U, 1 - q, m, jn, u);
        if (m == 0) { project<T, 0, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 0, -1>(gg, acc); }
        else if (m == 1) { project<T, 1, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 1, -1>(gg, acc); }
        else if (m == 2) { project<T, 2, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 2, -1>(gg, acc); }
        else { project<T, 3, -1>(sv, h); su3_mul_half<T, true>(u, h, gg); reconstruct_add<T, 3, -1>(gg, acc); }
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) rq[k] = cacc(rq[k], T(0.5), acc[k]);
  };
  // psi += v, V = v at the lane's site of parity q
  auto put = [&](const int q, const int r, const cx<T> (&v)[12]) {
    typedef typename St<P>::T TP;
    cx<TP> pv[12];
    if (a.first) {
#pragma unroll
      for (int k = 0; k < 12; ++k) pv[k] = {(TP)v[k].re, (TP)v[k].im};
    } else {
      ld_spinor<P, O32>(psi[q], r, ig[q], pv);
#pragma unroll
      for (int k = 0; k < 12; ++k) pv[k] = pv[k] + cx<TP>{(TP)v[k].re, (TP)v[k].im};
    }
    st_spinor<P, O32>(psi[q], r, ig[q], pv);
    if (a.write_v) st_spinor<S, O32>(vf[q], r, ig[q], v);
  };

  for (int r = 0; r < a.nrhs; ++r) {
    cx<T> re[12], ro[12];
    ld_spinor<S, O32>(rho[0], r, ig[0], re);
    ld_spinor<S, O32>(rho[1], r, ig[1], ro);
    // boundary: rho += 1/2 H_face V (the sites across the faces belong to blocks
    // of the other colour, whose corrections V the previous half-sweep stored)
    if (a.do_bnd) {
      bnd(0, r, re);
      bnd(1, r, ro);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      ro_l[k][j] = ro[k];
      xs_l[k][j] = {T(0), T(0)};
    }
    // source reduction: w = A_o^{-1} rho_o; b = rho_e + 1/2 H_L w
    cx<T> w[12], acc[12], rr[12], pe[12];
    clover(1, ro, w);
    hop_block(1, w, acc);
#pragma unroll
    for (int k = 0; k < 12; ++k) rr[k] = cacc(re[k], T(0.5), acc[k]);
    // minimal-residual steps on Dhat_L (even sites)
    for (int it = 0; it < a.nmr; ++it) {
      hop_block(0, rr, acc);  // odd sites: acc = H_L r
      cx<T> hh[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) hh[k] = T(-0.5) * acc[k];
      clover(1, hh, w);       // w = A_o^{-1} (-1/2 H r)
      hop_block(1, w, acc);   // even sites: acc = H_L w
      clover(0, rr, pe);
      T pr_re = 0, pr_im = 0, pp = 0;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        pe[k] = cacc(pe[k], T(0.5), acc[k]);
        pr_re = fmar(pe[k].re, rr[k].re, fmar(pe[k].im, rr[k].im, pr_re));
        pr_im = fmar(pe[k].re, rr[k].im, fmar(-pe[k].im, rr[k].re, pr_im));
        pp = fmar(pe[k].re, pe[k].re, fmar(pe[k].im, pe[k].im, pp));
      }
      T s0, s1, s2;
      block_sum3(pr_re, pr_im, pp, s0, s1, s2);
      cx<T> al = s2 > T(0) ? cx<T>{s0 / s2, s1 / s2} : cx<T>{T(0), T(0)};
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        xs_l[k][j] = fma_c(al, rr[k], xs_l[k][j]);
        rr[k] = fma_c(cx<T>{-al.re, -al.im}, pe[k], rr[k]);
      }
    }
    // odd reconstruction: v_o = A_o^{-1} (rho_o + 1/2 H_L v_e)
    cx<T> xs[12], vo[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) xs[k] = xs_l[k][j];
    hop_block(0, xs, acc);
    {
      cx<T> hh[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) hh[k] = cacc(ro_l[k][j], T(0.5), acc[k]);
      clover(1, hh, vo);
    }
    // write back: psi += v, V = v, rho = new block residual (r even, 0 odd)
    put(0, r, xs);
    put(1, r, vo);
    cx<T> zero[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) zero[k] = {T(0), T(0)};
    st_spinor<S, O32>(rho[0], r, ig[0], rr);
    st_spinor<S, O32>(rho[1], r, ig[1], zero);
  }
}

// every element offset of a field of nrhs right-hand sides (both parities) below 2^32 bytes
template <class S>
static bool sap_fits32(const FieldV<S>& f, int nrhs, int64_t poff, int64_t spoff) {
  const int64_t lim = (int64_t)1 << 32;
  int64_t e = ((int64_t)(nrhs - 1) * f.rs + poff + f.n) * (int64_t)sizeof(typename St<S>::E);
  int64_t sc = f.scale ? ((int64_t)(nrhs - 1) * f.srs + spoff + f.n) * 4 : 0;
  return e < lim && sc < lim;
}

// Face corrections of a half-sweep (the hops across the block faces from the
// sites of the neighbouring blocks, the other colour, whose corrections V the
// previous half-sweep stored):
//   rho += 1/2 H_face V.
// One lane per site of the blocks of colour a.col: the lanes enumerate only
// those sites (in an x3 row of a parity they are the runs of bs3/2 consecutive
// sites of every other block), load the links of the site's faces once and loop
// over the right-hand sides; consecutive lanes take consecutive sites, so the
// loads of rho and V are coalesced in runs of bs3/2.  The half-sweep then runs
// without its own face terms.
template <class S, class P>
__device__ __forceinline__ void sap_face_body(const SapArgs<S, P>& a, int bx) {
  typedef typename St<S>::T T;
  const Geo& g = a.g;
  const int t = bx * blockDim.x + threadIdx.x, p = blockIdx.y;
  const int hb = a.bs[3] >> 1, per_row = g.Lh3 >> 1;  // colour sites of a parity per x3 row
  if (t >= (g.Vh >> 1)) return;
  const int row = t / per_row, jr = t - row * per_row;
  int x[4];
  x[2] = row % g.L[2];
  x[1] = (row / g.L[2]) % g.L[1];
  x[0] = row / (g.L[2] * g.L[1]);
  const int k = jr / hb, o = jr - k * hb;
  const int bc3 = 2 * k + ((a.col + x[0] / a.bs[0] + x[1] / a.bs[1] + x[2] / a.bs[2]) & 1);
  const int i = row * g.Lh3 + bc3 * hb + o;
  x[3] = 2 * (bc3 * hb + o) + ((p + x[0] + x[1] + x[2]) & 1);
  int y[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) y[m] = x[m] - (x[m] / a.bs[m]) * a.bs[m];
  // the faces of the site: at most one per direction (even block extents >= 2);
  // their links kept in the storage type (FP16: half the registers)
  typedef typename St<S>::E E;
  E ur[4][9];
  int nb[4], dir[4];
  bool any = false;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    dir[m] = y[m] == a.bs[m] - 1 ? 1 : (y[m] == 0 ? -1 : 0);
    nb[m] = 0;
    // forward neighbour in the next block: the site's own link; backward: the neighbour's
    if (dir[m] != 0) nb[m] = nbr_idx(g, x, m, dir[m]);
    const E* ub = a.U.p + (int64_t)((dir[m] > 0 ? p : 1 - p) * 4 + m) * 9 * a.U.n + (dir[m] > 0 ? i : nb[m]);
#pragma unroll
    for (int c = 0; c < 9; ++c) ur[m][c] = dir[m] != 0 ? ub[(int64_t)c * a.U.n] : E{};
    any = any || dir[m] != 0;
  }
  if (!any) return;  // an interior site: nothing crosses a face
  FieldV<S> rho = a.rho, vn = a.V;
  rho.p += (int64_t)p * a.poff;
  vn.p += (int64_t)(1 - p) * a.poff;
  if (a.rho.scale) {
    rho.scale += (int64_t)p * a.spoff;
    vn.scale += (int64_t)(1 - p) * a.spoff;
  }
#pragma unroll 1
  for (int r = 0; r < a.nrhs; ++r) {
    cx<T> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {T(0), T(0)};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      cx<T> sv[12], h[6], gg[6], u[4][9];
      // FP16: convert at every use (an opaque copy of the stored link per
      // right-hand side keeps the compiler from holding all converted links)
      if constexpr (sizeof(S) == 2) {
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          uint32_t w = __builtin_bit_cast(uint32_t, ur[m][c]);
          asm volatile("" : "+v"(w));
          u[m][c] = St<S>::from(__builtin_bit_cast(E, w));
        }
      } else {
#pragma unroll
        for (int c = 0; c < 9; ++c) u[m][c] = St<S>::from(ur[m][c]);
      }
      if (dir[m] > 0) {
        ld_spinor<S>(vn, r, nb[m], sv);
        if (m == 0) { project<T, 0, +1>(sv, h); su3_mul_half<T, false>(u[m], h, gg); reconstruct_add<T, 0, +1>(gg, acc); }
        else if (m == 1) { project<T, 1, +1>(sv, h); su3_mul_half<T, false>(u[m], h, gg); reconstruct_add<T, 1, +1>(gg, acc); }
        else if (m == 2) { project<T, 2, +1>(sv, h); su3_mul_half<T, false>(u[m], h, gg); reconstruct_add<T, 2, +1>(gg, acc); }
        else { project<T, 3, +1>(sv, h); su3_mul_half<T, false>(u[m], h, gg); reconstruct_add<T, 3, +1>(gg, acc); }
      } else if (dir[m] < 0) {
        ld_spinor<S>(vn, r, nb[m], sv);
        if (m == 0) { project<T, 0, -1>(sv, h); su3_mul_half<T, true>(u[m], h, gg); reconstruct_add<T, 0, -1>(gg, acc); }
        else if (m == 1) { project<T, 1, -1>(sv, h); su3_mul_half<T, true>(u[m], h, gg); reconstruct_add<T, 1, -1>(gg, acc); }
        else if (m == 2) { project<T, 2, -1>(sv, h); su3_mul_half<T, true>(u[m], h, gg); reconstruct_add<T, 2, -1>(gg, acc); }
        else { project<T, 3, -1>(sv, h); su3_mul_half<T, true>(u[m], h, gg); reconstruct_add<T, 3, -1>(gg, acc); }
      }
    }
    cx<T> rv[12];
    ld_spinor<S>(rho, r, i, rv);
#pragma unroll
    for (int c = 0; c < 12; ++c) rv[c] = cacc(rv[c], T(0.5), acc[c]);
    st_spinor<S>(rho, r, i, rv);
  }
}

// (FP32 / FP16: at least two wavefronts per SIMD; the loop over the right-hand
// sides keeps the face links and up to four neighbour spinors live)
template <class S, class P>
__global__ void __launch_bounds__(256, sizeof(S) == 8 ? 1 : 2) k_sap_face(SapArgs<S, P> a) {
  sap_face_body<S, P>(a, blockIdx.x);
}
template <class S, class P>
__global__ void __launch_bounds__(256, sizeof(S) == 8 ? 1 : 2) k_sap_face_grp(Grp<SapArgs<S, P>> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  sap_face_body<S, P>(G.a[s], blockIdx.x - G.start[s]);
}

template <class S, class P>
hipError_t launch_sap_face(const SapArgs<S, P>& a, hipStream_t st) {
  const dim3 grid((unsigned)((a.g.Vh / 2 + 255) / 256), 2), blk(256);
  hipLaunchKernelGGL((k_sap_face<S, P>), grid, blk, 0, st, a);
  return hipGetLastError();
}

template <class S, class P>
hipError_t launch_sap_half(const SapArgs<S, P>& a, int nblk_colour, hipStream_t st) {
  int nsb = a.bs[0] * a.bs[1] * a.bs[2] * a.bs[3];
  if (nsb > 2 * kSapMaxHalf || nblk_colour <= 0) return hipErrorInvalidValue;
  if constexpr (sizeof(S) == 8) {
    // FP64: one lane per site pair (the per-site variant would hold links and
    // clover in registers only for FP32/FP16 storage)
    const bool o32 = sap_fits32(a.rho, a.nrhs, a.poff, a.spoff) && sap_fits32(a.V, a.nrhs, a.poff, a.spoff) &&
                     sap_fits32(a.psi, a.nrhs, a.poff, a.spoff);
    if (o32)
      hipLaunchKernelGGL((k_sap_pair<S, P, 2, true>), dim3(nblk_colour), dim3(nsb / 2), 0, st, a);
    else
      hipLaunchKernelGGL((k_sap_pair<S, P, 2, false>), dim3(nblk_colour), dim3(nsb / 2), 0, st, a);
  } else {
    const int v = a.variant ? a.variant : sap_default_variant(sizeof(S) == 2 ? 2 : 1);
    const bool o32 = sap_fits32(a.rho, a.nrhs, a.poff, a.spoff) && sap_fits32(a.V, a.nrhs, a.poff, a.spoff) &&
                     sap_fits32(a.psi, a.nrhs, a.poff, a.spoff);
    if (v == kSapPerSite) {
      // one lane per site, own links and clover in registers, rhs one after another
      hipLaunchKernelGGL((k_sap_half<S, P, 4>), dim3(nblk_colour), dim3(nsb), 0, st, a);
    } else if (v == kSapPerRhs) {
      // one workgroup per (block, right-hand side)
      const dim3 grid((unsigned)nblk_colour * (unsigned)a.nrhs), blk(nsb / 2);
      if (o32) hipLaunchKernelGGL((k_sap_rhs<S, P, true>), grid, blk, 0, st, a);
      else hipLaunchKernelGGL((k_sap_rhs<S, P, false>), grid, blk, 0, st, a);
    } else if constexpr (sizeof(S) == 4) {
      if (v != kSapStaged) return hipErrorInvalidValue;
      // FP32: one workgroup per (block, group of 4 right-hand sides), the block's
      // links staged in LDS, the clover blocks read from memory
      constexpr int R = 4;
      const int nhp = ((nsb / 2) + 63) & ~63;
      const dim3 grid((unsigned)nblk_colour * (unsigned)((a.nrhs + R - 1) / R)), blk(R * nhp);
      if (o32) hipLaunchKernelGGL((k_sap_lds<S, P, R, false, true>), grid, blk, 0, st, a);
      else hipLaunchKernelGGL((k_sap_lds<S, P, R, false, false>), grid, blk, 0, st, a);
    } else if constexpr (sizeof(S) == 2) {
      const int nhp = ((nsb / 2) + 63) & ~63;
      if (v == kSapStaged) {
        // one workgroup per (block, group of 4 right-hand sides), the block's links
        // and clover staged in LDS
        constexpr int R = 4;
        const dim3 grid((unsigned)nblk_colour * (unsigned)((a.nrhs + R - 1) / R)), blk(R * nhp);
        if (o32) hipLaunchKernelGGL((k_sap_lds<S, P, R, true, true>), grid, blk, 0, st, a);
        else hipLaunchKernelGGL((k_sap_lds<S, P, R, true, false>), grid, blk, 0, st, a);
      } else if (v == kSapStagedLinks) {
        // one workgroup per (block, pair of right-hand sides), the links staged
        // in LDS, two workgroups per CU
        constexpr int R = 2;
        const dim3 grid((unsigned)nblk_colour * (unsigned)((a.nrhs + R - 1) / R)), blk(R * nhp);
        if (o32) hipLaunchKernelGGL((k_sap_lds<S, P, R, false, true>), grid, blk, 0, st, a);
        else hipLaunchKernelGGL((k_sap_lds<S, P, R, false, false>), grid, blk, 0, st, a);
      } else {
        return hipErrorInvalidValue;
      }
    } else {
      return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

// several systems, FP32 storage (variants 1, 2, 3) or FP16 storage (1 to 4),
// every system with the same variant and block volume
template <class S, class P>
hipError_t launch_sap_face_grp(const SapArgs<S, P>* a, int ns, hipStream_t st) {
  if (ns < 1 || ns > kGrpMax) return hipErrorInvalidValue;
  Grp<SapArgs<S, P>> G = grp_new<SapArgs<S, P>>();
  for (int s = 0; s < ns; ++s) grp_add(G, a[s], (a[s].g.Vh / 2 + 255) / 256);
  hipLaunchKernelGGL((k_sap_face_grp<S, P>), dim3(G.start[ns], 2), dim3(256), 0, st, G);
  return hipGetLastError();
}

template <class S, class P>
hipError_t launch_sap_half_grp(const SapArgs<S, P>* a, int ns, hipStream_t st) {
  static_assert(sizeof(S) <= 4, "grouped half-sweeps: FP32 or FP16 storage");
  if (ns < 1 || ns > kGrpMax) return hipErrorInvalidValue;
  const int nsb = a[0].bs[0] * a[0].bs[1] * a[0].bs[2] * a[0].bs[3];
  const int vdef = sap_default_variant(sizeof(S) == 2 ? 2 : 1);
  const int v = a[0].variant ? a[0].variant : vdef;
  if (nsb > 2 * kSapMaxHalf) return hipErrorInvalidValue;
  Grp<SapArgs<S, P>> G = grp_new<SapArgs<S, P>>();
  bool o32 = true;
  for (int s = 0; s < ns; ++s) {
    const SapArgs<S, P>& b = a[s];
    const int vs = b.variant ? b.variant : vdef;
    if (b.bs[0] * b.bs[1] * b.bs[2] * b.bs[3] != nsb || vs != v) return hipErrorInvalidValue;
    const int nblk = b.nb[0] * b.nb[1] * b.nb[2] * b.nb[3] / 2;
    o32 = o32 && sap_fits32(b.rho, b.nrhs, b.poff, b.spoff) && sap_fits32(b.V, b.nrhs, b.poff, b.spoff) &&
          sap_fits32(b.psi, b.nrhs, b.poff, b.spoff);
    const int per = v == kSapPerRhs ? b.nrhs : v == kSapStaged ? (b.nrhs + 3) / 4
                    : v == kSapStagedLinks ? (b.nrhs + 1) / 2 : 1;
    grp_add(G, b, nblk * per);
  }
  if (v == kSapPerSite) {
    hipLaunchKernelGGL((k_sap_half_grp<S, P, 4>), dim3(G.start[ns]), dim3(nsb), 0, st, G);
  } else if (v == kSapPerRhs) {
    if (o32) hipLaunchKernelGGL((k_sap_rhs_grp<S, P, true>), dim3(G.start[ns]), dim3(nsb / 2), 0, st, G);
    else hipLaunchKernelGGL((k_sap_rhs_grp<S, P, false>), dim3(G.start[ns]), dim3(nsb / 2), 0, st, G);
  } else if (v == kSapStaged) {
    // 4 rhs per workgroup; FP16 also stages the clover blocks
    constexpr bool CL = sizeof(S) == 2;
    const dim3 blk(4 * (((nsb / 2) + 63) & ~63));
    if (o32) hipLaunchKernelGGL((k_sap_lds_grp<S, P, 4, CL, true>), dim3(G.start[ns]), blk, 0, st, G);
    else hipLaunchKernelGGL((k_sap_lds_grp<S, P, 4, CL, false>), dim3(G.start[ns]), blk, 0, st, G);
  } else if (v == kSapStagedLinks) {
    if constexpr (sizeof(S) == 2) {
      const dim3 blk(2 * (((nsb / 2) + 63) & ~63));
      if (o32) hipLaunchKernelGGL((k_sap_lds_grp<S, P, 2, false, true>), dim3(G.start[ns]), blk, 0, st, G);
      else hipLaunchKernelGGL((k_sap_lds_grp<S, P, 2, false, false>), dim3(G.start[ns]), blk, 0, st, G);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_sap_face_grp<float, float>(const SapArgs<float, float>*, int, hipStream_t);
template hipError_t launch_sap_half_grp<float, float>(const SapArgs<float, float>*, int, hipStream_t);
template hipError_t launch_sap_face_grp<__half, float>(const SapArgs<__half, float>*, int, hipStream_t);
template hipError_t launch_sap_half_grp<__half, float>(const SapArgs<__half, float>*, int, hipStream_t);

template hipError_t launch_sap_half<double, double>(const SapArgs<double, double>&, int, hipStream_t);
template hipError_t launch_sap_face<double, double>(const SapArgs<double, double>&, hipStream_t);
template hipError_t launch_sap_face<float, float>(const SapArgs<float, float>&, hipStream_t);
template hipError_t launch_sap_face<__half, float>(const SapArgs<__half, float>&, hipStream_t);
template hipError_t launch_sap_half<float, float>(const SapArgs<float, float>&, int, hipStream_t);
template hipError_t launch_sap_half<__half, float>(const SapArgs<__half, float>&, int, hipStream_t);

}  // namespace qdd
