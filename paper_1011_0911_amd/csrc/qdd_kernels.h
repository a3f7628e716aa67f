// Launcher declarations shared by the kernel translation units and the host
// library (qdd_api.cpp).
#pragma once
#include "qdd_internal.h"

namespace qdd {

// operator data of one storage precision
template <class S>
struct DevOp {
  LinkV<S> U;       // hopping links (boundary sign folded in)
  CloverV<S> A;     // A(x) on both parities
  CloverV<S> Ainv;  // A(x)^{-1} on both parities
};

// launch shape (picked by the autotuner)
struct LaunchCfg {
  int block = 256;  // threads per block
  int nr = 1;       // right-hand sides per thread (register reuse of the links); 0 = staged
                    // variant: the tile's links and clover in LDS, each lane loops over rhs
  int xcd = 2;      // block walk: 0 linear, 1 XCD slabs, 2 XCD slabs walked time-slice first,
                    // 3 XCD slabs of L1/8 x1 planes walked time slice by time slice; Dhat with nr 1:
                    // + 4 streaming loads of links and clover, + 8 streaming load of the
                    // site's own spinor and store of the output (data a pass touches once),
                    // + 16 compressed links (two rows read, the third rebuilt); Dhat with nr 2, 4:
                    // + 32 a lane loads its nr right-hand sides of a component in one word
                    // (interleaved batches; the streaming and compression bits then apply too);
                    // Dhat (nr >= 1): + 64 pass B walks the tiles backwards
  int sb = 0;       // sites per block (0 = block); block/sb lane groups take further rhs
};

// Dhat with the rhs-vector loads (walk field + 32): nr consecutive right-hand
// sides of a site in one load of at most 16 bytes (FP32: nr 2; FP16: nr 2, 4)
inline bool dhat_vec_ok(int prec, int nr) { return (prec == 1 && nr == 2) || (prec == 2 && (nr == 2 || nr == 4)); }

// LDS bytes of the staged Dhat variant for a tile of sb sites (108 complex slots
// per site: 8 links and the clover), and the budget it must stay within
inline size_t staged_lds_bytes(int prec, int sb) {
  return (size_t)108 * sb * (prec == 0 ? 16 : prec == 1 ? 8 : 4);
}
constexpr size_t kStagedLdsMax = 64 * 1024;

// pass: bit 0 = pass A, bit 1 = pass B; ev (optional) is recorded between them
template <class S>
hipError_t launch_dhat(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> tmp, FieldV<S> out, int nrhs,
                       const LaunchCfg& c, hipStream_t st, int pass = 3, hipEvent_t ev = nullptr);
// plain HBM copy (16-byte vectors), the bandwidth reference
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
// shift (device, nrhs doubles, optional): per-rhs diagonal shifts of D, for
// several masses in one launch: D(kappa_r) = D(kappa_0) + (1/(2 kappa_r) -
// 1/(2 kappa_0)) because only the diagonal of the clover term depends on kappa
constexpr int kMaxShift = 64;
// ce (device, nrhs doubles, optional; not together with shift): per-rhs factor
// on the even sites' clover term, D'(r) = D + (ce[r] - 1) A_e on the even sites
template <class S>
hipError_t launch_dw(const Geo& g, const DevOp<S>& op, FieldV<S> in, FieldV<S> out, int64_t poff, int64_t spoff,
                     int nrhs, const LaunchCfg& c, hipStream_t st, const double* shift = nullptr,
                     const double* ce = nullptr);

// ---- several systems in one launch (the grouped solve of qdd_solve_multi)
// The workgroups of one launch are split among up to kGrpMax independent systems
// (different lattices, masses, batch sizes): system s owns the workgroups
// [start[s], start[s+1]) and runs the single-system kernel body on its own
// arguments a[s], with its own workgroup numbering, so every system computes
// exactly what its own launch would.  The table travels by value in the
// kernel-argument segment; ny is the extent of the second grid dimension (the
// largest right-hand-side count), whose surplus workgroups exit at once.
constexpr int kGrpMax = 12;
template <class A>
struct Grp {
  A a[kGrpMax];
  int start[kGrpMax + 1];
  int ns;
  int ny;
};
__device__ inline int grp_sys(const int* start, int ns, int b) {
  int s = 0;
  for (int j = 1; j < ns; ++j) s += b >= start[j];
  return s;
}
template <class A>
inline void grp_add(Grp<A>& G, const A& a, int nblk, int ny = 1) {
  static_assert(sizeof(Grp<A>) <= 4096, "a group table must fit the kernel-argument segment");
  if (G.ns == 0) {
    G.start[0] = 0;
    G.ny = 1;
  }
  G.a[G.ns] = a;
  G.start[G.ns + 1] = G.start[G.ns] + nblk;
  G.ny = ny > G.ny ? ny : G.ny;
  ++G.ns;
}
template <class A>
inline Grp<A> grp_new() {
  Grp<A> G;
  G.ns = 0;
  G.ny = 1;
  G.start[0] = 0;
  return G;
}

// full D of one system in a grouped launch (poff, spoff: parity offsets of the
// full fields; the launch fills in its walk of the tiles)
template <class S>
struct DwArgs {
  Geo g;
  LinkV<S> U;
  CloverV<S> A;
  FieldV<S> in, out;
  int64_t poff, spoff;
  int nrhs, nrg, order, sb;
};
// one launch of the full D over ns systems with the common launch shape c
// (block and rhs per lane shared, walk and tile size per system as c gives them)
template <class S>
hipError_t launch_dw_grp(const DwArgs<S>* a, int ns, const LaunchCfg& c, hipStream_t st);

// ---- packing / conversion (qdd_pack.hip)

// canonical complex128 links [V][4][3][3] -> FP64 internal hopping links (sign folded in)
hipError_t launch_pack_links(const Geo& g, const double* canon, double2* U, hipStream_t st);
// element-wise precision conversion of an array of n complex elements
hipError_t launch_convert(const double2* in, float2* out, int64_t n, hipStream_t st);
hipError_t launch_convert(const double2* in, __half2* out, int64_t n, hipStream_t st);
// canonical spinors [nrhs][V or Vh][4][3] complex128 <-> internal fields
// (even_only: canonical even-restricted input, internal [rhs][12][Vh]; otherwise
// internal full field [rhs][parity][12][Vh])
template <class S>
hipError_t launch_pack_spinor(const Geo& g, const double* canon, FieldV<S> f, int nrhs, int even_only, int64_t poff,
                              int64_t spoff, hipStream_t st);
template <class S>
hipError_t launch_unpack_spinor(const Geo& g, FieldV<S> f, double* canon, int nrhs, int even_only, int64_t poff,
                                int64_t spoff, hipStream_t st);
// convert between internal precisions (same layout): n sites per component, rhs count * parities
template <class SI, class SO>
hipError_t launch_field_convert(FieldV<SI> in, FieldV<SO> out, int nvec, hipStream_t st);
// the same over ns systems in one launch (in[s], out[s], nvec[s])
template <class SI, class SO>
hipError_t launch_field_convert_grp(const FieldV<SI>* in, const FieldV<SO>* out, const int* nvec, int ns,
                                    hipStream_t st);

// ---- clover (qdd_clover.hip)
// builds A and A^{-1} (FP64, both parities) from the FP64 internal links; counts
// blocks whose Cholesky factorisation fails into *bad (device int)
// Dirichlet blocks of the block solver: extents, blocks per direction, count,
// sites of one parity per block
struct BlkGeo {
  int bs[4], nb[4];
  int nblk, neb;
};
hipError_t launch_blk_gather(const Geo& g, const BlkGeo& B, const double2* U, const double2* A, const double2* Ai,
                             double2* BU, double2* BA, double2* BAi, hipStream_t st);
hipError_t launch_blk_bicgstab(const Geo& g, const BlkGeo& B, const double2* BU, const double2* BA,
                               const double2* BAi, double2* work, const double2* eta, double2* psi, int nrhs,
                               double tol, int maxit, int* iters, double* res, hipStream_t st);

// pseudofermion terms of the force: fields [parity][Vh][12] complex (X, Y and
// their odd-site images), the even source phi, weight c and clover shift s
struct FrcTerms {
  int nt = 0;
  const double2* X[2] = {nullptr, nullptr};
  const double2* Y[2] = {nullptr, nullptr};
  const double2* phi[2] = {nullptr, nullptr};
  double c[2] = {0, 0}, s[2] = {0, 0};
};
hipError_t launch_force_odd(const Geo& g, const DevOp<double>& op, int nt, double2* X, double2* Y, hipStream_t st);
hipError_t launch_force_src(const Geo& g, const DevOp<double>& op, const double2* psi, const double2* xi,
                            const double2* phi2, double dm, double2* src, hipStream_t st);
hipError_t launch_force(const Geo& g, const DevOp<double>& op, const double2* U, double det_w, double csw,
                        const FrcTerms& T, double* lt, double* force, hipStream_t st);

hipError_t launch_clover(const Geo& g, const double2* U, double diag, double csw, double2* A, double2* Ai, int* bad,
                         hipStream_t st);

// ---- mass preconditioning (qdd_action.hip)
// part[p * nb + b], nb = clover_logdet_blocks(Vh): partial sums over parity p of
// log det A(x) (NaN where a block is not positive definite)
int clover_logdet_blocks(int64_t Vh);
hipError_t launch_clover_logdet(const Geo& g, const CloverV<double>& A, double* part, hipStream_t st);
// out = A_e^{-1} out + dm in on even sites, nrhs right-hand sides (out holding Dhat in)
hipError_t launch_apply_w_finish(const Geo& g, const FieldV<double>& in, const FieldV<double>& out,
                                 const CloverV<double>& Ai, int nrhs, double dm, hipStream_t st);
// even sites of the full field eta (view with parity 0 at its base) = A_e phi,
// phi canonical even complex128 [rhs][site][4][3] (device)
hipError_t launch_qs_source(const Geo& g, const double* phi_c, const FieldV<double>& eta, const CloverV<double>& A,
                            int nrhs, hipStream_t st);

}  // namespace qdd
