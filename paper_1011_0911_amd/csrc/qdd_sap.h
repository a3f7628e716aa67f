// Arguments of the Schwarz half-sweep kernel (qdd_sap.hip).
#pragma once
#include "qdd_kernels.h"

namespace qdd {
constexpr int kSapMaxHalf = 128;  // even (= odd) sites per block

template <class S, class P>
struct SapArgs {
  Geo g;
  int bs[4], nb[4];  // block extents, blocks per direction
  int col;           // colour of the blocks of this half-sweep
  int nrhs, nmr;
  int do_bnd;   // apply the face corrections of the previous half-sweep inside the half-sweep
                // (the solver applies them with launch_sap_face first and clears it)
  int first;    // psi not yet written on these blocks (first cycle)
  int write_v;  // store the correction for the next half-sweep
  int variant;  // FP32/FP16 kernel: 1 per-site (registers), 2 per (block, rhs), 3 LDS-staged links and
                // (FP16) clover, 4 rhs per workgroup, 4 LDS-staged links, 2 rhs (FP16 only)
  LinkV<S> U;
  CloverV<S> A, Ai;
  FieldV<S> rho, V;  // full fields [rhs][parity][12][Vh]
  FieldV<P> psi;
  int64_t poff, spoff;  // parity offsets (elements, scales)
};

// variants of the FP32 / FP16 half-sweep kernel (FP64 has one)
constexpr int kSapPerSite = 1, kSapPerRhs = 2, kSapStaged = 3, kSapStagedLinks = 4;
// the variant used when none was set: the LDS-staged kernel for FP16 storage,
// the per-site one for FP32
inline int sap_default_variant(int prec) { return prec == 2 ? kSapStaged : kSapPerSite; }
inline bool sap_variant_ok(int prec, int v) { return prec != 0 && v >= 1 && v <= (prec == 2 ? 4 : 3); }

template <class S, class P>
hipError_t launch_sap_half(const SapArgs<S, P>& a, int nblk_colour, hipStream_t st);
// rho += 1/2 H_face V on the sites of the blocks of colour a.col (the face
// corrections of a half-sweep, applied before it with do_bnd off)
template <class S, class P>
hipError_t launch_sap_face(const SapArgs<S, P>& a, hipStream_t st);
// the same two steps for ns systems in one launch each (FP32 storage; every
// system with the same block volume and variant, 1, 2 or 3)
template <class S, class P>
hipError_t launch_sap_face_grp(const SapArgs<S, P>* a, int ns, hipStream_t st);
template <class S, class P>
hipError_t launch_sap_half_grp(const SapArgs<S, P>* a, int ns, hipStream_t st);
}  // namespace qdd
