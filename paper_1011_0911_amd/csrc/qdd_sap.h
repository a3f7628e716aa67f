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
  int do_bnd;   // apply the face corrections of the previous half-sweep
  int first;    // psi not yet written on these blocks (first cycle)
  int write_v;  // store the correction for the next half-sweep
  LinkV<S> U;
  CloverV<S> A, Ai;
  FieldV<S> rho, V;  // full fields [rhs][parity][12][Vh]
  FieldV<P> psi;
  int64_t poff, spoff;  // parity offsets (elements, scales)
};

template <class S, class P>
hipError_t launch_sap_half(const SapArgs<S, P>& a, int nblk_colour, hipStream_t st);
}  // namespace qdd
