// Internal definitions of the qdd HIP library (gfx950).
//
// Device data layout (everything parity-split, structure-of-arrays so that lane
// i of a wavefront touches site i and consecutive lanes read consecutive
// addresses):
//   * site index within a parity:  i = lex >> 1,  lex = ((x0*L1+x1)*L2+x2)*L3+x3
//   * spinor field (one parity, one right-hand side): 12 complex components,
//     stored component-major  f[k][i], k = 3*spin + colour
//   * gauge field (hopping copy): U[p][mu][k][i], k = 3*row + col, the fermion
//     time-boundary sign folded in (the clover build removes it again)
//   * clover: two Hermitian 6x6 chirality blocks per site, 18 "slots" each
//     (3 slots of diagonal pairs, 15 upper off-diagonal complex entries),
//     stored slot-major  A[p][slot][i]
//   * element type: double2 (FP64), float2 (FP32) or half2 (FP16 storage; the
//     spinors then carry one FP32 scale per site, |entries| <= 1 after scaling)
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <cstdint>

namespace qdd {

// --------------------------------------------------------------- complex
template <class T>
struct cx {
  T re, im;
};
template <class T>
__device__ __host__ inline cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <class T>
__device__ __host__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __host__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__device__ __host__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ __host__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T>
__device__ __host__ inline cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <class T>
__device__ __host__ inline cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <class T>
__device__ __host__ inline cx<T> ti(cx<T> a) { return {-a.im, a.re}; }
template <class T>
__device__ __host__ inline cx<T> tmi(cx<T> a) { return {a.im, -a.re}; }
// real fused multiply-add (one rounding); written out so that a complex
// multiply-accumulate is exactly two fused operations per real component
__device__ __host__ inline float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __host__ inline double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <class T>
__device__ __host__ inline cx<T> fma_c(cx<T> a, cx<T> b, cx<T> c) {  // a*b + c
  return {fmar(a.re, b.re, fmar(-a.im, b.im, c.re)), fmar(a.re, b.im, fmar(a.im, b.re, c.im))};
}
template <class T>
__device__ __host__ inline cx<T> fmac_c(cx<T> a, cx<T> b, cx<T> c) {  // conj(a)*b + c
  return {fmar(a.re, b.re, fmar(a.im, b.im, c.re)), fmar(a.re, b.im, fmar(-a.im, b.re, c.im))};
}

// --------------------------------------------------------------- storage
// Storage traits: element type E (one complex), accumulate type T.
template <class S>
struct St;
template <>
struct St<double> {
  typedef double2 E;
  typedef double T;
  static __device__ inline cx<double> ldc(const E* p) {  // cached load (re-used data)
    E v = *p;
    return {v.x, v.y};
  }
  static __device__ inline void st(E* p, cx<double> v) { *p = make_double2(v.re, v.im); }
  static __device__ inline cx<double> from(E v) { return {v.x, v.y}; }
  static __device__ inline cx<double> from_reg(E v) { return {v.x, v.y}; }
  static __device__ inline E to(cx<double> v) { return make_double2(v.re, v.im); }
};
template <>
struct St<float> {
  typedef float2 E;
  typedef float T;
  static __device__ inline cx<float> ldc(const E* p) {
    E v = *p;
    return {v.x, v.y};
  }
  static __device__ inline void st(E* p, cx<float> v) { *p = make_float2(v.re, v.im); }
  static __device__ inline cx<float> from(E v) { return {v.x, v.y}; }
  static __device__ inline cx<float> from_reg(E v) { return {v.x, v.y}; }
  static __device__ inline E to(cx<float> v) { return make_float2(v.re, v.im); }
};
template <>
struct St<__half> {
  typedef __half2 E;
  typedef float T;
  static __device__ inline cx<float> ldc(const E* p) {
    E v = *p;
    float2 f = __half22float2(v);
    return {f.x, f.y};
  }
  static __device__ inline void st(E* p, cx<float> v) { *p = __floats2half2_rn(v.re, v.im); }
  static __device__ inline cx<float> from(E v) {
    float2 f = __half22float2(v);
    return {f.x, f.y};
  }
  // converted once into registers (spinor components feed additions, where a
  // mixed-precision fused operation cannot absorb the conversion; leaving the
  // choice to the compiler costs far more registers)
  static __device__ inline cx<float> from_reg(E v) {
    float2 f = __half22float2(v);
    asm("" : "+v"(f.x), "+v"(f.y));
    return {f.x, f.y};
  }
  static __device__ inline E to(cx<float> v) { return __floats2half2_rn(v.re, v.im); }
};

// --------------------------------------------------------------- geometry
struct Geo {
  int L[4];
  int Lh3;     // L3 / 2
  int Vh;      // sites per parity
  int V;
  int bc;      // time-boundary sign of the fermion field (-1 antiperiodic)
};

// coordinates of site i of parity p
__device__ __host__ inline void site_coords(const Geo& g, int p, int i, int x[4]) {
  int row = i / g.Lh3;
  int h = i - row * g.Lh3;
  x[2] = row % g.L[2];
  int t = row / g.L[2];
  x[1] = t % g.L[1];
  x[0] = t / g.L[1];
  x[3] = 2 * h + ((p + x[0] + x[1] + x[2]) & 1);
}

__device__ __host__ inline int lex_of(const Geo& g, const int x[4]) {
  return ((x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
}

// index (in the opposite parity) of x + mu (dir = +1) or x - mu (dir = -1)
__device__ __host__ inline int nbr_idx(const Geo& g, const int x[4], int mu, int dir) {
  int y[4] = {x[0], x[1], x[2], x[3]};
  int v = y[mu] + dir;
  y[mu] = v < 0 ? v + g.L[mu] : (v >= g.L[mu] ? v - g.L[mu] : v);
  return lex_of(g, y) >> 1;
}

// --------------------------------------------------------------- field views
// A parity-restricted field of 12 complex components per site: element
// (rhs r, component k, site i) at p[r * rs + k * n + i * ss].  Two layouts:
//   blocked      [rhs][12][sites]   rs = 12 sites (or more), n = sites, ss = 1
//   interleaved  [12][sites][rhs]   rs = 1, n = sites * nrhs, ss = nrhs
// (the interleaved one puts the right-hand sides of a site next to each other,
// so a wavefront of sites x rhs reads contiguous memory and a neighbour's
// spinors of all right-hand sides share cache lines).
template <class S>
struct FieldV {
  typename St<S>::E* p;
  float* scale;  // FP16 only: per-site scale at scale[r * srs + i * sss] (nullptr otherwise)
  int64_t rs;    // element stride between right-hand sides
  int64_t srs;   // scale stride between right-hand sides
  int n;         // component stride (elements)
  int ss = 1;    // site stride (elements)
  int sss = 1;   // site stride of the scales
};

// element at a 32-bit byte offset from a base pointer.  With a base that is the
// same for the whole wavefront (a field pointer plus a component offset) the
// load or store takes the scalar-base + 32-bit vector-offset form: one offset
// register serves all components and no 64-bit address arithmetic is needed.
// The base MUST be the same for every lane of the wavefront: it goes through
// readfirstlane, which keeps the compiler from folding the per-component
// offsets into 64-bit per-lane addresses.
__device__ inline uintptr_t uniform_addr(const void* a) {
  uintptr_t v = reinterpret_cast<uintptr_t>(a);
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uintptr_t)hi << 32) | lo;
}
// raw 4/8/16-byte words moved through global-address-space pointers
template <int B>
struct RawW;
template <>
struct RawW<4> { typedef unsigned int T; };
template <>
struct RawW<8> { typedef unsigned int T __attribute__((ext_vector_type(2))); };
template <>
struct RawW<16> { typedef unsigned int T __attribute__((ext_vector_type(4))); };

// NT: non-temporal (streaming) access, for data a pass touches only once, so
// that it does not push reused neighbour data out of the L2
template <class E, bool NT = false>
__device__ inline E ld_off(const E* base, uint32_t byte_off) {
  typedef typename RawW<sizeof(E)>::T R;
  typedef const __attribute__((address_space(1))) R* GP;
  GP a = reinterpret_cast<GP>(uniform_addr(base) + byte_off);
  R raw;
  if constexpr (NT) raw = __builtin_nontemporal_load(a);
  else raw = *a;
  E v;
  __builtin_memcpy(&v, &raw, sizeof(E));
  return v;
}
template <class E, bool NT = false>
__device__ inline void st_off(E* base, uint32_t byte_off, E v) {
  typedef typename RawW<sizeof(E)>::T R;
  typedef __attribute__((address_space(1))) R* GP;
  R raw;
  __builtin_memcpy(&raw, &v, sizeof(E));
  GP a = reinterpret_cast<GP>(uniform_addr(base) + byte_off);
  if constexpr (NT) __builtin_nontemporal_store(raw, a);
  else *a = raw;
}

// load / store of a 12-component spinor of site i, rhs r.  O32: the caller
// guarantees that the field view is the same for the whole wavefront and that
// every element offset of the field, (r * rs + i) elements, is below 2^32
// bytes, so the offsets are formed in 32 bits from scalar component bases.
template <class S, bool O32 = false>
__device__ inline void ld_spinor(const FieldV<S>& f, int r, int i, cx<typename St<S>::T> s[12]) {
  typedef typename St<S>::E E;
  if constexpr (O32) {
    const uint32_t vo = (uint32_t)(r * f.rs + (int64_t)i * f.ss) * (uint32_t)sizeof(E);
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = St<S>::from_reg(ld_off(f.p + (int64_t)k * f.n, vo));
  } else {
    const E* b = f.p + r * f.rs + (int64_t)i * f.ss;
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = St<S>::from_reg(b[(int64_t)k * f.n]);
  }
  if constexpr (sizeof(S) == 2) {
    float sc = f.scale[r * f.srs + (int64_t)i * f.sss];
#pragma unroll
    for (int k = 0; k < 12; ++k) { s[k].re *= sc; s[k].im *= sc; }
  }
}

// the stored components without the FP16 scale, and the scale (1 for FP32/FP64)
template <class S, bool O32 = false, bool NT = false>
__device__ inline typename St<S>::T ld_spinor_raw(const FieldV<S>& f, int r, int i, cx<typename St<S>::T> s[12]) {
  typedef typename St<S>::E E;
  if constexpr (O32) {
    const uint32_t vo = (uint32_t)(r * f.rs + (int64_t)i * f.ss) * (uint32_t)sizeof(E);
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = St<S>::from_reg(ld_off<E, NT>(f.p + (int64_t)k * f.n, vo));
    if constexpr (sizeof(S) == 2) return ld_off<float, NT>(f.scale, (uint32_t)(r * f.srs + (int64_t)i * f.sss) * 4u);
    else return typename St<S>::T(1);
  } else {
    const E* b = f.p + r * f.rs + (int64_t)i * f.ss;
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = St<S>::from_reg(b[(int64_t)k * f.n]);
    if constexpr (sizeof(S) == 2) return f.scale[r * f.srs + (int64_t)i * f.sss];
    else return typename St<S>::T(1);
  }
}

template <class S, bool O32 = false, bool NT = false>
__device__ inline void st_spinor(const FieldV<S>& f, int r, int i, const cx<typename St<S>::T> s[12]) {
  typedef typename St<S>::E E;
  auto put = [&](int k, cx<typename St<S>::T> v) {
    if constexpr (O32) st_off<E, NT>(f.p + (int64_t)k * f.n, (uint32_t)(r * f.rs + (int64_t)i * f.ss) * (uint32_t)sizeof(E), St<S>::to(v));
    else St<S>::st(f.p + r * f.rs + (int64_t)i * f.ss + (int64_t)k * f.n, v);
  };
  if constexpr (sizeof(S) == 2) {
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(s[k].re), fabsf(s[k].im)));
    float sc = m > 0.f ? m : 1.f;
    float inv = 1.f / sc;
    if constexpr (O32) st_off<float, NT>(f.scale, (uint32_t)(r * f.srs + (int64_t)i * f.sss) * 4u, sc);
    else f.scale[r * f.srs + (int64_t)i * f.sss] = sc;
#pragma unroll
    for (int k = 0; k < 12; ++k) put(k, cx<float>{s[k].re * inv, s[k].im * inv});
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) put(k, s[k]);
  }
}

// gauge field: U[p][mu][k][i], n = Vh
template <class S>
struct LinkV {
  const typename St<S>::E* p;
  int n;
};
template <class S>
__device__ inline void ld_link(const LinkV<S>& u, int par, int mu, int i, cx<typename St<S>::T> m[9]) {
  const typename St<S>::E* b = u.p + ((int64_t)(par * 4 + mu) * 9) * u.n + i;
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = St<S>::ldc(b + (int64_t)k * u.n);
}
// the same for a parity and direction that are uniform across the wavefront
// (scalar component bases, one 32-bit offset)
template <class S, bool NT = false>
__device__ inline void ld_link_u(const LinkV<S>& u, int par, int mu, int i, cx<typename St<S>::T> m[9]) {
  typedef typename St<S>::E E;
  const E* b = u.p + ((int64_t)(par * 4 + mu) * 9) * u.n;
  const uint32_t vo = (uint32_t)i * (uint32_t)sizeof(E);  // i < n: always within 32 bits
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = St<S>::from(ld_off<E, NT>(b + (int64_t)k * u.n, vo));
}

// the same, reading only the first two rows (components 0..5 of the
// component-major link arrays, 12 of the 18 reals) and rebuilding the third:
// for U in SU(3) it is the complex conjugate of the cross product of the first
// two; sgn is the fermion boundary sign folded into this stored link (the
// product of two signed rows loses it)
template <class T>
__device__ inline void link_row3(T sgn, cx<T> m[9]) {
  auto cross = [&](int a0, int a1, int b0, int b1) {
    // conj(m[a0] m[b1] - m[a1] m[b0]) * sgn
    const T re = m[a0].re * m[b1].re - m[a0].im * m[b1].im - (m[a1].re * m[b0].re - m[a1].im * m[b0].im);
    const T im = m[a0].re * m[b1].im + m[a0].im * m[b1].re - (m[a1].re * m[b0].im + m[a1].im * m[b0].re);
    return cx<T>{sgn * re, -sgn * im};
  };
  m[6] = cross(1, 2, 4, 5);  // conj(m1 m5 - m2 m4)
  m[7] = cross(2, 0, 5, 3);  // conj(m2 m3 - m0 m5)
  m[8] = cross(0, 1, 3, 4);  // conj(m0 m4 - m1 m3)
}

template <class S, bool NT = false>
__device__ inline void ld_link_u12(const LinkV<S>& u, int par, int mu, int i, typename St<S>::T sgn,
                                   cx<typename St<S>::T> m[9]) {
  typedef typename St<S>::E E;
  typedef typename St<S>::T T;
  const E* b = u.p + ((int64_t)(par * 4 + mu) * 9) * u.n;
  const uint32_t vo = (uint32_t)i * (uint32_t)sizeof(E);
#pragma unroll
  for (int k = 0; k < 6; ++k) m[k] = St<S>::from(ld_off<E, NT>(b + (int64_t)k * u.n, vo));
  link_row3<T>(sgn, m);
}

// clover: A[p][slot][i], 36 slots (2 blocks x 18)
template <class S>
struct CloverV {
  const typename St<S>::E* p;
  int n;
};

// y = A x for one Hermitian 6x6 block stored in 18 slots
template <class T>
__device__ inline void herm6_mul(const cx<T> a[18], const cx<T> x[6], cx<T> y[6]) {
  // diagonal
  T d[6] = {a[0].re, a[0].im, a[1].re, a[1].im, a[2].re, a[2].im};
#pragma unroll
  for (int r = 0; r < 6; ++r) y[r] = d[r] * x[r];
  int s = 3;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r + 1; c < 6; ++c) {
      cx<T> v = a[s++];
      y[r] = fma_c(v, x[c], y[r]);
      y[c] = fmac_c(v, x[r], y[c]);
    }
}

template <class S>
__device__ inline void clover_apply(const CloverV<S>& A, int par, int i, const cx<typename St<S>::T> in[12],
                                    cx<typename St<S>::T> out[12]) {
  typedef typename St<S>::T T;
  const typename St<S>::E* b = A.p + (int64_t)par * 36 * A.n + i;
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    cx<T> a[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) a[k] = St<S>::ldc(b + (int64_t)(blk * 18 + k) * A.n);
    herm6_mul<T>(a, in + 6 * blk, out + 6 * blk);
  }
}
// the same for a parity that is uniform across the wavefront
template <class S, bool NT = false>
__device__ inline void clover_apply_u(const CloverV<S>& A, int par, int i, const cx<typename St<S>::T> in[12],
                                      cx<typename St<S>::T> out[12]) {
  typedef typename St<S>::T T;
  typedef typename St<S>::E E;
  const E* b = A.p + (int64_t)par * 36 * A.n;
  const uint32_t vo = (uint32_t)i * (uint32_t)sizeof(E);
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    cx<T> a[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) a[k] = St<S>::from(ld_off<E, NT>(b + (int64_t)(blk * 18 + k) * A.n, vo));
    herm6_mul<T>(a, in + 6 * blk, out + 6 * blk);
  }
}

// --------------------------------------------------------------- spin projection
// (1 - sg*gamma_mu) psi = [h ; M h] with h = psi_up + P psi_lo (2 spins x 3 colours);
// sg = +1 is the forward hop (1 - gamma), sg = -1 the backward hop (1 + gamma).
// Chiral basis: g0 = [[0,-1],[-1,0]], gk = [[0,-i sk],[i sk,0]].
template <class T, int MU, int SG>
__device__ inline void project(const cx<T> s[12], cx<T> h[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<T> u0 = s[c], u1 = s[3 + c], l0 = s[6 + c], l1 = s[9 + c];
    if constexpr (MU == 0) {
      // P = +1 (forward), -1 (backward)
      h[c] = SG > 0 ? u0 + l0 : u0 - l0;
      h[3 + c] = SG > 0 ? u1 + l1 : u1 - l1;
    } else if constexpr (MU == 1) {
      // i s1 v = (i v1, i v0); P = +i s1 (fwd), -i s1 (bwd)
      h[c] = SG > 0 ? u0 + ti(l1) : u0 - ti(l1);
      h[3 + c] = SG > 0 ? u1 + ti(l0) : u1 - ti(l0);
    } else if constexpr (MU == 2) {
      // i s2 v = (v1, -v0)
      h[c] = SG > 0 ? u0 + l1 : u0 - l1;
      h[3 + c] = SG > 0 ? u1 - l0 : u1 + l0;
    } else {
      // i s3 v = (i v0, -i v1)
      h[c] = SG > 0 ? u0 + ti(l0) : u0 - ti(l0);
      h[3 + c] = SG > 0 ? u1 - ti(l1) : u1 + ti(l1);
    }
  }
}

// acc += c [g ; M g]: M = +P for mu = 0 and M = -P for mu = 1,2,3.  The factor c
// (the -1/4 of Dhat, an FP16 scale) rides on the accumulating fused
// multiply-adds; c = 1 gives plain additions.
template <class T>
__device__ inline cx<T> cacc(cx<T> a, T c, cx<T> b) { return {fmar(c, b.re, a.re), fmar(c, b.im, a.im)}; }
template <class T, int MU, int SG>
__device__ inline void reconstruct_add(const cx<T> g[6], cx<T> acc[12], T c = T(1)) {
  const T m = -c;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    cx<T> g0 = g[k], g1 = g[3 + k];
    acc[k] = cacc(acc[k], c, g0);
    acc[3 + k] = cacc(acc[3 + k], c, g1);
    if constexpr (MU == 0) {
      // M = +1 (fwd), -1 (bwd)
      acc[6 + k] = cacc(acc[6 + k], SG > 0 ? c : m, g0);
      acc[9 + k] = cacc(acc[9 + k], SG > 0 ? c : m, g1);
    } else if constexpr (MU == 1) {
      // M = -i s1 (fwd): (-i g1, -i g0); +i s1 (bwd)
      acc[6 + k] = cacc(acc[6 + k], SG > 0 ? m : c, ti(g1));
      acc[9 + k] = cacc(acc[9 + k], SG > 0 ? m : c, ti(g0));
    } else if constexpr (MU == 2) {
      // M = -i s2 (fwd): -(g1, -g0) = (-g1, g0)
      acc[6 + k] = cacc(acc[6 + k], SG > 0 ? m : c, g1);
      acc[9 + k] = cacc(acc[9 + k], SG > 0 ? c : m, g0);
    } else {
      // M = -i s3 (fwd): (-i g0, +i g1)
      acc[6 + k] = cacc(acc[6 + k], SG > 0 ? m : c, ti(g0));
      acc[9 + k] = cacc(acc[9 + k], SG > 0 ? c : m, ti(g1));
    }
  }
}

// g = U h (forward) or U^dag h (backward), per spin row of the half spinor
template <class T, bool DAG>
__device__ inline void su3_mul_half(const cx<T> u[9], const cx<T> h[6], cx<T> g[6]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<T> acc{T(0), T(0)};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (DAG) acc = fmac_c(u[b * 3 + a], h[3 * s + b], acc);
        else acc = fma_c(u[a * 3 + b], h[3 * s + b], acc);
      }
      g[3 * s + a] = acc;
    }
}

}  // namespace qdd
