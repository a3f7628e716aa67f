// Gauge ingest and field (un)packing: canonical complex128 arrays at the
// library boundary <-> the parity-split structure-of-arrays device layout.
#include "qdd_kernels.h"

namespace qdd {

// one thread per (site, direction); the fermion time-boundary sign is folded
// into the hopping copy of the links on the last time slice
__global__ void k_pack_links(Geo g, const double* canon, double2* U) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)g.V * 4) return;
  int lex = (int)(t >> 2), mu = (int)(t & 3);
  int x3 = lex % g.L[3], r = lex / g.L[3];
  int x2 = r % g.L[2];
  r /= g.L[2];
  int x1 = r % g.L[1], x0 = r / g.L[1];
  int p = (x0 + x1 + x2 + x3) & 1, i = lex >> 1;
  double s = (mu == 0 && x0 == g.L[0] - 1) ? (double)g.bc : 1.0;
  const double* src = canon + t * 18;
  double2* dst = U + (int64_t)(p * 4 + mu) * 9 * g.Vh + i;
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[(int64_t)k * g.Vh] = make_double2(s * src[2 * k], s * src[2 * k + 1]);
}

// plain 16-byte-vector copy: the HBM bandwidth reference of the benchmarks
__global__ void k_copy(uint4* dst, const uint4* src, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = src[t];
}
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  int64_t n = (int64_t)(bytes / 16);
  int nb = (int)std::min<int64_t>((n + 255) / 256, 256 * 64);
  if (n > 0) hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, st, (uint4*)dst, (const uint4*)src, n);
  return hipGetLastError();
}

hipError_t launch_pack_links(const Geo& g, const double* canon, double2* U, hipStream_t st) {
  int64_t n = (int64_t)g.V * 4;
  hipLaunchKernelGGL(k_pack_links, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, canon, U);
  return hipGetLastError();
}

__global__ void k_convert_f(const double2* in, float2* out, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = make_float2((float)in[t].x, (float)in[t].y);
}
__global__ void k_convert_h(const double2* in, __half2* out, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = __floats2half2_rn((float)in[t].x, (float)in[t].y);
}
hipError_t launch_convert(const double2* in, float2* out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_convert_f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}
hipError_t launch_convert(const double2* in, __half2* out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_convert_h, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

// thread per (rhs, canonical site); full fields: canonical [r][lex][12];
// even-only: canonical [r][i][12] with i = lex >> 1 of the even sites
template <class S>
__global__ void k_pack_spinor(Geo g, const double* canon, FieldV<S> f, int nrhs, int even_only, int64_t poff,
                              int64_t spoff) {
  typedef typename St<S>::T T;
  int nsite = even_only ? g.Vh : g.V;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nsite * nrhs) return;
  int r = (int)(t / nsite), s = (int)(t % nsite);
  int p = 0, i = s;
  if (!even_only) {
    int x3 = s % g.L[3], q = s / g.L[3];
    int x2 = q % g.L[2];
    q /= g.L[2];
    p = (x3 + x2 + (q % g.L[1]) + q / g.L[1]) & 1;
    i = s >> 1;
  }
  const double* src = canon + t * 24;
  cx<T> v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = {(T)src[2 * k], (T)src[2 * k + 1]};
  FieldV<S> d = f;
  d.p += p * poff;
  if (d.scale) d.scale += p * spoff;
  st_spinor(d, r, i, v);
}

template <class S>
__global__ void k_unpack_spinor(Geo g, FieldV<S> f, double* canon, int nrhs, int even_only, int64_t poff,
                                int64_t spoff) {
  typedef typename St<S>::T T;
  int nsite = even_only ? g.Vh : g.V;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nsite * nrhs) return;
  int r = (int)(t / nsite), s = (int)(t % nsite);
  int p = 0, i = s;
  if (!even_only) {
    int x3 = s % g.L[3], q = s / g.L[3];
    int x2 = q % g.L[2];
    q /= g.L[2];
    p = (x3 + x2 + (q % g.L[1]) + q / g.L[1]) & 1;
    i = s >> 1;
  }
  FieldV<S> d = f;
  d.p += p * poff;
  if (d.scale) d.scale += p * spoff;
  cx<T> v[12];
  ld_spinor(d, r, i, v);
  double* dst = canon + t * 24;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    dst[2 * k] = (double)v[k].re;
    dst[2 * k + 1] = (double)v[k].im;
  }
}

template <class S>
hipError_t launch_pack_spinor(const Geo& g, const double* canon, FieldV<S> f, int nrhs, int even_only, int64_t poff,
                              int64_t spoff, hipStream_t st) {
  int64_t n = (int64_t)(even_only ? g.Vh : g.V) * nrhs;
  hipLaunchKernelGGL((k_pack_spinor<S>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, canon, f, nrhs,
                     even_only, poff, spoff);
  return hipGetLastError();
}
template <class S>
hipError_t launch_unpack_spinor(const Geo& g, FieldV<S> f, double* canon, int nrhs, int even_only, int64_t poff,
                                int64_t spoff, hipStream_t st) {
  int64_t n = (int64_t)(even_only ? g.Vh : g.V) * nrhs;
  hipLaunchKernelGGL((k_unpack_spinor<S>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, f, canon, nrhs,
                     even_only, poff, spoff);
  return hipGetLastError();
}

// precision conversion of nvec vectors of n sites (layout [vec][12][n] with the
// views' rhs strides)
template <class SI, class SO>
__device__ __forceinline__ void field_convert_body(const FieldV<SI>& in, const FieldV<SO>& out, int nvec, int bid) {
  int64_t t = (int64_t)bid * blockDim.x + threadIdx.x;
  if (t >= (int64_t)in.n * nvec) return;
  int v = (int)(t / in.n), i = (int)(t % in.n);
  cx<typename St<SI>::T> a[12];
  ld_spinor(in, v, i, a);
  cx<typename St<SO>::T> b[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = {(typename St<SO>::T)a[k].re, (typename St<SO>::T)a[k].im};
  st_spinor(out, v, i, b);
}
template <class SI, class SO>
__global__ void k_field_convert(FieldV<SI> in, FieldV<SO> out, int nvec) {
  field_convert_body<SI, SO>(in, out, nvec, blockIdx.x);
}
template <class SI, class SO>
struct ConvArgs {
  FieldV<SI> in;
  FieldV<SO> out;
  int nvec;
};
template <class SI, class SO>
__global__ void k_field_convert_grp(Grp<ConvArgs<SI, SO>> G) {
  const int s = grp_sys(G.start, G.ns, blockIdx.x);
  const ConvArgs<SI, SO>& a = G.a[s];
  field_convert_body<SI, SO>(a.in, a.out, a.nvec, blockIdx.x - G.start[s]);
}
template <class SI, class SO>
hipError_t launch_field_convert_grp(const FieldV<SI>* in, const FieldV<SO>* out, const int* nvec, int ns,
                                    hipStream_t st) {
  if (ns < 1 || ns > kGrpMax) return hipErrorInvalidValue;
  Grp<ConvArgs<SI, SO>> G = grp_new<ConvArgs<SI, SO>>();
  for (int s = 0; s < ns; ++s)
    grp_add(G, ConvArgs<SI, SO>{in[s], out[s], nvec[s]}, (int)(((int64_t)in[s].n * nvec[s] + 255) / 256));
  hipLaunchKernelGGL((k_field_convert_grp<SI, SO>), dim3(G.start[ns]), dim3(256), 0, st, G);
  return hipGetLastError();
}
template hipError_t launch_field_convert_grp<double, float>(const FieldV<double>*, const FieldV<float>*, const int*,
                                                            int, hipStream_t);
template hipError_t launch_field_convert_grp<float, double>(const FieldV<float>*, const FieldV<double>*, const int*,
                                                            int, hipStream_t);
template hipError_t launch_field_convert_grp<double, __half>(const FieldV<double>*, const FieldV<__half>*,
                                                             const int*, int, hipStream_t);

template <class SI, class SO>
hipError_t launch_field_convert(FieldV<SI> in, FieldV<SO> out, int nvec, hipStream_t st) {
  int64_t n = (int64_t)in.n * nvec;
  hipLaunchKernelGGL((k_field_convert<SI, SO>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, nvec);
  return hipGetLastError();
}

#define INST(S)                                                                                               \
  template hipError_t launch_pack_spinor<S>(const Geo&, const double*, FieldV<S>, int, int, int64_t, int64_t, \
                                            hipStream_t);                                                     \
  template hipError_t launch_unpack_spinor<S>(const Geo&, FieldV<S>, double*, int, int, int64_t, int64_t, hipStream_t);
INST(double)
INST(float)
INST(__half)
#undef INST
template hipError_t launch_field_convert<double, float>(FieldV<double>, FieldV<float>, int, hipStream_t);
template hipError_t launch_field_convert<double, __half>(FieldV<double>, FieldV<__half>, int, hipStream_t);
template hipError_t launch_field_convert<float, double>(FieldV<float>, FieldV<double>, int, hipStream_t);
template hipError_t launch_field_convert<__half, double>(FieldV<__half>, FieldV<double>, int, hipStream_t);
template hipError_t launch_field_convert<float, float>(FieldV<float>, FieldV<float>, int, hipStream_t);
template hipError_t launch_field_convert<double, double>(FieldV<double>, FieldV<double>, int, hipStream_t);
template hipError_t launch_field_convert<__half, __half>(FieldV<__half>, FieldV<__half>, int, hipStream_t);
template hipError_t launch_field_convert<float, __half>(FieldV<float>, FieldV<__half>, int, hipStream_t);
template hipError_t launch_field_convert<__half, float>(FieldV<__half>, FieldV<float>, int, hipStream_t);

}  // namespace qdd
