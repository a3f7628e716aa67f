// Launchers of the network kernels (qdd_net.hip).
#pragma once
#include "qdd_kernels.h"

namespace qdd {
// one layer: out (cout channels, at most 16) = sum W (T_d in) ; channel stride cs
// (elements); wmx: the layer's weights arranged by launch_net_wmx with the same
// scratch_ch.  scratch: scratch_ch channel fields the weights-first form of a
// one-output-channel layer may use (it needs 9; with fewer it is not used).
// terms: BF16 terms per transported input, 3 (exact split, FP32 accuracy), 2 or 1
hipError_t launch_net_layer(const Geo& g, const LinkV<float>& U, const uint16_t* wmx, int cin, int cout,
                            const float2* in, float2* out, int64_t cs, float2* scratch, int scratch_ch, int terms,
                            hipStream_t st);
bool net_weights_first(int cin, int cout, int scratch_ch);
// BF16 matrix-core operands of a layer from its BF16 complex weights wb
// (net_wmx_elems 16-bit elements)
size_t net_wmx_elems(int cin, int cout, int scratch_ch);
hipError_t launch_net_wmx(const uint32_t* wb, int cin, int cout, int scratch_ch, uint16_t* wmx, hipStream_t st);
// grad += dloss/dW of one layer from its input `in` and output gradient `gy`;
// part: partial-product scratch of part_floats floats, at least
// net_wgrad_part_floats(V, cin, cout)
size_t net_wgrad_part_floats(int64_t V, int cin, int cout);
hipError_t launch_net_wgrad(const Geo& g, const LinkV<float>& U, int cin, int cout, const float2* in,
                            const float2* gy, int64_t cs, float* part, size_t part_floats, float2* grad,
                            hipStream_t st);
hipError_t launch_net_to_bf16(const float2* w, uint32_t* wb, int n, hipStream_t st);
hipError_t launch_net_adjoint(const uint32_t* wb, int cin, int cout, uint32_t* wa, hipStream_t st);
hipError_t launch_net_out_grad(const float2* y, const float2* e, float escale, float invZ, float2* gy, int64_t n,
                               double* part, int nb, hipStream_t st);
hipError_t launch_net_adam(float2* w, const float2* g, float4* mv, int n, float lr, int step, hipStream_t st);
hipError_t launch_norm2_f(const float2* x, int64_t n, double* part, int nb, hipStream_t st);
template <class E>
hipError_t launch_scale_to_f(float2* y, const E* x, double a, int64_t n, hipStream_t st);
hipError_t launch_err_from(float2* e, const double2* psi, int64_t n, hipStream_t st);
hipError_t launch_sub_f(double2* a, const float2* b, int64_t n, hipStream_t st);
}  // namespace qdd
