// Dhat apply for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc): the
// odd-site intermediate t_o = A_o^{-1} H_oe psi_e of the two-pass Schur
// complement (Eq. 2) lives in a file-scope device array instead of the
// context's workspace.  The kernels are those of qdd_dw_hat.
//
// The array is one per GPU, held from the first use on that GPU until the
// process ends.  In host code its name is only a stand-in: the per-device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and only that address is handed to kernels.
#include "qdd_api_internal.h"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of `scratch` on `dev` (the current device); nullptr on error
void* scratch_on(int dev, hipError_t* err) {
  *err = hipSuccess;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" qdd_status qdd_dw_hat_static(qdd_ctx* x, qdd_prec prec, int nrhs, const void* in, void* out) {
  if (!x || !in || !out || nrhs < 1 || nrhs > x->cfg.max_nrhs || prec < QDD_F64 || prec > QDD_F16) {
    if (x) x->fail("qdd_dw_hat_static: invalid arguments");
    return QDD_EINVAL;
  }
  if (!x->have_clover) { x->fail("qdd_dw_hat_static before qdd_set_params"); return QDD_ESTATE; }
  const size_t need = x->dhat_tmp_bytes(prec, nrhs);
  if (need > kScratchBytes) {
    x->fail("qdd_dw_hat_static: the odd-site intermediate needs %zu bytes, above the %zu-byte static scratch",
            need, kScratchBytes);
    return QDD_EINVAL;
  }
  int dev = -1;
  HCK(x, hipGetDevice(&dev));
  if (dev != x->device) {
    x->fail("qdd_dw_hat_static: device %d is current, the context lives on device %d", dev, x->device);
    return QDD_EINVAL;
  }
  hipError_t e = hipSuccess;
  void* p = scratch_on(dev, &e);
  HCK(x, e);
  // pass A writes every element of t_o (and of its scales) before pass B reads
  // it, so the array needs no clearing between calls
  HCK(x, x->dhat(prec, nrhs, (void*)in, out, nullptr, p));
  return QDD_OK;
}
