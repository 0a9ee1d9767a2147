// The library's static device scratch and the one entry point that uses it
// (kv_project_mixed_static): the mixed-form projection for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The scratch is a file-scope __device__ array, so every GPU the library
// runs on holds its own copy until the process ends.  In host code the
// array's name only stands for it: its device address on each GPU comes
// from hipGetSymbolAddress, taken once per device (with that device
// current) when the first context is created there, and only that address
// is ever passed to kernels or copies.
#include <mutex>

#include "kv_internal.h"

namespace kv {
namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};  // device address of scratch on each GPU (null: not set up)

}  // namespace

int static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return 1;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return 0;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return 1;
  g_ptr[device] = static_cast<double*>(p);
  return 0;
}

}  // namespace kv

extern "C" int kv_project_mixed_static(kv_ctx* c, double* y, double* div_max, int* sweeps) {
  using namespace kv;
  if (!c) return KV_EINVAL;
  if (!y) {
    c->err = "null vector";
    return KV_EINVAL;
  }
  if (!mixed_grid(c)) {
    c->err = "kv_project_mixed_static: the mixed projection needs every axis mirror-symmetric with an even cell count";
    return KV_EINVAL;
  }
  const size_t need = mixed_scratch_bytes(c);
  if (need > kStaticScratchBytes) {
    char msg[200];
    snprintf(msg, sizeof msg,
             "kv_project_mixed_static: the grid needs %zu bytes of scratch, above the static %zu (use kv_project "
             "with a workspace)",
             need, kStaticScratchBytes);
    c->err = msg;
    return KV_EINVAL;
  }
  double* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (c->device >= 0 && c->device < kMaxDevices) ptr = g_ptr[c->device];
  }
  if (!ptr) {
    c->err = "kv_project_mixed_static: static scratch not set up on this device";
    return KV_EDEVICE;
  }
  // no phase timing here: its events would be created on demand
  const bool timing = c->timing;
  c->timing = false;
  const int rc = project_mixed_with(c, y, div_max, sweeps, ptr);
  c->timing = timing;
  return rc;
}
