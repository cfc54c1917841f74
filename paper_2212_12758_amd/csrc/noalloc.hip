// Allocation-free entry point: fab_solve on a static device scratch array.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation), the
// per-request workspace of a blocking solve -- basis, partial sums, sketch
// partials, dense tail, status words -- and the sampled SRHT rows live in
// `scratch`, a file-scope device array of FAB_NOALLOC_SCRATCH_BYTES that every
// GPU the library runs on holds until the process ends.  Host code never uses
// the array's name as an address: fab_init calls noalloc_setup for its device,
// which looks the array up with hipGetSymbolAddress (with that device
// current) and keeps the device address per device; kernels receive that
// address as their workspace argument like any arena block.
//
// The array is shared by every call on one GPU and keeps the last call's
// contents; the solve clears every region it reads before writing it (as it
// does for reused arena blocks).  Calls on one GPU are serialised by a per-
// device mutex here, and each call returns only after its stream has
// finished, so two calls never use the array at the same time.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fab.h"

static __device__ __align__(256) char scratch[FAB_NOALLOC_SCRATCH_BYTES];

namespace fab {
int solve_fixed_workspace(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f, const fab_params* p,
                          double* out, fab_info* info, char* ws, size_t bytes);
int ctx_device(fab_ctx ctx);

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_setup_mu;
void* g_scratch[kMaxDevices] = {};
std::mutex g_call_mu[kMaxDevices];
}  // namespace

// Once per device, with that device current: the device address of `scratch`.
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return FAB_EINVAL;
  std::lock_guard<std::mutex> lk(g_setup_mu);
  if (g_scratch[device]) return FAB_OK;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return FAB_EDEVICE;
  if (cur != device && hipSetDevice(device) != hipSuccess) return FAB_EDEVICE;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return FAB_EDEVICE;
  }
  g_scratch[device] = ptr;
  return FAB_OK;
}
}  // namespace fab

extern "C" int fab_solve_noalloc(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f,
                                 const fab_params* p, double* out, fab_info* info) {
  const int dev = fab::ctx_device(ctx);
  if (dev < 0 || dev >= fab::kMaxDevices) return FAB_EINVAL;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(fab::g_setup_mu);
    ws = fab::g_scratch[dev];
  }
  if (!ws) return FAB_EDEVICE;   // fab_init sets it up for the context's device
  std::lock_guard<std::mutex> lk(fab::g_call_mu[dev]);
  return fab::solve_fixed_workspace(ctx, A, b, nrhs, f, p, out, info, (char*)ws, FAB_NOALLOC_SCRATCH_BYTES);
}
