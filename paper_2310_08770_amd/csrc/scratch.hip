// The library's static device scratch: working memory for
// ccpt_track_batch_static, which callers use where they cannot allocate
// device memory (graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Each GPU the library runs on holds its own copy of the array
// from module load until the process ends.
//
// Host code never names the array itself (in host code its name is a
// host-side stand-in, not a device address): the device address is taken
// once per device with hipGetSymbolAddress, with that device current, and
// kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace ccpt {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return 0;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) return -1;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
  g_ptr[device] = p;
  return 0;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

}  // namespace ccpt
