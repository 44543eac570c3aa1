// The fixed device buffer of mp_cgemm_ex_noalloc: a file-scope array in the
// library's code object, one copy per device, held until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in for the device symbol): the device address of each
// device's copy is looked up once, with that device current, and used
// instead.
#include <mutex>

#include "../../include/mpcgemm.h"
#include "mpcg_internal.h"

namespace mpcg {
namespace {

static __device__ __align__(256) unsigned char scratch[MPCG_NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

hipError_t noalloc_scratch(hipStream_t stream, void** ptr, size_t* bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    // the status word (first 256 bytes) starts at zero; a kernel, so that a
    // first call under graph capture records no memset node
    e = launch_fill_zero(p, 256, stream);
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  *bytes = MPCG_NOALLOC_BYTES;
  return hipSuccess;
}

int* noalloc_status_word() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return static_cast<int*>(g_scratch_ptr[dev]);
}

}  // namespace mpcg
