// Device-resident scratch of the allocation-free preconditioner entry point
// (hdp_apply_precond_noalloc): one fixed array per GPU, held until the process
// ends, whose address is looked up once per device at set-up.
//
// The array's name is a host-side stand-in in host code; kernels receive the
// device address returned by hipGetSymbolAddress, never the name itself.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "internal.hpp"

namespace hdp {

namespace {
constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per device
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;   // per device ordinal, null until resolved
}  // namespace

const size_t SCRATCH_BYTES = kScratchBytes;

void scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) fail(HDP_E_DEVICE, "invalid device ordinal");
  if (size_t(device) >= g_scratch_addr.size()) g_scratch_addr.resize(size_t(device) + 1, nullptr);
  if (g_scratch_addr[size_t(device)]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    fail(HDP_E_DEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
  }
  g_scratch_addr[size_t(device)] = p;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || size_t(device) >= g_scratch_addr.size()) return nullptr;
  return g_scratch_addr[size_t(device)];
}

}  // namespace hdp
