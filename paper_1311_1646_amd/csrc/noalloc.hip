// Statically allocated device scratch of dmrg_sigma_noalloc, for callers that
// cannot allocate device memory.
//
// The array lives in the code object: every GPU the library runs on holds its
// own copy for the life of the process, at its own address.  In host code the
// array's name only stands in for it, so the address is looked up once per
// device (with that device current) and only that address is passed to
// kernels.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "common.hpp"

namespace dmrg {

namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t scratch_bytes() { return kScratchBytes; }

void* scratch_address(int device) {
  DMRG_REQUIRE(device >= 0 && device < kMaxDevices, DMRG_ERR_INVALID_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    DMRG_REQUIRE(e == hipSuccess && p, DMRG_ERR_HIP,
                 std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace dmrg
