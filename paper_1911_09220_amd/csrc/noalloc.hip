// Operator apply for callers that cannot allocate device memory: the scratch
// memory of the deterministic scatter (one element vector per element) lives in a
// file-scope device array instead of a caller workspace.  Each GPU the library runs
// on holds its own copy of the array, at its own address, until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "capi.hpp"
#include "internal.hpp"

// The array's name is a host-side stand-in in host code: host code only ever uses
// the per-device address returned by hipGetSymbolAddress.
static __device__ __align__(256) char scratch[PAFEM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of the array, looked up once per device with
// that device current (it is current here: the caller's stream belongs to it).
void* scratch_for_current_device() {
  int dev = -1;
  pafem::hip_check(hipGetDevice(&dev), "hipGetDevice");
  pafem::require(dev >= 0 && dev < kMaxDevices, PAFEM_EUNSUPPORTED,
                 "device index " + std::to_string(dev) + " beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    pafem::hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)),
                     "hipGetSymbolAddress(scratch)");
    pafem::require(ptr != nullptr, PAFEM_EHIP, "hipGetSymbolAddress returned null");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" pafem_status pafem_op_apply_noalloc(pafem_op op, const double* x, double* y,
                                               void* stream) {
  using namespace pafem;
  return guarded([&] {
    require(op && x && y, PAFEM_EINVAL, "null pointer argument");
    require(x != y, PAFEM_EINVAL, "x and y must not alias");
    void* work = nullptr;
    if (op->op.flags & PAFEM_OP_SCATTER_EVEC) {
      const size_t need = op_work_bytes(op->op);
      require(need <= size_t(PAFEM_NOALLOC_SCRATCH_BYTES), PAFEM_ESHAPE,
              "element vectors need " + std::to_string(need) + " bytes, more than the " +
                  std::to_string(size_t(PAFEM_NOALLOC_SCRATCH_BYTES)) +
                  " bytes of scratch of pafem_op_apply_noalloc");
      work = scratch_for_current_device();
    }
    // every element-vector entry is written by the apply before the gather reads it,
    // so the scratch needs no clearing between calls
    apply_op(op->op, x, y, work, static_cast<hipStream_t>(stream));
  });
}
