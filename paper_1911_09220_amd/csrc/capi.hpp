// Helpers shared by the C entry points: status capture, argument checks, and
// the operator apply used by every solver.
#pragma once

#include <hip/hip_runtime_api.h>

#include <new>
#include <string>

#include "internal.hpp"

namespace pafem {

extern thread_local std::string g_last_error;

inline pafem_status fail(pafem_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

inline void hip_check(hipError_t err, const char* what) {
  if (err != hipSuccess) throw Error(PAFEM_EHIP, std::string(what) + ": " + hipGetErrorString(err));
}

inline void require(bool cond, pafem_status code, const std::string& msg) {
  if (!cond) throw Error(code, msg);
}

template <typename F>
pafem_status guarded(F&& f) {
  try {
    f();
    return PAFEM_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "out of host memory";
    return PAFEM_EINVAL;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return PAFEM_EINVAL;
  }
}

// Workspace bytes of one operator application (element vector of the
// deterministic scatter; also the diagonal's element vector).
size_t op_work_bytes(const Op& op);
// y = A x on the op's stream; `work` holds op_work_bytes(op).
// y_ready: y already holds the apply init (x on essential dofs when constrained, else 0)
void apply_op(const Op& op, const void* x, void* y, void* work, hipStream_t st,
              double* dotp = nullptr, bool y_ready = false);

}  // namespace pafem

// Opaque handle types of the C ABI.
struct pafem_mesh_s {
  pafem::Mesh m;
};
struct pafem_space_s {
  pafem::Space* s;
};
struct pafem_op_s {
  pafem::Op op;
};
