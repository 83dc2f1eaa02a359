// Host batch object behind pafem_batch_* (batch.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "batch.hpp"
#include "internal.hpp"

namespace pafem {

class Batch {
 public:
  Batch(const std::vector<const Op*>& ops, int nrhs, void* work, size_t work_bytes);
  ~Batch();
  Batch(const Batch&) = delete;
  Batch& operator=(const Batch&) = delete;

  static size_t workspace_bytes(int nops);
  // Y_m = A_m X_m for every mesh: one graph launch (captured on first use and
  // again whenever the vector pointers or tile choices change).
  void apply(const void* const* x, void* const* y, hipStream_t st);
  // Time every tile candidate of every order; cache winners by (arch, kind,
  // dtype, nrhs, order).  Synchronous.
  void autotune(const void* const* x, void* const* y, const char* cache_path, int reps,
                hipStream_t st);
  void set_candidate(int p, int cand);
  std::string describe() const;

 private:
  struct Group {
    int p = 0, first = 0, count = 0, cand = 0;
  };
  struct Timing {
    int p, cand;
    float ms;
  };
  void build_descriptors(const void* const* x, void* const* y);
  void upload(hipStream_t st);
  int group_blocks(const Group& g) const;
  void launch_group(const Group& g, hipStream_t st) const;
  void launch_all(hipStream_t st) const;
  void prepare(const void* const* x, void* const* y, hipStream_t st);

  std::vector<const Op*> ops;
  std::vector<int> order;  // position in the order-sorted list -> index in ops
  std::vector<Group> groups;
  std::vector<BatchMesh> host;
  std::vector<Timing> timings;
  BatchMesh* d_meshes = nullptr;
  int nrhs = 0, kind = 0, qdtype = 0, vdtype = 0;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> cur_x;
  std::vector<void*> cur_y;
  bool dirty = true;
};

}  // namespace pafem
