// Replay of fixed launch sequences from HIP graphs.  A solver iteration is a fixed
// sequence of kernel launches whose arguments do not change between iterations, so it
// is captured once (on a private stream, nothing runs during capture) and replayed on
// the caller's stream: one launch per replay instead of one per kernel.  Only kernels
// are captured (no memset or copy nodes).
#pragma once

#include <hip/hip_runtime_api.h>

#include <atomic>

#include "capi.hpp"

namespace pafem {

// Process-wide switch (pafem_set_graph_mode): 1 = replay solver iterations from
// graphs (default), 0 = launch every kernel directly.
std::atomic<int>& graph_mode_flag();
inline bool graphs_enabled() { return graph_mode_flag().load(std::memory_order_relaxed) != 0; }

class CapturedGraph {
 public:
  CapturedGraph() = default;
  CapturedGraph(const CapturedGraph&) = delete;
  CapturedGraph& operator=(const CapturedGraph&) = delete;
  ~CapturedGraph() { reset(); }

  bool ready() const { return exec_ != nullptr; }

  // Records body(stream) into the graph; body must only launch kernels.
  template <typename F>
  void capture(F&& body) {
    reset();
    hip_check(hipStreamCreateWithFlags(&cs_, hipStreamNonBlocking), "capture stream");
    hip_check(hipStreamBeginCapture(cs_, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      body(cs_);
    } catch (...) {
      hipGraph_t g = nullptr;
      hipStreamEndCapture(cs_, &g);
      if (g) hipGraphDestroy(g);
      throw;
    }
    hip_check(hipStreamEndCapture(cs_, &graph_), "end capture");
    hip_check(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0), "graph instantiate");
  }

  void launch(hipStream_t st) { hip_check(hipGraphLaunch(exec_, st), "graph launch"); }

  void reset() {
    if (exec_) hipGraphExecDestroy(exec_);
    if (graph_) hipGraphDestroy(graph_);
    if (cs_) hipStreamDestroy(cs_);
    exec_ = nullptr;
    graph_ = nullptr;
    cs_ = nullptr;
  }

 private:
  hipStream_t cs_ = nullptr;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
};

}  // namespace pafem
