// Host side of the batched apply: groups meshes by order, keeps the device
// descriptors, captures the whole batch (init + one grouped launch per order)
// into a HIP graph, and tunes the tile shape of every order by timing the
// candidates (results cached in a small text file).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <tuple>

#include "batch.hpp"
#include "batch_host.hpp"

namespace pafem {

namespace {

void hipc(hipError_t err, const char* what) {
  if (err != hipSuccess) throw Error(PAFEM_EHIP, std::string(what) + ": " + hipGetErrorString(err));
}

// largest right-hand-side chunk first: the default before tuning
bool candidate_ok(int p, int cand, int nrhs, int vdtype) {
  if (cand < 0 || cand >= kBatchCandidates) return false;
  if (nrhs % batch_tile_rhs(cand)) return false;
  if (cand == kBatchMfmaCandidate) return vdtype == PAFEM_F64 && p <= 4;
  // tiles built per order (k_batch.hip): larger ones would exceed the registers
  if (cand == 1 && p > 5) return false;
  if (cand == 2 && p > 3) return false;
  if (cand == 3 && p > 3) return false;
  return true;
}

int default_candidate(int p, int nrhs, int vdtype) {
  const int order_pref[] = {2, 1, 0, 4};
  for (int c : order_pref)
    if (candidate_ok(p, c, nrhs, vdtype)) return c;
  return -1;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  const auto colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

}  // namespace

Batch::Batch(const std::vector<const Op*>& ops_in, int nrhs_in, void* work, size_t work_bytes)
    : ops(ops_in), nrhs(nrhs_in) {
  if (ops.empty()) throw Error(PAFEM_EINVAL, "empty batch");
  if (nrhs < 2 || nrhs % 2) throw Error(PAFEM_EINVAL, "nrhs must be a positive even number");
  qdtype = ops[0]->qdtype;
  kind = ops[0]->kind;
  if (kind != PAFEM_MASS && kind != PAFEM_DIFFUSION)
    throw Error(PAFEM_EUNSUPPORTED, "batched apply: mass or diffusion operators with stored D");
  for (const Op* o : ops) {
    if (o->qdtype != qdtype || o->kind != kind)
      throw Error(PAFEM_EINVAL, "all operators of a batch need the same kind and qdata dtype");
    if (o->space->dim != 3) throw Error(PAFEM_EUNSUPPORTED, "batched apply is built for hexahedra");
    if (o->flags & PAFEM_OP_VECTOR3) throw Error(PAFEM_EUNSUPPORTED, "batched apply of vector operators");
    if (o->space->p > 6) throw Error(PAFEM_EUNSUPPORTED, "batched apply is built for orders 1..6");
    if (o->q1d != o->space->p + 2) throw Error(PAFEM_EUNSUPPORTED, "batched apply needs q1d = p+2");
  }
  if (qdtype == PAFEM_F64)
    vdtype = PAFEM_F64;
  else if (qdtype == PAFEM_F32)
    vdtype = PAFEM_F32;
  else
    throw Error(PAFEM_EUNSUPPORTED, "batched apply supports F64 and F32 operators");
  if (!work || work_bytes < workspace_bytes(int(ops.size())))
    throw Error(PAFEM_ESHAPE, "batch workspace too small");
  d_meshes = static_cast<BatchMesh*>(work);
  // meshes sorted by order; one group per order
  order.resize(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) order[i] = int(i);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return ops[a]->space->p < ops[b]->space->p; });
  for (size_t k = 0; k < order.size(); ++k) {
    const int p = ops[order[k]]->space->p;
    if (groups.empty() || groups.back().p != p) {
      Group g;
      g.p = p;
      g.first = int(k);
      g.count = 0;
      g.cand = default_candidate(p, nrhs, vdtype);
      if (g.cand < 0) throw Error(PAFEM_EINVAL, "no tile shape divides nrhs");
      groups.push_back(g);
    }
    groups.back().count++;
  }
  hipc(hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking), "batch stream");
}

Batch::~Batch() {
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  if (capture_stream) hipStreamDestroy(capture_stream);
}

size_t Batch::workspace_bytes(int nops) { return align256(sizeof(BatchMesh) * size_t(nops)); }

void Batch::build_descriptors(const void* const* x, void* const* y) {
  host.assign(ops.size(), BatchMesh{});
  for (const Group& g : groups) {
    const int ne_tile = batch_tile_elems(g.cand);
    int block = 0;
    for (int k = g.first; k < g.first + g.count; ++k) {
      const Op* o = ops[order[k]];
      const DevSpace& sp = o->space->dev;
      BatchMesh& M = host[k];
      M.gmap = sp.gmap;
      M.bmask = sp.bmask;
      M.qdata = o->qdata;
      M.x = x[order[k]];
      M.y = y[order[k]];
      M.ne = int32_t(sp.ne);
      M.ndofs = int32_t(sp.ndofs);
      M.block_begin = block;
      M.constrained = (o->flags & PAFEM_OP_CONSTRAINED) ? 1 : 0;
      block += int((sp.ne + ne_tile - 1) / ne_tile);
    }
  }
}

int Batch::group_blocks(const Group& g) const {
  const int ne_tile = batch_tile_elems(g.cand);
  int blocks = 0;
  for (int k = g.first; k < g.first + g.count; ++k)
    blocks += int((ops[order[k]]->space->ne + ne_tile - 1) / ne_tile);
  return blocks;
}

void Batch::upload(hipStream_t st) {
  hipc(hipMemcpyAsync(d_meshes, host.data(), sizeof(BatchMesh) * host.size(),
                      hipMemcpyHostToDevice, st),
       "batch descriptors");
  hipc(hipStreamSynchronize(st), "batch descriptors sync");
}

void Batch::launch_group(const Group& g, hipStream_t st) const {
  const Op* o = ops[order[g.first]];
  const DevSpace& sp = o->space->dev;
  const int Q = g.p + 2, D = g.p + 1;
  // the 1D tables B (then G) of this order, in the compute precision
  const size_t off = table_offset_doubles(Q, D, sp.ng) + 2 * Q;
  const void* tabB = vdtype == PAFEM_F64 ? static_cast<const void*>(sp.tables + off)
                                         : static_cast<const void*>(sp.tables32 + off);
  if (!launch_batch_apply(g.p, g.cand, vdtype, qdtype, kind, d_meshes + g.first, g.count,
                          group_blocks(g), tabB, nrhs, st))
    throw Error(PAFEM_EUNSUPPORTED, "batched kernel not built for order " + std::to_string(g.p));
}

void Batch::launch_all(hipStream_t st) const {
  launch_batch_init(vdtype, d_meshes, int(ops.size()), nrhs, st);
  for (const Group& g : groups) launch_group(g, st);
}

void Batch::prepare(const void* const* x, void* const* y, hipStream_t st) {
  std::vector<const void*> xs(x, x + ops.size());
  std::vector<void*> ys(y, y + ops.size());
  if (exec && xs == cur_x && ys == cur_y && !dirty) return;
  build_descriptors(x, y);
  upload(st);
  if (exec) {
    hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  if (graph) {
    hipGraphDestroy(graph);
    graph = nullptr;
  }
  // capture on the library's own stream; the graph is then launched on the caller's
  hipc(hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    launch_all(capture_stream);
  } catch (...) {
    hipGraph_t g = nullptr;
    hipStreamEndCapture(capture_stream, &g);
    if (g) hipGraphDestroy(g);
    throw;
  }
  hipc(hipStreamEndCapture(capture_stream, &graph), "end capture");
  hipc(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
  cur_x = xs;
  cur_y = ys;
  dirty = false;
}

void Batch::apply(const void* const* x, void* const* y, hipStream_t st) {
  prepare(x, y, st);
  hipc(hipGraphLaunch(exec, st), "graph launch");
}

void Batch::set_candidate(int p, int cand) {
  for (Group& g : groups)
    if (g.p == p) {
      const int c = cand < 0 ? default_candidate(p, nrhs, vdtype) : cand;
      if (!candidate_ok(p, c, nrhs, vdtype))
        throw Error(PAFEM_EINVAL, "tile candidate " + std::to_string(cand) +
                                      " not available for order " + std::to_string(p));
      g.cand = c;
      dirty = true;
      return;
    }
  throw Error(PAFEM_EINVAL, "no mesh of order " + std::to_string(p) + " in the batch");
}

void Batch::autotune(const void* const* x, void* const* y, const char* cache_path, int reps,
                     hipStream_t st) {
  const std::string arch = arch_name();
  // cache lines: arch kind dtype nrhs p candidate
  std::map<std::tuple<std::string, int, int, int, int>, int> cache;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string a;
    int k, dt, nr, p, c;
    while (in >> a >> k >> dt >> nr >> p >> c) cache[{a, k, dt, nr, p}] = c;
  }
  bool changed = false;
  reps = std::max(1, reps);
  for (Group& g : groups) {
    const auto key = std::make_tuple(arch, kind, vdtype, nrhs, g.p);
    const auto hit = cache.find(key);
    if (hit != cache.end() && candidate_ok(g.p, hit->second, nrhs, vdtype)) {
      g.cand = hit->second;
      continue;
    }
    float best = 1e30f;
    int best_c = g.cand;
    hipEvent_t a, b;
    hipc(hipEventCreate(&a), "event");
    hipc(hipEventCreate(&b), "event");
    for (int c = 0; c < kBatchCandidates; ++c) {
      if (!candidate_ok(g.p, c, nrhs, vdtype)) continue;
      g.cand = c;
      build_descriptors(x, y);
      upload(st);
      launch_group(g, st);  // warm-up
      hipc(hipEventRecord(a, st), "event");
      for (int r = 0; r < reps; ++r) launch_group(g, st);
      hipc(hipEventRecord(b, st), "event");
      hipc(hipEventSynchronize(b), "event sync");
      float ms = 0.f;
      hipc(hipEventElapsedTime(&ms, a, b), "event time");
      timings.push_back({g.p, c, ms / reps});
      if (ms < best) {
        best = ms;
        best_c = c;
      }
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    g.cand = best_c;
    cache[key] = best_c;
    changed = true;
  }
  dirty = true;
  if (cache_path && changed) {
    std::ofstream out(cache_path);
    for (const auto& kv : cache)
      out << std::get<0>(kv.first) << ' ' << std::get<1>(kv.first) << ' ' << std::get<2>(kv.first)
          << ' ' << std::get<3>(kv.first) << ' ' << std::get<4>(kv.first) << ' ' << kv.second
          << '\n';
  }
}

std::string Batch::describe() const {
  std::ostringstream os;
  os << "{\"nrhs\": " << nrhs << ", \"dtype\": \"" << (vdtype == PAFEM_F64 ? "f64" : "f32")
     << "\", \"groups\": [";
  for (size_t i = 0; i < groups.size(); ++i) {
    const Group& g = groups[i];
    os << (i ? ", " : "") << "{\"p\": " << g.p << ", \"meshes\": " << g.count
       << ", \"tile_elems\": " << batch_tile_elems(g.cand)
       << ", \"tile_rhs\": " << batch_tile_rhs(g.cand) << ", \"candidate\": " << g.cand << "}";
  }
  os << "], \"tuning\": [";
  for (size_t i = 0; i < timings.size(); ++i)
    os << (i ? ", " : "") << "{\"p\": " << timings[i].p << ", \"candidate\": " << timings[i].cand
       << ", \"ms\": " << timings[i].ms << "}";
  os << "]}";
  return os.str();
}

}  // namespace pafem
