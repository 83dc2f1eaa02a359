// Learned element preconditioner: the network object (parameters -- the element
// network and the element basis V --, Adam state, bf16 copies and activations in
// one caller-owned device buffer), the preconditioner application, the training
// loss and its gradient, and flexible CG with a Jacobi fallback.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "capi.hpp"
#include "launch.hpp"
#include "mg.hpp"
#include "mlp.hpp"
#include "solver.hpp"

namespace pafem {

namespace {

constexpr int kLossPartials = 2 * 512;
constexpr int kNetIn = 16;  // 8 octant log-ratios, padded to the MFMA K step

int round16(int v) { return (v + 15) / 16 * 16; }

struct NetDims {
  int p = 0, dpe = 0, in = 0, hid = 0, out = 0;
  int64_t nparams = 0;
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0, oV = 0;
};

// Parameters, FP32, in this order: W1 [hid][in], b1, W2 [hid][hid], b2,
// W3 [out][hid], b3 [out], V [(p+1)^3][out]; out = kLowRank.
NetDims net_dims(int order, int hidden) {
  if (order < 1 || order > 4) throw Error(PAFEM_EUNSUPPORTED, "learned preconditioner: orders 1..4");
  if (hidden < 16 || hidden > 128 || hidden % 16)
    throw Error(PAFEM_EINVAL, "hidden width must be a multiple of 16 in 16..128");
  NetDims d;
  d.p = order;
  d.dpe = (order + 1) * (order + 1) * (order + 1);
  d.in = kNetIn;
  d.hid = hidden;
  d.out = kLowRank;
  d.oW1 = 0;
  d.ob1 = d.oW1 + int64_t(d.hid) * d.in;
  d.oW2 = d.ob1 + d.hid;
  d.ob2 = d.oW2 + int64_t(d.hid) * d.hid;
  d.oW3 = d.ob2 + d.hid;
  d.ob3 = d.oW3 + int64_t(d.out) * d.hid;
  d.oV = d.ob3 + d.out;
  d.nparams = d.oV + int64_t(d.dpe) * d.out;
  return d;
}

struct NetLayout {
  size_t params, grads, m, v, w1b, w2b, w2tb, w3b, w3tb, X, H1, H2, O, dO, dZ2, dZ1, part, partb,
      total;
};

NetLayout net_layout(const NetDims& d, int64_t rows, int64_t train_rows) {
  NetLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  const size_t np = size_t(d.nparams);
  L.params = take(np * 4);
  L.grads = take(np * 4);
  L.m = take(np * 4);
  L.v = take(np * 4);
  L.w1b = take(size_t(d.hid) * d.in * 2);
  L.w2b = take(size_t(d.hid) * d.hid * 2);
  L.w2tb = take(size_t(d.hid) * d.hid * 2);
  L.w3b = take(size_t(d.out) * d.hid * 2);
  L.w3tb = take(size_t(d.hid) * d.out * 2);
  L.X = take(size_t(rows) * d.in * 2);
  L.H1 = take(size_t(rows) * d.hid * 2);
  L.H2 = take(size_t(rows) * d.hid * 2);
  L.O = take(size_t(rows) * d.out * 4);
  L.dO = take(size_t(train_rows) * d.out * 2);
  L.dZ2 = take(size_t(train_rows) * d.hid * 2);
  L.dZ1 = take(size_t(train_rows) * d.hid * 2);
  // partial weight gradients of the largest layer (N x K of the three GEMMs)
  const size_t nblk = size_t(std::max(1, wgrad_blocks(int(std::max<int64_t>(train_rows, 1)))));
  const size_t nk = size_t(std::max({d.hid * d.in, d.hid * d.hid, d.out * d.hid}));
  L.part = take(nblk * nk * 4);
  L.partb = take(nblk * std::max(d.hid, d.out) * 4);
  L.total = o;
  return L;
}

}  // namespace

struct Net {
  NetDims d;
  NetLayout L;
  int64_t rows = 0, train_rows = 0;
  char* base = nullptr;
  int step = 0;
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(base + off);
  }
  float* params() const { return at<float>(L.params); }
  float* grads() const { return at<float>(L.grads); }

  void refresh_bf16(hipStream_t st) const {
    launch_cast_weights(params() + d.oW1, at<uint16_t>(L.w1b), nullptr, d.hid, d.in, st);
    launch_cast_weights(params() + d.oW2, at<uint16_t>(L.w2b), at<uint16_t>(L.w2tb), d.hid, d.hid,
                        st);
    launch_cast_weights(params() + d.oW3, at<uint16_t>(L.w3b), at<uint16_t>(L.w3tb), d.out, d.hid,
                        st);
  }

  void forward(const uint16_t* X, int64_t n, hipStream_t st) const {
    if (n > rows) throw Error(PAFEM_ESHAPE, "more rows than the network was created for");
    const int M = int(n);
    launch_gemm_rows(kEpiReluBf16, X, at<uint16_t>(L.w1b), params() + d.ob1, nullptr,
                     at<uint16_t>(L.H1), M, d.hid, d.in, st);
    launch_gemm_rows(kEpiReluBf16, at<uint16_t>(L.H1), at<uint16_t>(L.w2b), params() + d.ob2,
                     nullptr, at<uint16_t>(L.H2), M, d.hid, d.hid, st);
    launch_gemm_rows(kEpiBiasF32, at<uint16_t>(L.H2), at<uint16_t>(L.w3b), params() + d.ob3,
                     nullptr, at<float>(L.O), M, d.out, d.hid, st);
  }

  // gradients of sum(dO * out) for the last forward pass on X (rows n)
  void backward(const uint16_t* X, const uint16_t* dO, int64_t n, hipStream_t st) const {
    if (n > train_rows) throw Error(PAFEM_ESHAPE, "more rows than the network trains on");
    const int M = int(n);
    float* part = at<float>(L.part);
    float* partb = at<float>(L.partb);
    launch_gemm_wgrad(dO, at<uint16_t>(L.H2), part, partb, grads() + d.oW3, grads() + d.ob3, M,
                      d.out, d.hid, st);
    launch_gemm_rows(kEpiMaskBf16, dO, at<uint16_t>(L.w3tb), nullptr, at<uint16_t>(L.H2),
                     at<uint16_t>(L.dZ2), M, d.hid, d.out, st);
    launch_gemm_wgrad(at<uint16_t>(L.dZ2), at<uint16_t>(L.H1), part, partb, grads() + d.oW2,
                      grads() + d.ob2, M, d.hid, d.hid, st);
    launch_gemm_rows(kEpiMaskBf16, at<uint16_t>(L.dZ2), at<uint16_t>(L.w2tb), nullptr,
                     at<uint16_t>(L.H1), at<uint16_t>(L.dZ1), M, d.hid, d.hid, st);
    launch_gemm_wgrad(at<uint16_t>(L.dZ1), X, part, partb, grads() + d.oW1, grads() + d.ob1, M,
                      d.hid, d.in, st);
  }

  void adam(float lr, hipStream_t st) {
    ++step;
    launch_adam(params(), grads(), at<float>(L.m), at<float>(L.v), int(d.nparams), lr, 0.9f,
                0.999f, 1e-8f, step, st);
    refresh_bf16(st);
  }
};

namespace {

struct LearnedLayout {
  size_t z, t, u, v, w, c, idb, partV, partials, ticket, scal, opwork, total;
};

LearnedLayout learned_layout(const Op& op) {
  const Space& s = *op.space;
  const size_t n = size_t(s.ndofs);
  LearnedLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.z = take(n * 8);
  L.t = take(n * 8);
  L.u = take(n * 8);
  L.v = take(n * 8);
  L.w = take(n * 8);
  L.c = take(size_t(s.ne) * kLowRank * 4);
  L.idb = take(size_t(s.ne) * 4);
  L.partV = take(size_t(kLowRankGradBlocks) * s.dpe * kLowRank * 4);
  L.partials = take(kLossPartials * 8);
  L.ticket = take(64);
  L.scal = take(64);
  L.opwork = take(op_work_bytes(op));
  L.total = o;
  return L;
}

void check_net_op(const Net& net, const Op& op) {
  require(!(op.flags & PAFEM_OP_VECTOR3), PAFEM_EUNSUPPORTED, "the learned preconditioner needs a scalar operator");
  require(op.space->dim == 3, PAFEM_EUNSUPPORTED, "the learned preconditioner is built for hexahedra");
  require(op.qdtype == PAFEM_F64, PAFEM_EINVAL, "learned preconditioner needs an FP64 operator");
  require(op.space->p == net.d.p, PAFEM_EINVAL, "network order differs from the space order");
  require(op.space->ne <= net.rows, PAFEM_ESHAPE, "mesh has more elements than the network rows");
}

// Element weights for this operator and the current parameters: the network on
// the element features, then c = softplus(output) and 1 / dbar_E.
void learned_setup(const Net& net, const Op& op, const float* feats, const double* diag,
                   char* work, const LearnedLayout& W, hipStream_t st) {
  const DevSpace& sp = op.space->dev;
  launch_net_inputs(sp, feats, net.d.in, net.at<uint16_t>(net.L.X), st);
  net.forward(net.at<uint16_t>(net.L.X), sp.ne, st);
  launch_lowrank_coeffs(sp, diag, net.at<float>(net.L.O), reinterpret_cast<float*>(work + W.c),
                        reinterpret_cast<float*>(work + W.idb), st);
}

// z += the low-rank correction of r, with the element weights of the last learned_setup
void learned_correct(const Net& net, const Op& op, const double* r, double* z, char* work,
                     const LearnedLayout& W, hipStream_t st) {
  launch_lowrank_apply(op.space->dev, net.params() + net.d.oV,
                       reinterpret_cast<const float*>(work + W.c),
                       reinterpret_cast<const float*>(work + W.idb), r, z, st);
}

// z = M(r) with the element weights of the last learned_setup
void learned_apply(const Net& net, const Op& op, const double* diag, const double* r, double* z,
                   char* work, const LearnedLayout& W, hipStream_t st,
                   int ess_mode = kJacobiEssZero) {
  launch_jacobi(op.space->dev, r, diag, z, st, ess_mode);
  learned_correct(net, op, r, z, work, W, st);
}

}  // namespace

}  // namespace pafem

using namespace pafem;

struct pafem_net_s {
  Net net;
};

extern "C" {

pafem_status pafem_net_storage_bytes(int32_t order, int32_t hidden, int64_t max_rows,
                                     int64_t max_train_rows, size_t* nbytes) {
  return guarded([&] {
    require(nbytes && max_rows > 0 && max_train_rows >= 0 && max_train_rows <= max_rows,
            PAFEM_EINVAL, "bad arguments");
    *nbytes = net_layout(net_dims(order, hidden), max_rows, max_train_rows).total;
  });
}

pafem_status pafem_net_create(int32_t order, int32_t hidden, int64_t max_rows,
                              int64_t max_train_rows, void* storage, size_t nbytes,
                              pafem_net* out) {
  return guarded([&] {
    require(out && storage && max_rows > 0 && max_train_rows >= 0 && max_train_rows <= max_rows,
            PAFEM_EINVAL, "bad arguments");
    require(max_rows < (int64_t(1) << 31), PAFEM_EINVAL, "too many rows");
    const NetDims d = net_dims(order, hidden);
    const NetLayout L = net_layout(d, max_rows, max_train_rows);
    require(nbytes >= L.total, PAFEM_ESHAPE, "storage too small: need " + std::to_string(L.total));
    require((reinterpret_cast<uintptr_t>(storage) & 255) == 0, PAFEM_EINVAL,
            "storage must be 256-byte aligned");
    auto* n = new pafem_net_s();
    n->net.d = d;
    n->net.L = L;
    n->net.rows = max_rows;
    n->net.train_rows = max_train_rows;
    n->net.base = static_cast<char*>(storage);
    *out = n;
  });
}

void pafem_net_destroy(pafem_net net) { delete net; }

pafem_status pafem_net_dims(pafem_net net, int32_t* in_dim, int32_t* hidden, int32_t* out_dim,
                            int64_t* nparams) {
  return guarded([&] {
    require(net != nullptr, PAFEM_EINVAL, "null network");
    const NetDims& d = net->net.d;
    if (in_dim) *in_dim = d.in;
    if (hidden) *hidden = d.hid;
    if (out_dim) *out_dim = d.out;
    if (nparams) *nparams = d.nparams;
  });
}

pafem_status pafem_net_set_params(pafem_net net, const float* host_params, void* stream) {
  return guarded([&] {
    require(net && host_params, PAFEM_EINVAL, "null pointer argument");
    Net& n = net->net;
    auto st = static_cast<hipStream_t>(stream);
    const size_t bytes = size_t(n.d.nparams) * 4;
    hip_check(hipMemcpyAsync(n.params(), host_params, bytes, hipMemcpyHostToDevice, st), "params");
    hip_check(hipMemsetAsync(n.at<float>(n.L.m), 0, bytes, st), "adam m");
    hip_check(hipMemsetAsync(n.at<float>(n.L.v), 0, bytes, st), "adam v");
    hip_check(hipMemsetAsync(n.grads(), 0, bytes, st), "grads");
    n.step = 0;
    n.refresh_bf16(st);
    hip_check(hipStreamSynchronize(st), "params sync");
  });
}

pafem_status pafem_net_get_params(pafem_net net, float* host_params, void* stream) {
  return guarded([&] {
    require(net && host_params, PAFEM_EINVAL, "null pointer argument");
    auto st = static_cast<hipStream_t>(stream);
    hip_check(hipMemcpyAsync(host_params, net->net.params(), size_t(net->net.d.nparams) * 4,
                             hipMemcpyDeviceToHost, st), "params");
    hip_check(hipStreamSynchronize(st), "params sync");
  });
}

pafem_status pafem_net_get_grads(pafem_net net, float* host_grads, void* stream) {
  return guarded([&] {
    require(net && host_grads, PAFEM_EINVAL, "null pointer argument");
    auto st = static_cast<hipStream_t>(stream);
    hip_check(hipMemcpyAsync(host_grads, net->net.grads(), size_t(net->net.d.nparams) * 4,
                             hipMemcpyDeviceToHost, st), "grads");
    hip_check(hipStreamSynchronize(st), "grads sync");
  });
}

pafem_status pafem_net_get_state(pafem_net net, float* host_state, int32_t* step, void* stream) {
  return guarded([&] {
    require(net && host_state && step, PAFEM_EINVAL, "null pointer argument");
    const Net& n = net->net;
    auto st = static_cast<hipStream_t>(stream);
    const size_t count = size_t(n.d.nparams);
    hip_check(hipMemcpyAsync(host_state, n.params(), count * 4, hipMemcpyDeviceToHost, st),
              "state params");
    hip_check(hipMemcpyAsync(host_state + count, n.at<float>(n.L.m), count * 4,
                             hipMemcpyDeviceToHost, st), "state adam m");
    hip_check(hipMemcpyAsync(host_state + 2 * count, n.at<float>(n.L.v), count * 4,
                             hipMemcpyDeviceToHost, st), "state adam v");
    hip_check(hipStreamSynchronize(st), "state sync");
    *step = n.step;
  });
}

pafem_status pafem_net_set_state(pafem_net net, const float* host_state, int32_t step,
                                 void* stream) {
  return guarded([&] {
    require(net && host_state, PAFEM_EINVAL, "null pointer argument");
    require(step >= 0, PAFEM_EINVAL, "negative Adam step count");
    Net& n = net->net;
    auto st = static_cast<hipStream_t>(stream);
    const size_t count = size_t(n.d.nparams);
    hip_check(hipMemcpyAsync(n.params(), host_state, count * 4, hipMemcpyHostToDevice, st),
              "state params");
    hip_check(hipMemcpyAsync(n.at<float>(n.L.m), host_state + count, count * 4,
                             hipMemcpyHostToDevice, st), "state adam m");
    hip_check(hipMemcpyAsync(n.at<float>(n.L.v), host_state + 2 * count, count * 4,
                             hipMemcpyHostToDevice, st), "state adam v");
    hip_check(hipMemsetAsync(n.grads(), 0, count * 4, st), "grads");
    n.step = step;
    n.refresh_bf16(st);
    hip_check(hipStreamSynchronize(st), "state sync");
  });
}

pafem_status pafem_net_forward(pafem_net net, const uint16_t* x, float* out, int64_t rows,
                               void* stream) {
  return guarded([&] {
    require(net && x && out && rows > 0, PAFEM_EINVAL, "bad arguments");
    const Net& n = net->net;
    auto st = static_cast<hipStream_t>(stream);
    n.forward(x, rows, st);
    hip_check(hipMemcpyAsync(out, n.at<float>(n.L.O), size_t(rows) * n.d.out * 4,
                             hipMemcpyDeviceToDevice, st), "forward output");
  });
}

pafem_status pafem_net_backward(pafem_net net, const uint16_t* x, const uint16_t* dout,
                                int64_t rows, void* stream) {
  return guarded([&] {
    require(net && x && dout && rows > 0, PAFEM_EINVAL, "bad arguments");
    const Net& n = net->net;
    auto st = static_cast<hipStream_t>(stream);
    n.forward(x, rows, st);
    n.backward(x, dout, rows, st);
  });
}

pafem_status pafem_net_adam_step(pafem_net net, float lr, void* stream) {
  return guarded([&] {
    require(net != nullptr, PAFEM_EINVAL, "null network");
    net->net.adam(lr, static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"

namespace pafem {

void learned_precond(const Net& net, const Op& op, const float* feats, const double* diag,
                     const double* r, double* z, void* work, size_t work_bytes, hipStream_t st) {
  check_net_op(net, op);
  const LearnedLayout W = learned_layout(op);
  require(work && work_bytes >= W.total, PAFEM_ESHAPE, "workspace too small");
  char* w = static_cast<char*>(work);
  learned_setup(net, op, feats, diag, w, W, st);
  learned_apply(net, op, diag, r, z, w, W, st);
}

void learned_loss_grad(Net& net, const Op& op, const float* feats, const double* diag,
                       const double* r, const double* e, double* loss, void* work,
                       size_t work_bytes, hipStream_t st) {
  check_net_op(net, op);
  require(op.space->ne <= net.train_rows, PAFEM_ESHAPE,
          "mesh has more elements than the network trains on");
  const LearnedLayout W = learned_layout(op);
  require(work && work_bytes >= W.total, PAFEM_ESHAPE, "workspace too small");
  char* w = static_cast<char*>(work);
  const DevSpace& sp = op.space->dev;
  auto* z = reinterpret_cast<double*>(w + W.z);
  auto* t = reinterpret_cast<double*>(w + W.t);
  auto* u = reinterpret_cast<double*>(w + W.u);
  auto* v = reinterpret_cast<double*>(w + W.v);
  auto* g = reinterpret_cast<double*>(w + W.w);
  auto* partials = reinterpret_cast<double*>(w + W.partials);
  auto* ticket = reinterpret_cast<uint32_t*>(w + W.ticket);
  auto* scal = reinterpret_cast<double*>(w + W.scal);
  learned_setup(net, op, feats, diag, w, W, st);
  learned_apply(net, op, diag, r, z, w, W, st);
  launch_diff(e, z, t, sp.ndofs, st);
  apply_op(op, t, u, w + W.opwork, st);
  // the reduction ticket is cleared by a kernel rather than a memset (no memset nodes
  // when the caller's stream is being captured); capture of this call is not tested
  launch_fill(reinterpret_cast<double*>(ticket), 0.0, 1, st);
  launch_loss(sp, u, r, diag, v, partials, ticket, scal, st);
  apply_op(op, v, g, w + W.opwork, st);
  // dL/dz = scal[1] * g; the basis gradient goes straight into the gradient vector
  launch_lowrank_grad(sp, net.params() + net.d.oV, reinterpret_cast<const float*>(w + W.c),
                      reinterpret_cast<const float*>(w + W.idb), r, g, scal + 1,
                      net.at<uint16_t>(net.L.dO), reinterpret_cast<float*>(w + W.partV),
                      net.grads() + net.d.oV, st);
  net.backward(net.at<uint16_t>(net.L.X), net.at<uint16_t>(net.L.dO), sp.ne, st);
  if (loss) hip_check(hipMemcpyAsync(loss, scal, 8, hipMemcpyDeviceToDevice, st), "loss copy");
}

// ---- flexible CG ---------------------------------------------------------------

struct FCGLayout {
  size_t state, partials, hist, r, z, zold, p, q, dotp, learned, total;
};

FCGLayout fcg_layout(const Op& op, int max_iter) {
  const size_t n = size_t(op.space->ndofs);
  FCGLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.state = take(sizeof(CGState));
  L.partials = take(3 * kCGBlocks * sizeof(double));
  L.hist = take((size_t(max_iter) + 1) * sizeof(double));
  L.r = take(n * 8);
  L.z = take(n * 8);
  L.zold = take(n * 8);
  L.p = take(n * 8);
  L.q = take(n * 8);
  L.dotp = take(size_t(pa_apply_blocks(op.space->dev)) * sizeof(double));
  L.learned = take(learned_layout(op).total);
  L.total = o;
  return L;
}

size_t fcg_work_bytes(const Op& op, int max_iter) { return fcg_layout(op, max_iter).total; }

// returns 0 ok, PAFEM_ENOTCONV or PAFEM_EBREAKDOWN
pafem_status fcg_solve(const Op& op, Net* net, const float* feats, const double* diag,
                       const double* b, double* x, void* work, size_t work_bytes,
                       const pafem_solve_opts& opts, pafem_fcg_result& res, hipStream_t st) {
  require(op.qdtype == PAFEM_F64, PAFEM_EINVAL, "FCG needs an FP64 operator");
  require(!mixed_or_nonsymmetric(op.kind), PAFEM_EINVAL,
          "CG needs a symmetric operator");
  require(!(op.flags & PAFEM_OP_VECTOR3), PAFEM_EUNSUPPORTED, "FCG needs a scalar operator");
  require(diag != nullptr, PAFEM_EINVAL, "FCG needs the operator diagonal");
  if (net) {
    check_net_op(*net, op);
    require(feats != nullptr, PAFEM_EINVAL, "learned preconditioner needs element features");
  }
  const FCGLayout L = fcg_layout(op, opts.max_iter);
  require(work && work_bytes >= L.total, PAFEM_ESHAPE,
          "workspace too small: need " + std::to_string(L.total));
  char* w = static_cast<char*>(work);
  auto* state = reinterpret_cast<CGState*>(w + L.state);
  auto* partials = reinterpret_cast<double*>(w + L.partials);
  auto* hist = reinterpret_cast<double*>(w + L.hist);
  auto* r = reinterpret_cast<double*>(w + L.r);
  auto* z = reinterpret_cast<double*>(w + L.z);
  auto* zold = reinterpret_cast<double*>(w + L.zold);
  auto* p = reinterpret_cast<double*>(w + L.p);
  auto* q = reinterpret_cast<double*>(w + L.q);
  auto* dotp = reinterpret_cast<double*>(w + L.dotp);
  const int nap = pa_apply_blocks(op.space->dev);
  const uint8_t* ess = (op.flags & PAFEM_OP_CONSTRAINED) ? op.space->dev.bmask : nullptr;
  char* lw = w + L.learned;
  const LearnedLayout LW = learned_layout(op);
  const DevSpace& sp = op.space->dev;
  const int64_t n = sp.ndofs;
  bool use_net = net != nullptr;
  res = pafem_fcg_result{};
  res.fallback_iter = -1;

  if (use_net) learned_setup(*net, op, feats, diag, lw, LW, st);
  // a constrained operator is the identity on the essential rows: the preconditioner
  // passes r through there; an unconstrained one gets Jacobi on every row (the learned
  // correction touches only the non-essential dofs either way)
  const int ess_mode = ess ? kJacobiEssKeep : kJacobiEssDiag;
  auto precond = [&](const double* rr, double* zz) {
    if (use_net)
      learned_apply(*net, op, diag, rr, zz, lw, LW, st, ess_mode);
    else
      launch_jacobi(sp, rr, diag, zz, st, ess_mode);
  };

  launch_cg_reset(state, opts.max_iter + 1, st);
  if (!opts.zero_guess) apply_op(op, x, q, lw + LW.opwork, st);
  launch_fcg_init(state, partials, b, opts.zero_guess ? nullptr : q, x, r, opts.zero_guess,
                  opts.rel_tol, hist, n, st);
  precond(r, z);
  launch_fcg_start(state, partials, r, z, p, n, st);
  const int check = std::max(1, opts.check_every);
  double best_rr = 1e308;
  int launched = 0;
  CGState h{};
  while (true) {
    hip_check(hipMemcpyAsync(&h, state, sizeof(CGState), hipMemcpyDeviceToHost, st), "state");
    hip_check(hipStreamSynchronize(st), "fcg sync");
    if (h.done == 1) break;
    const bool bad = h.done == 2 || h.done == 3 || !std::isfinite(h.rr) ||
                     (h.iter > 0 && h.rr > 1e6 * best_rr);
    if (bad) {
      if (!use_net) break;  // Jacobi itself failed: breakdown
      // fall back to Jacobi-PCG from the current iterate
      use_net = false;
      res.fell_back = 1;
      res.fallback_iter = h.iter;
      hip_check(hipMemsetAsync(&state->done, 0, 4, st), "reset flag");
      apply_op(op, x, q, lw + LW.opwork, st);
      launch_fcg_init(state, partials, b, q, x, r, 0, opts.rel_tol, nullptr, n, st);
      precond(r, z);
      launch_fcg_start(state, partials, r, z, p, n, st);
      continue;
    }
    if (h.iter > 0) best_rr = std::min(best_rr, h.rr);
    if (launched >= opts.max_iter || h.iter >= opts.max_iter) break;
    const int batch = std::min(check, opts.max_iter - launched);
    for (int k = 0; k < batch; ++k) {
      apply_op(op, p, q, lw + LW.opwork, st, dotp);
      launch_cg_alpha<double>(state, partials, dotp, nap, ess, p, n, st);
      // new z into the spare buffer: the update writes its Jacobi part
      launch_fcg_update(state, partials, x, r, p, q, diag, ess, zold, hist, n, st);
      if (use_net) learned_correct(*net, op, r, zold, lw, LW, st);
      launch_fcg_beta(state, partials, r, zold, z, n, st);
      launch_fcg_direction(state, zold, p, n, st);
      std::swap(z, zold);
    }
    launched += batch;
  }
  apply_op(op, x, q, lw + LW.opwork, st);
  launch_residual(state, partials, b, q, nullptr, n, st);
  hip_check(hipMemcpyAsync(&h, state, sizeof(CGState), hipMemcpyDeviceToHost, st), "state");
  hip_check(hipStreamSynchronize(st), "fcg sync");
  res.iters = h.iter;
  res.converged = h.done == 1;
  res.rel_res = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
  res.true_rel_res = h.bb > 0 ? std::sqrt(h.res2 / h.bb) : 0.0;
  if (opts.res_hist && opts.res_hist_cap > 0) {
    const int nh = std::min(opts.res_hist_cap, h.iter + 1);
    hip_check(hipMemcpy(opts.res_hist, hist, size_t(nh) * sizeof(double), hipMemcpyDeviceToHost),
              "history");
  }
  if (h.done == 1) return PAFEM_OK;
  if (h.done == 2 || h.done == 3) return PAFEM_EBREAKDOWN;
  return PAFEM_ENOTCONV;
}

}  // namespace pafem

extern "C" {

pafem_status pafem_learned_features(pafem_space space, const double* kappa, int32_t q1d,
                                    float* feats, void* stream) {
  return guarded([&] {
    require(space && space->s && feats, PAFEM_EINVAL, "null pointer argument");
    require(space->s->uploaded, PAFEM_EINVAL, "space has no device image");
    require(space->s->dim == 3, PAFEM_EUNSUPPORTED, "element features are built for hexahedra");
    require(q1d >= 1 && q1d <= kMaxQ1d, PAFEM_EUNSUPPORTED, "q1d out of range");
    launch_patch_features(space->s->dev, kappa, q1d, feats, static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_learned_workspace_bytes(pafem_op op, size_t* nbytes) {
  return guarded([&] {
    require(op && nbytes, PAFEM_EINVAL, "null pointer argument");
    *nbytes = learned_layout(op->op).total;
  });
}

pafem_status pafem_learned_precond(pafem_net net, pafem_op op, const float* feats,
                                   const double* diag, const double* r, double* z, void* work,
                                   size_t work_bytes, void* stream) {
  return guarded([&] {
    require(net && op && feats && diag && r && z, PAFEM_EINVAL, "null pointer argument");
    learned_precond(net->net, op->op, feats, diag, r, z, work, work_bytes,
                    static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_learned_loss_grad(pafem_net net, pafem_op op, const float* feats,
                                     const double* diag, const double* r, const double* e,
                                     double* loss, void* work, size_t work_bytes, void* stream) {
  return guarded([&] {
    require(net && op && feats && diag && r && e, PAFEM_EINVAL, "null pointer argument");
    learned_loss_grad(net->net, op->op, feats, diag, r, e, loss, work, work_bytes,
                      static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_fcg_workspace_bytes(pafem_op op, int32_t max_iter, size_t* nbytes) {
  return guarded([&] {
    require(op && nbytes && max_iter >= 0, PAFEM_EINVAL, "bad arguments");
    *nbytes = fcg_work_bytes(op->op, max_iter);
  });
}

pafem_status pafem_fcg_solve(pafem_op op, pafem_net net, const float* feats, const double* diag,
                             const double* b, double* x, void* work, size_t work_bytes,
                             const pafem_solve_opts* opts, pafem_fcg_result* result,
                             void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  pafem_status status = PAFEM_OK;
  pafem_status rc = guarded([&] {
    require(op && b && x && opts && result, PAFEM_EINVAL, "null pointer argument");
    require(opts->max_iter >= 0 && opts->rel_tol >= 0.0, PAFEM_EINVAL, "bad solver options");
    status = fcg_solve(op->op, net ? &net->net : nullptr, feats, diag, b, x, work, work_bytes,
                       *opts, *result, static_cast<hipStream_t>(stream));
    if (status == PAFEM_EBREAKDOWN) fail(status, "FCG breakdown");
    if (status == PAFEM_ENOTCONV) fail(status, "FCG did not converge");
  });
  if (result)
    result->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc != PAFEM_OK ? rc : status;
}

}  // extern "C"
