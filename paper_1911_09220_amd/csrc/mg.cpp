// Order multigrid: host orchestration of transfers, Chebyshev-Jacobi smoothing,
// power iteration, the V-cycle and flexible CG ("Scalable Linear Solvers":
// preconditioners for partially assembled operators need no matrix entries).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "capi.hpp"
#include "graph.hpp"
#include "internal.hpp"
#include "launch.hpp"
#include "mg.hpp"
#include "solver.hpp"

using namespace pafem;

namespace pafem {

struct PMG {
  int L = 0;
  std::vector<const Op*> ops;
  std::vector<const double*> diag;
  std::vector<double> lmax;
  std::vector<Interp1D> interp;  // interp[l]: level l+1 -> level l
  pafem_pmg_opts o{};
};

namespace {

const Space& uploaded(pafem_space sp) {
  require(sp != nullptr && sp->s != nullptr, PAFEM_EINVAL, "null space");
  require(sp->s->uploaded, PAFEM_EINVAL, "space has no device image: call pafem_space_upload");
  return *sp->s;
}

// h: the fine space is on a uniform refinement of the coarse space's mesh; the fine
// nodes are then mapped into each half of the parent's interval, (half + x) / 2
Interp1D make_interp(int pc, int pf, bool h) {
  require(pc >= 1 && pc <= pf, PAFEM_EINVAL, "transfer needs 1 <= coarse order <= fine order");
  require(pf + 1 <= kMaxInterpNodes, PAFEM_EINVAL, "transfer orders above 8 are not built");
  const int dc = pc + 1, df = pf + 1;
  std::vector<double> nc(dc), nf(df), pts(df), B(size_t(df) * dc), G(size_t(df) * dc);
  gauss_lobatto_01(dc, nc.data());
  gauss_lobatto_01(df, nf.data());
  Interp1D I{};
  I.h = h ? 1 : 0;
  for (int half = 0; half < (h ? 2 : 1); ++half) {
    for (int k = 0; k < df; ++k) pts[size_t(k)] = h ? 0.5 * (half + nf[size_t(k)]) : nf[size_t(k)];
    lagrange_tables(dc, nc.data(), df, pts.data(), B.data(), G.data());
    for (int k = 0; k < df * dc; ++k) I.v[half][k] = B[size_t(k)];
  }
  return I;
}

// true when the fine space's mesh is a uniform refinement of the coarse space's mesh
bool check_pair(const Space& c, const Space& f) {
  require(c.dim == 3 && f.dim == 3, PAFEM_EUNSUPPORTED, "order transfers are built for hexahedra");
  require(c.family == kFamilyH1 && f.family == kFamilyH1, PAFEM_EINVAL,
          "transfers are built between H1 spaces");
  const bool h = c.mesh != f.mesh;
  require(!h || (f.mesh->parent_id != 0 && f.mesh->parent_id == c.mesh->id), PAFEM_EINVAL,
          "transfer spaces must be built on one mesh object, or the fine one on a refinement "
          "of the coarse one's mesh");
  require(c.p <= f.p, PAFEM_EINVAL, "coarse order above fine order");
  return h;
}

struct SmootherLayout {
  size_t r, d, y, partials, scal, opwork, total;
};

SmootherLayout smoother_layout(const Op& op) {
  const size_t n = size_t(op.space->ndofs);
  SmootherLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.r = take(n * 8);
  L.d = take(n * 8);
  L.y = take(n * 8);
  L.partials = take(2 * kCGBlocks * sizeof(double));
  L.scal = take(64);  // scal, lam, ticket
  L.opwork = take(op_work_bytes(op));
  L.total = o;
  return L;
}

void check_smoother_op(const Op& op) {
  require(!(op.flags & PAFEM_OP_VECTOR3), PAFEM_EUNSUPPORTED, "smoothers need a scalar operator");
  require(op.qdtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "smoothers need an f64 operator");
  require(op.kind == PAFEM_DIFFUSION || op.kind == PAFEM_DIFFUSION_GEOM || op.kind == PAFEM_MASS,
          PAFEM_EINVAL, "smoothers need a mass or diffusion operator");
}

// degree steps of Chebyshev-Jacobi on A x = b; r, d, y: scratch vectors of n
void chebyshev(const Op& op, const double* diag, double lmax, double lo, double hi, int degree,
               const double* b, double* x, bool zero_guess, double* r, double* d, double* y,
               void* opwork, hipStream_t st) {
  const int64_t n = op.space->ndofs;
  if (degree <= 0) {
    if (zero_guess) launch_fill(x, 0.0, n, st);
    return;
  }
  const double theta = 0.5 * (hi + lo) * lmax, delta = 0.5 * (hi - lo) * lmax;
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (!zero_guess) apply_op(op, x, y, opwork, st);
  launch_cheb_start(b, zero_guess ? nullptr : y, diag, r, d, x, 1.0 / theta, zero_guess, n, st);
  for (int k = 1; k < degree; ++k) {
    apply_op(op, d, y, opwork, st);
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    launch_cheb_step(y, diag, r, d, x, rho_new * rho, 2.0 * rho_new / delta, n, st);
    rho = rho_new;
  }
}

void check_cheb_params(double lmax, double lo, double hi, int degree) {
  require(std::isfinite(lmax) && lmax > 0.0, PAFEM_EINVAL, "lmax must be positive");
  require(lo >= 0.0 && hi > lo && std::isfinite(hi), PAFEM_EINVAL,
          "Chebyshev interval needs 0 <= lo < hi");
  require(degree >= 0 && degree <= 64, PAFEM_EINVAL, "Chebyshev degree must be in [0, 64]");
}

// ---- V-cycle workspace --------------------------------------------------------------

struct LevelBufs {
  double *b = nullptr, *x = nullptr, *y = nullptr, *r = nullptr, *d = nullptr;
};

struct VLayout {
  std::vector<size_t> b, x, y, r, d;
  size_t state = 0, partials = 0, hist = 0, dotp = 0, opwork = 0, total = 0;
};

VLayout vcycle_layout(const PMG& g, size_t base) {
  VLayout L;
  size_t o = base;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  size_t opw = 0;
  for (int l = 0; l < g.L; ++l) {
    const size_t n = size_t(g.ops[size_t(l)]->space->ndofs) * 8;
    L.b.push_back(l == 0 ? 0 : take(n));
    L.x.push_back(l == 0 ? 0 : take(n));
    L.y.push_back(take(n));
    L.r.push_back(take(n));
    L.d.push_back(take(n));
    opw = std::max(opw, op_work_bytes(*g.ops[size_t(l)]));
  }
  const Op& c = *g.ops[size_t(g.L - 1)];
  L.state = take(sizeof(CGState));
  L.partials = take(3 * kCGBlocks * sizeof(double));
  L.hist = take((size_t(std::max(0, g.o.coarse_iters)) + 1) * sizeof(double));
  L.dotp = take(size_t(pa_apply_blocks(c.space->dev)) * sizeof(double));
  L.opwork = take(opw);
  L.total = o;
  return L;
}

struct VBufs {
  std::vector<LevelBufs> lv;
  CGState* state;
  double *partials, *hist, *dotp;
  void* opwork;
};

VBufs vcycle_bufs(const PMG& g, const VLayout& L, char* w) {
  VBufs B;
  for (int l = 0; l < g.L; ++l) {
    LevelBufs b;
    if (l > 0) {
      b.b = reinterpret_cast<double*>(w + L.b[size_t(l)]);
      b.x = reinterpret_cast<double*>(w + L.x[size_t(l)]);
    }
    b.y = reinterpret_cast<double*>(w + L.y[size_t(l)]);
    b.r = reinterpret_cast<double*>(w + L.r[size_t(l)]);
    b.d = reinterpret_cast<double*>(w + L.d[size_t(l)]);
    B.lv.push_back(b);
  }
  B.state = reinterpret_cast<CGState*>(w + L.state);
  B.partials = reinterpret_cast<double*>(w + L.partials);
  B.hist = reinterpret_cast<double*>(w + L.hist);
  B.dotp = reinterpret_cast<double*>(w + L.dotp);
  B.opwork = w + L.opwork;
  return B;
}

// Jacobi-PCG from zero with a fixed iteration count (stops early only on an exact
// zero residual or a breakdown): r, d, q are the level's r, d, y
void coarse_pcg(const PMG& g, const double* b, double* x, VBufs& B, hipStream_t st) {
  const int l = g.L - 1;
  const Op& op = *g.ops[size_t(l)];
  const double* diag = g.diag[size_t(l)];
  const int64_t n = op.space->ndofs;
  const int iters = std::max(0, g.o.coarse_iters);
  LevelBufs& v = B.lv[size_t(l)];
  const int nap = pa_apply_blocks(op.space->dev);
  const uint8_t* ess = (op.flags & PAFEM_OP_CONSTRAINED) ? op.space->dev.bmask : nullptr;
  launch_cg_reset(B.state, iters + 1, st);
  launch_cg_init<double, double>(B.state, B.partials, b, 1.0, nullptr, diag, x, v.r, v.d, 1, 0.0,
                                 B.hist, n, st);
  for (int k = 0; k < iters; ++k) {
    apply_op(op, v.d, v.y, B.opwork, st, B.dotp);
    launch_cg_alpha<double>(B.state, B.partials, B.dotp, nap, ess, v.d, n, st);
    launch_cg_update<double>(B.state, B.partials, x, v.r, v.d, v.y, diag, B.hist, n, st);
    launch_cg_direction<double>(B.state, v.r, diag, v.d, n, st);
  }
}

void vcycle(const PMG& g, int l, const double* b, double* x, VBufs& B, hipStream_t st) {
  if (l == g.L - 1) {
    coarse_pcg(g, b, x, B, st);
    return;
  }
  const Op& op = *g.ops[size_t(l)];
  const double* diag = g.diag[size_t(l)];
  LevelBufs& v = B.lv[size_t(l)];
  LevelBufs& c = B.lv[size_t(l + 1)];
  const DevSpace& fs = op.space->dev;
  const DevSpace& cs = g.ops[size_t(l + 1)]->space->dev;
  chebyshev(op, diag, g.lmax[size_t(l)], g.o.lo, g.o.hi, g.o.degree, b, x, true, v.r, v.d, v.y,
            B.opwork, st);
  apply_op(op, x, v.y, B.opwork, st);
  launch_restrict(fs, cs, g.interp[size_t(l)], b, v.y, c.b, st);
  vcycle(g, l + 1, c.b, c.x, B, st);
  launch_prolongate(cs, fs, g.interp[size_t(l)], c.x, x, true, st);
  chebyshev(op, diag, g.lmax[size_t(l)], g.o.lo, g.o.hi, g.o.degree, b, x, false, v.r, v.d, v.y,
            B.opwork, st);
}

struct FLayout {
  size_t state, partials, hist, r, z, zold, p, q, dotp, total;
};

FLayout fcg_layout_mg(const Op& op, int max_iter) {
  const size_t n = size_t(op.space->ndofs);
  FLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.state = take(sizeof(CGState));
  L.partials = take(3 * kCGBlocks * sizeof(double));
  L.hist = take((size_t(std::max(0, max_iter)) + 1) * sizeof(double));
  L.r = take(n * 8);
  L.z = take(n * 8);
  L.zold = take(n * 8);
  L.p = take(n * 8);
  L.q = take(n * 8);
  L.dotp = take(size_t(pa_apply_blocks(op.space->dev)) * sizeof(double));
  L.total = o;
  return L;
}

}  // namespace
}  // namespace pafem

struct pafem_pmg_s {
  pafem::PMG g;
};

extern "C" {

pafem_status pafem_coeff_element_mean(pafem_space space, int32_t kind, const double* coeff,
                                      int32_t q1d_in, int32_t q1d_out, double* out,
                                      void* stream) {
  return guarded([&] {
    const Space& s = uploaded(space);
    require(coeff && out, PAFEM_EINVAL, "null pointer argument");
    require(s.dim == 3, PAFEM_EUNSUPPORTED, "element means are built for hexahedra");
    require(kind == PAFEM_MEAN_ARITHMETIC || kind == PAFEM_MEAN_GEOMETRIC ||
                kind == PAFEM_MEAN_HARMONIC,
            PAFEM_EINVAL, "unknown mean");
    require(q1d_in >= 1 && q1d_in <= kMaxQ1d && q1d_out >= 1 && q1d_out <= kMaxQ1d, PAFEM_EINVAL,
            "q1d out of range");
    launch_coeff_mean(coeff, s.ne, q1d_in * q1d_in * q1d_in, q1d_out * q1d_out * q1d_out, kind,
                      out, static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_coeff_parent_mean(pafem_space fine, pafem_space coarse, int32_t kind,
                                     const double* coeff, int32_t q1d_in, int32_t q1d_out,
                                     double* out, void* stream) {
  return guarded([&] {
    const Space& f = uploaded(fine);
    const Space& c = uploaded(coarse);
    require(coeff && out, PAFEM_EINVAL, "null pointer argument");
    require(c.dim == 3 && f.dim == 3, PAFEM_EUNSUPPORTED, "element means are built for hexahedra");
    require(f.mesh->parent_id != 0 && f.mesh->parent_id == c.mesh->id, PAFEM_EINVAL,
            "the fine space's mesh is not a refinement of the coarse space's mesh");
    require(kind == PAFEM_MEAN_ARITHMETIC || kind == PAFEM_MEAN_GEOMETRIC ||
                kind == PAFEM_MEAN_HARMONIC,
            PAFEM_EINVAL, "unknown mean");
    require(q1d_in >= 1 && q1d_in <= kMaxQ1d && q1d_out >= 1 && q1d_out <= kMaxQ1d, PAFEM_EINVAL,
            "q1d out of range");
    // children 8 e .. 8 e + 7 of coarse element e are contiguous in the caller order
    launch_coeff_mean(coeff, c.ne, 8 * q1d_in * q1d_in * q1d_in, q1d_out * q1d_out * q1d_out,
                      kind, out, static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_prolongate(pafem_space coarse, pafem_space fine, const double* xc, double* yf,
                              int32_t add, void* stream) {
  return guarded([&] {
    const Space& c = uploaded(coarse);
    const Space& f = uploaded(fine);
    require(xc && yf, PAFEM_EINVAL, "null pointer argument");
    const bool h = check_pair(c, f);
    launch_prolongate(c.dev, f.dev, make_interp(c.p, f.p, h), xc, yf, add != 0,
                      static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_restrict(pafem_space fine, pafem_space coarse, const double* bf,
                            const double* yf, double* rc, void* stream) {
  return guarded([&] {
    const Space& c = uploaded(coarse);
    const Space& f = uploaded(fine);
    require(bf && rc, PAFEM_EINVAL, "null pointer argument");
    const bool h = check_pair(c, f);
    launch_restrict(f.dev, c.dev, make_interp(c.p, f.p, h), bf, yf, rc,
                    static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_smoother_workspace_bytes(pafem_op op, size_t* nbytes) {
  return guarded([&] {
    require(op && nbytes, PAFEM_EINVAL, "null pointer argument");
    *nbytes = smoother_layout(op->op).total;
  });
}

pafem_status pafem_op_lambda_max(pafem_op op, const double* diag, double* v, int32_t iters,
                                 void* work, size_t work_bytes, double* lambda, void* stream) {
  return guarded([&] {
    require(op && diag && v && work && lambda, PAFEM_EINVAL, "null pointer argument");
    const Op& o = op->op;
    check_smoother_op(o);
    require(iters >= 1, PAFEM_EINVAL, "power iteration needs iters >= 1");
    const SmootherLayout L = smoother_layout(o);
    require(work_bytes >= L.total, PAFEM_ESHAPE,
            "workspace too small: need " + std::to_string(L.total));
    auto st = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(work);
    double* wv = reinterpret_cast<double*>(w + L.y);
    double* partials = reinterpret_cast<double*>(w + L.partials);
    double* scal = reinterpret_cast<double*>(w + L.scal);
    double* lam = scal + 1;
    auto* ticket = reinterpret_cast<uint32_t*>(scal + 2);
    const int64_t n = o.space->ndofs;
    const uint8_t* ess = (o.flags & PAFEM_OP_CONSTRAINED) ? o.space->dev.bmask : nullptr;
    // the reduction ticket is cleared by a kernel rather than a memset; the call as a
    // whole is synchronous (it reads lambda back), so it cannot be captured in a graph
    launch_fill(reinterpret_cast<double*>(scal + 2), 0.0, 1, st);
    launch_power_norm(v, diag, ess, partials, ticket, scal, n, st);
    for (int k = 0; k < iters; ++k) {
      apply_op(o, v, wv, w + L.opwork, st);
      launch_power_step(v, wv, diag, partials, ticket, scal, lam, n, st);
    }
    hip_check(hipMemcpyAsync(lambda, lam, sizeof(double), hipMemcpyDeviceToHost, st), "read");
    hip_check(hipStreamSynchronize(st), "power iteration sync");
  });
}

pafem_status pafem_chebyshev_smooth(pafem_op op, const double* diag, double lmax, double lo,
                                    double hi, int32_t degree, const double* b, double* x,
                                    int32_t zero_guess, void* work, size_t work_bytes,
                                    void* stream) {
  return guarded([&] {
    require(op && diag && b && x && work, PAFEM_EINVAL, "null pointer argument");
    const Op& o = op->op;
    check_smoother_op(o);
    check_cheb_params(lmax, lo, hi, degree);
    const SmootherLayout L = smoother_layout(o);
    require(work_bytes >= L.total, PAFEM_ESHAPE,
            "workspace too small: need " + std::to_string(L.total));
    char* w = static_cast<char*>(work);
    chebyshev(o, diag, lmax, lo, hi, degree, b, x, zero_guess != 0,
              reinterpret_cast<double*>(w + L.r), reinterpret_cast<double*>(w + L.d),
              reinterpret_cast<double*>(w + L.y), w + L.opwork, static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_pmg_create(int32_t nlevels, const pafem_op* ops, const double* const* diags,
                              const double* lmax, const pafem_pmg_opts* opts, pafem_pmg* out) {
  return guarded([&] {
    require(ops && diags && lmax && opts && out, PAFEM_EINVAL, "null pointer argument");
    require(nlevels >= 1 && nlevels <= 16, PAFEM_EINVAL, "nlevels must be in [1, 16]");
    check_cheb_params(1.0, opts->lo, opts->hi, opts->degree);
    require(opts->coarse_iters >= 0 && opts->coarse_iters <= 100000, PAFEM_EINVAL,
            "coarse_iters out of range");
    PMG g;
    g.L = nlevels;
    g.o = *opts;
    for (int l = 0; l < nlevels; ++l) {
      require(ops[l] != nullptr && diags[l] != nullptr, PAFEM_EINVAL, "null level");
      const Op& o = ops[l]->op;
      require(o.qdtype == PAFEM_F64 &&
                  (o.kind == PAFEM_DIFFUSION || o.kind == PAFEM_DIFFUSION_GEOM),
              PAFEM_EUNSUPPORTED, "levels must be f64 diffusion operators");
      require(o.flags & PAFEM_OP_CONSTRAINED, PAFEM_EINVAL, "levels must be constrained");
      require(!(o.flags & PAFEM_OP_VECTOR3), PAFEM_EUNSUPPORTED, "levels must be scalar operators");
      require(o.space->dim == 3, PAFEM_EUNSUPPORTED, "order multigrid is built for hexahedra");
      require(std::isfinite(lmax[l]) && lmax[l] > 0.0, PAFEM_EINVAL, "lmax must be positive");
      g.ops.push_back(&o);
      g.diag.push_back(diags[l]);
      g.lmax.push_back(lmax[l]);
      if (l > 0) {
        const bool h = check_pair(*o.space, *g.ops[size_t(l - 1)]->space);
        g.interp.push_back(make_interp(o.space->p, g.ops[size_t(l - 1)]->space->p, h));
      }
    }
    *out = new pafem_pmg_s{std::move(g)};
  });
}

void pafem_pmg_destroy(pafem_pmg pmg) { delete pmg; }

pafem_status pafem_pmg_workspace_bytes(pafem_pmg pmg, int32_t max_iter, size_t* nbytes) {
  return guarded([&] {
    require(pmg && nbytes, PAFEM_EINVAL, "null pointer argument");
    const size_t base = max_iter < 0 ? 0 : fcg_layout_mg(*pmg->g.ops[0], max_iter).total;
    *nbytes = vcycle_layout(pmg->g, base).total;
  });
}

pafem_status pafem_pmg_vcycle(pafem_pmg pmg, const double* r, double* z, void* work,
                              size_t work_bytes, void* stream) {
  return guarded([&] {
    require(pmg && r && z && work, PAFEM_EINVAL, "null pointer argument");
    const PMG& g = pmg->g;
    const VLayout L = vcycle_layout(g, 0);
    require(work_bytes >= L.total, PAFEM_ESHAPE,
            "workspace too small: need " + std::to_string(L.total));
    VBufs B = vcycle_bufs(g, L, static_cast<char*>(work));
    vcycle(g, 0, r, z, B, static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_pmg_fcg_solve(pafem_pmg pmg, const double* b, double* x, void* work,
                                 size_t work_bytes, const pafem_solve_opts* opts,
                                 pafem_solve_result* result, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  pafem_status status = PAFEM_OK;
  pafem_status rc = guarded([&] {
    require(pmg && b && x && work && opts && result, PAFEM_EINVAL, "null pointer argument");
    require(opts->max_iter >= 0 && opts->rel_tol >= 0.0, PAFEM_EINVAL, "bad solver options");
    const PMG& g = pmg->g;
    const Op& op = *g.ops[0];
    const FLayout F = fcg_layout_mg(op, opts->max_iter);
    const VLayout V = vcycle_layout(g, F.total);
    require(work_bytes >= V.total, PAFEM_ESHAPE,
            "workspace too small: need " + std::to_string(V.total));
    char* w = static_cast<char*>(work);
    VBufs B = vcycle_bufs(g, V, w);
    auto* state = reinterpret_cast<CGState*>(w + F.state);
    auto* partials = reinterpret_cast<double*>(w + F.partials);
    auto* hist = reinterpret_cast<double*>(w + F.hist);
    auto* r = reinterpret_cast<double*>(w + F.r);
    auto* z = reinterpret_cast<double*>(w + F.z);
    auto* zold = reinterpret_cast<double*>(w + F.zold);
    auto* p = reinterpret_cast<double*>(w + F.p);
    auto* q = reinterpret_cast<double*>(w + F.q);
    auto* dotp = reinterpret_cast<double*>(w + F.dotp);
    const DevSpace& sp = op.space->dev;
    const int64_t n = sp.ndofs;
    const int nap = pa_apply_blocks(sp);
    const uint8_t* ess = sp.bmask;
    auto st = static_cast<hipStream_t>(stream);

    launch_cg_reset(state, opts->max_iter + 1, st);
    if (!opts->zero_guess) apply_op(op, x, q, B.opwork, st);
    launch_fcg_init(state, partials, b, opts->zero_guess ? nullptr : q, x, r, opts->zero_guess,
                    opts->rel_tol, hist, n, st);
    vcycle(g, 0, r, z, B, st);
    launch_fcg_start(state, partials, r, z, p, n, st);
    // one iteration: the new preconditioned residual goes to zn, zc holds the current one
    auto iteration = [&](hipStream_t s2, double* zc, double* zn) {
      apply_op(op, p, q, B.opwork, s2, dotp);
      launch_cg_alpha<double>(state, partials, dotp, nap, ess, p, n, s2);
      launch_fcg_update(state, partials, x, r, p, q, g.diag[0], ess, zn, hist, n, s2);
      vcycle(g, 0, r, zn, B, s2);
      launch_fcg_beta(state, partials, r, zn, zc, n, s2);
      launch_fcg_direction(state, zn, p, n, s2);
    };
    const bool graphs = graphs_enabled();
    int check = std::max(1, opts->check_every);
    if (graphs) check += check & 1;  // whole pairs of iterations per host check
    CapturedGraph pair;               // two iterations, z -> zold -> z
    int launched = 0;
    CGState h{};
    while (true) {
      hip_check(hipMemcpyAsync(&h, state, sizeof(CGState), hipMemcpyDeviceToHost, st), "state");
      hip_check(hipStreamSynchronize(st), "fcg sync");
      if (h.done != 0 || launched >= opts->max_iter || h.iter >= opts->max_iter) break;
      const int batch = std::min(check, opts->max_iter - launched);
      int k = 0;
      if (graphs && batch >= 2) {
        if (!pair.ready())
          pair.capture([&](hipStream_t cs) {
            iteration(cs, z, zold);
            iteration(cs, zold, z);
          });
        for (; k + 2 <= batch; k += 2) pair.launch(st);
      }
      for (; k < batch; ++k) {  // only the last batch can be odd
        iteration(st, z, zold);
        std::swap(z, zold);
      }
      launched += batch;
    }
    apply_op(op, x, q, B.opwork, st);
    launch_residual(state, partials, b, q, nullptr, n, st);
    hip_check(hipMemcpyAsync(&h, state, sizeof(CGState), hipMemcpyDeviceToHost, st), "state");
    hip_check(hipStreamSynchronize(st), "fcg sync");
    result->iters = h.iter;
    result->converged = h.done == 1;
    result->rel_res = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    result->true_rel_res = h.bb > 0 ? std::sqrt(h.res2 / h.bb) : 0.0;
    if (opts->res_hist && opts->res_hist_cap > 0) {
      const int nh = std::min(opts->res_hist_cap, h.iter + 1);
      hip_check(hipMemcpy(opts->res_hist, hist, size_t(nh) * sizeof(double),
                          hipMemcpyDeviceToHost), "history read");
    }
    if (h.done == 2 || h.done == 3)
      status = fail(PAFEM_EBREAKDOWN, "FCG breakdown at iteration " + std::to_string(h.iter));
    else if (h.done != 1)
      status = fail(PAFEM_ENOTCONV, "FCG did not converge in " + std::to_string(h.iter) +
                                        " iterations");
  });
  if (result)
    result->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc != PAFEM_OK ? rc : status;
}

}  // extern "C"
