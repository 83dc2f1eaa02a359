// Batched multi-right-hand-side apply over many meshes: device descriptors and
// launchers (k_batch.hip), used by the host batch object (batch.cpp).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "internal.hpp"

namespace pafem {

// One mesh of a batch, as the kernels see it.
struct BatchMesh {
  const int32_t* gmap;   // device-order element->dof map, ~g on essential dofs
  const uint8_t* bmask;  // essential-dof mask
  const void* qdata;     // tile-interleaved quadrature data
  const void* x;         // [ndofs][nrhs]
  void* y;               // [ndofs][nrhs]
  int32_t ne, ndofs;
  int32_t block_begin;   // first workgroup of this mesh within its order's launch
  int32_t constrained;
};

// candidates 0..4: vector-unit tiles (k_batch.hip); 5: FP64 matrix cores, one element x
// 16 right-hand sides per workgroup (k_batch_mfma.hip), orders 1..4
constexpr int kBatchCandidates = 6;
constexpr int kBatchMfmaCandidate = 5;
int batch_tile_elems(int cand);
int batch_tile_rhs(int cand);
// Launches the multi-rhs apply of one order group; false if the (order,
// candidate, dtype) combination is not built.
// tabB: the order's 1D B table followed by its G table, in the vector dtype
bool launch_batch_apply(int p, int cand, int vdtype, int qdtype, int kind,
                        const BatchMesh* meshes, int nmesh, int nblocks, const void* tabB,
                        int nrhs, hipStream_t st);
void launch_batch_init(int vdtype, const BatchMesh* meshes, int nmesh, int nrhs, hipStream_t st);
// the matrix-core variant (FP64, orders 1..4, nrhs a multiple of 16); false otherwise
bool launch_batch_apply_mfma(int p, int kind, const BatchMesh* meshes, int nmesh, int nblocks,
                             const double* tabB, int nrhs, hipStream_t st);

}  // namespace pafem
