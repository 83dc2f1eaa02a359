// Device-side helpers for gfx950 (CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pafem {

constexpr int kWave = 64;
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, one L2 each

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD b % 8).
// Remap so that each XCD works on one contiguous range of tiles: neighbouring
// element tiles share dofs, and keeping them on one die keeps the shared x/y
// lines in one L2.  Bijective for any grid size.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int xcd = bid % kNumXcd, idx = bid / kNumXcd;
  const int base = nblocks / kNumXcd, rem = nblocks % kNumXcd;
  return xcd * base + min(xcd, rem) + idx;
}

// p itself, but opaque to the optimizer: loads through the result are issued after
// this point and are not merged with loads through other copies of p.  Applied per loop
// iteration to a uniform table pointer, it keeps the iteration's table entries in
// scalar registers for that iteration only, instead of every entry of an unrolled loop
// nest being loaded up front and spilled (p >= 6 tables exceed the scalar registers).
// The result points into the constant address space (read-only for the kernel's
// lifetime), so the loads stay scalar.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ const_ptr<T> opaque_ptr(const T* p) {
  // the address is uniform; readfirstlane states so where the compiler cannot see it
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
  uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
  __asm__ volatile("" : "+s"(lo), "+s"(hi));
  return reinterpret_cast<const_ptr<T>>((uint64_t(hi) << 32) | lo);
}

// bfloat16 storage as raw 16-bit patterns (round-to-nearest-even on conversion).
struct bf16 {
  uint16_t bits;
};
__device__ __host__ __forceinline__ float bf16_to_float(bf16 h) {
  union {
    uint32_t u;
    float f;
  } v;
  v.u = uint32_t(h.bits) << 16;
  return v.f;
}

template <typename TC, typename TD>
__device__ __forceinline__ TC load_value(const TD* p) {
  return TC(__builtin_nontemporal_load(p));
}
template <>
__device__ __forceinline__ float load_value<float, bf16>(const bf16* p) {
  const uint16_t raw = __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p));
  return bf16_to_float(bf16{raw});
}

// Two adjacent stored values (components 2k and 2k+1 of one quadrature point in the
// paired diffusion layout) with one non-temporal load: 16 bytes per lane in FP64.
typedef double pafem_d2 __attribute__((ext_vector_type(2)));
typedef float pafem_f2 __attribute__((ext_vector_type(2)));
template <typename TC, typename TD>
__device__ __forceinline__ void load_pair(const TD* p, TC& a, TC& b);
template <>
__device__ __forceinline__ void load_pair<double, double>(const double* p, double& a, double& b) {
  const pafem_d2 v = __builtin_nontemporal_load(reinterpret_cast<const pafem_d2*>(p));
  a = v.x;
  b = v.y;
}
template <>
__device__ __forceinline__ void load_pair<float, float>(const float* p, float& a, float& b) {
  const pafem_f2 v = __builtin_nontemporal_load(reinterpret_cast<const pafem_f2*>(p));
  a = v.x;
  b = v.y;
}
template <>
__device__ __forceinline__ void load_pair<float, bf16>(const bf16* p, float& a, float& b) {
  const uint32_t raw = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
  a = bf16_to_float(bf16{uint16_t(raw & 0xffffu)});
  b = bf16_to_float(bf16{uint16_t(raw >> 16)});
}

// Sum over the 64 lanes of a wave (butterfly: every lane ends with the total,
// fixed association order, so results are reproducible run to run).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Deterministic block sum; `scratch` holds blockDim.x / 64 doubles in LDS.
// Returns the total in every thread.  Contains __syncthreads().
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum(v);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += scratch[w];
  __syncthreads();
  return t;
}

// ---- deterministic grid reductions -------------------------------------------
// Each block stores one partial per quantity; the last block to arrive (atomic
// ticket) sums all partials in index order.

__device__ __forceinline__ void store_partial(double* partials, double v) {
  __hip_atomic_store(&partials[blockIdx.x], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_partial(const double* partials, int i) {
  return __hip_atomic_load(const_cast<double*>(&partials[i]), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes this block's partials (thread 0 already stored them) and returns true in
// every thread of the last block to arrive.
__device__ inline bool arrive_last(uint32_t* ticket) {
  __shared__ int last;
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t t = atomicAdd(ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last != 0;
}

// Sum of partials[0..gridDim.x) in a fixed order, valid in every thread.
__device__ inline double sum_partials(const double* partials, double* scratch) {
  double v = 0.0;
  for (int i = threadIdx.x; i < int(gridDim.x); i += blockDim.x) v += load_partial(partials, i);
  return block_sum(v, scratch);
}

}  // namespace pafem
