// Shared device helpers: status codes, limb-major loads and stores, wave
// reductions.  All multiple-double arrays are limb-major ("structure of
// arrays by limb", Section 1.2): limb l of element q of an array with
// `stride` elements per limb is at base[l * stride + q].
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include "md.hpp"
#include "../../include/mdnewton.h"

namespace mdk {

using md::MD;

template <int L>
__device__ __forceinline__ void ld(const double *base, size_t stride, size_t q, double (&v)[L]) {
#pragma unroll
  for (int l = 0; l < L; ++l) v[l] = base[(size_t)l * stride + q];
}

template <int L>
__device__ __forceinline__ void st(double *base, size_t stride, size_t q, const double (&v)[L]) {
#pragma unroll
  for (int l = 0; l < L; ++l) base[(size_t)l * stride + q] = v[l];
}

// Order this wave's LDS and global memory operations (all lanes of a worker
// group live in one wavefront, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Sum of an md value over `width` consecutive lanes (width a power of two <= 64),
// butterfly order, result in every lane of the team.
template <int L>
__device__ __forceinline__ void team_sum(double (&v)[L], int width) {
  for (int off = width >> 1; off > 0; off >>= 1) {
    double o[L], s[L];
#pragma unroll
    for (int l = 0; l < L; ++l) o[l] = __shfl_xor(v[l], off, 64);
    MD<L>::add(v, o, s);
    md::copy<L>(s, v);
  }
}

// Record a device-side condition; the first error wins.
__device__ __forceinline__ void set_status(int32_t *status, int32_t code) {
  if (status) atomicCAS(status, 0, code);
}

}  // namespace mdk
