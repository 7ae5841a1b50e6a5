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

// Agent-scope relaxed loads and stores (no fences).  They bypass the caches
// that are not coherent across the chip (global_load/store with sc1), so a
// value handed from one workgroup of a running kernel to another is seen
// without cache maintenance: the writer stores with st_agent, waits for its
// stores (wait_vm), then raises a flag; the reader polls the flag and then
// loads with ld_agent.  A release or acquire fence would instead write back
// or invalidate a whole L2 at every hand-over.
template <int L>
__device__ __forceinline__ void ld_agent(const double *base, size_t stride, size_t q, double (&v)[L]) {
#pragma unroll
  for (int l = 0; l < L; ++l) v[l] = __hip_atomic_load(base + (size_t)l * stride + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int L>
__device__ __forceinline__ void st_agent(double *base, size_t stride, size_t q, const double (&v)[L]) {
#pragma unroll
  for (int l = 0; l < L; ++l) __hip_atomic_store(base + (size_t)l * stride + q, v[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until this wave's outstanding memory operations have completed (for
// agent-scope stores: performed at the agent's coherence point).
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0); }

// Order this wave's LDS and global memory operations (all lanes of a worker
// group live in one wavefront, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Lane exchange by a DPP move (data-parallel primitive: a VALU operand
// permutation, no LDS round trip) of both halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// DPP controls: quad permutations [1,0,3,2] (xor 1) and [2,3,0,1] (xor 2),
// half-row mirror (lane i <-> 7-i in a group of 8), row mirror (i <-> 15-i in
// a row of 16).
enum : int { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140 };

template <int L, int CTRL>
__device__ __forceinline__ void team_step_dpp(double (&v)[L]) {
  double o[L], s[L];
#pragma unroll
  for (int l = 0; l < L; ++l) o[l] = dpp_f64<CTRL>(v[l]);
  MD<L>::add(v, o, s);
  md::copy<L>(s, v);
}

template <int L>
__device__ __forceinline__ void team_step_xor(double (&v)[L], int off) {
  double o[L], s[L];
#pragma unroll
  for (int l = 0; l < L; ++l) o[l] = __shfl_xor(v[l], off, 64);
  MD<L>::add(v, o, s);
  md::copy<L>(s, v);
}

template <int L, int CTRL>
__device__ __forceinline__ void team_step_dpp_lazy(double (&u)[L]) {
  double o[L];
#pragma unroll
  for (int l = 0; l < L; ++l) o[l] = dpp_f64<CTRL>(u[l]);
  MD<L>::add_lazy(u, o);
}

template <int L>
__device__ __forceinline__ void team_step_xor_lazy(double (&u)[L], int off) {
  double o[L];
#pragma unroll
  for (int l = 0; l < L; ++l) o[l] = __shfl_xor(u[l], off, 64);
  MD<L>::add_lazy(u, o);
}

// The same butterfly on accumulators of level sums (the state of
// MD<L>::fma_lazy; a renormalized md number is one too): each level adds
// two accumulators without renormalizing, and the caller renormalizes the
// total once (MD<L>::renorm).  For quad doubles a level costs 40
// instructions instead of the 73 of a renormalized addition.
template <int L>
__device__ __forceinline__ void team_sum_lazy(double (&u)[L], int width) {
  if (width >= 2) team_step_dpp_lazy<L, DPP_XOR1>(u);
  if (width >= 4) team_step_dpp_lazy<L, DPP_XOR2>(u);
  if (width >= 8) team_step_dpp_lazy<L, DPP_HALF_MIRROR>(u);
  if (width >= 16) team_step_dpp_lazy<L, DPP_MIRROR>(u);
  if (width >= 32) team_step_xor_lazy<L>(u, 16);
  if (width >= 64) team_step_xor_lazy<L>(u, 32);
}

// Sum of an md value over `width` consecutive lanes (width a power of two <=
// 64, teams aligned to their width), result in every lane of the team.  The
// first four levels stay inside a row of 16 lanes and use DPP: exchanges
// xor 1 and xor 2, then the two mirrors, which pair each lane with one in the
// other half of its group of 8 (16); the partial sums are uniform over each
// half by then, so that pairing completes the sum of the group.  Levels 16
// and 32 cross rows and use the LDS permute.  All lanes of a team must be
// active.
template <int L>
__device__ __forceinline__ void team_sum(double (&v)[L], int width) {
  if (width >= 2) team_step_dpp<L, DPP_XOR1>(v);
  if (width >= 4) team_step_dpp<L, DPP_XOR2>(v);
  if (width >= 8) team_step_dpp<L, DPP_HALF_MIRROR>(v);
  if (width >= 16) team_step_dpp<L, DPP_MIRROR>(v);
  if (width >= 32) team_step_xor<L>(v, 16);
  if (width >= 64) team_step_xor<L>(v, 32);
}

// Record a device-side condition; the first error wins.
__device__ __forceinline__ void set_status(int32_t *status, int32_t code) {
  if (status) atomicCAS(status, 0, code);
}

// One thread waits until *ctr >= target, a count that workgroups of a
// launch on another stream raise once their agent-scope stores are
// performed.  Bounded: false (and MD_EHIP in status) when it runs out.
__device__ __forceinline__ bool wait_count(const int *ctr, int target, int32_t *status) {
  long spins = 0;
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(2);
    if (++spins > (1L << 22)) {
      set_status(status, MD_EHIP);
      return false;
    }
  }
  return true;
}

// Dispatch a launch on the limb count: the statement sees LL as a constant.
#define MD_DISPATCH(L, ...)                                 \
  switch (L) {                                              \
    case 1: { constexpr int LL = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int LL = 2; __VA_ARGS__; } break; \
    case 4: { constexpr int LL = 4; __VA_ARGS__; } break; \
    case 8: { constexpr int LL = 8; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                   \
  }

}  // namespace mdk
