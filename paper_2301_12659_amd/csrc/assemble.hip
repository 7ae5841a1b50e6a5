// Assembly of the residual and Jacobian series from the monomial values and
// derivative products (Section 2: b(t) = -p(x(t)), A(t) = p'(x(t))), in a
// fixed monomial order so that results are reproducible, with the size of the
// terms of each residual coefficient for the staggered method's stopping test
// (Section 4).
#include "common.hpp"
#include "kernels.hpp"
#include "md.hpp"

#include <algorithm>

namespace mdk {

// b_i(t) = -(c_{i,0}(t) + sum_{m in P_i} value_m(t)) for the first Dc
// coefficients s, four lanes per (i, s): lane j adds the constant (j = 0)
// and the values of monomials j, j + 4, ... of row i, in monomial order, with
// renormalized additions; a two-level butterfly of renormalized additions
// adds the four partial sums (a fixed order, reproducible).  A residual is a
// sum that cancels: level sums accumulated across the terms and renormalized
// once lose up to six times more against the size of the terms (exact
// rational checks on the host) and can leave overlapping limbs.  tsz (nullable, [n][D])
// gets the size of the terms whose rounding errors reach b_{i,s}, against
// which the staggered method judges it: |c_{i,0,s}| + sum_m vsize_{m,s}, the
// largest product of each monomial's chain (|value_{m,s}| when vsize is null;
// leading limbs).  rt (nullable): coefficient-major copy for the staged
// solve.  clear (nullable): clear_count ints set to zero on the way, and
// empty (nullable): empty_count hand-over slots emptied (the staged solve's
// counters and dx slots, for the solve the caller launches next on this
// stream).
template <int L>
__device__ __forceinline__ void assemble_b_block(unsigned bid, int n, int D, int Dc, int m, const int32_t *poly_ptr,
                                                 const double *cst, const double *val, double *b, double *tsz,
                                                 const double *vsize, TOut rt, int *clear, int clear_count,
                                                 double *empty, size_t empty_count) {
  const size_t t = (size_t)bid * blockDim.x + threadIdx.x;
  if (clear && t < (size_t)clear_count) clear[t] = 0;
  if (empty && t < empty_count) empty[t] = __longlong_as_double(SLOT_EMPTY);
  const size_t nD = (size_t)n * D, mD = (size_t)m * D;
  const size_t task = t >> 2;
  const int j = (int)(t & 3);
  const bool live = task < (size_t)n * Dc;
  const size_t tk = live ? task : 0;
  const int i = (int)(tk / Dc), s = (int)(tk - (size_t)i * Dc);
  const size_t q = (size_t)i * D + s;
  double r[L];
  md::zero<L>(r);
  double size = 0.0;
  if (live) {
    const int mend = poly_ptr[i + 1];
    bool have = j == 0;
    if (have) {
      ld<L>(cst, nD, q, r);
      size = fabs(r[0]);
    }
    // the lane's values in batches of four, each batch loaded before it is added
    for (int mb = poly_ptr[i] + j; mb < mend; mb += 16) {
      double v[4][L], sz[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int mj = mb + 4 * u;
        if (mj < mend) {
          ld<L>(val, mD, (size_t)mj * D + s, v[u]);
          sz[u] = vsize ? vsize[(size_t)mj * D + s] : fabs(v[u][0]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (mb + 4 * u < mend) {
          if (have) {
            double t[L];
            MD<L>::add(r, v[u], t);
            md::copy<L>(t, r);
            size += sz[u];
          } else {
            md::copy<L>(v[u], r);
            size = sz[u];
            have = true;
          }
        }
      }
    }
  }
  team_sum<L>(r, 4);
  const double s01 = size + __shfl_xor(size, 1, 64);
  size = s01 + __shfl_xor(s01, 2, 64);
  md::neg<L>(r, r);
  if (live && j == 0) {
    st<L>(b, nD, q, r);
    if (tsz) tsz[q] = size;
    if (rt.p && s >= rt.lo && s < rt.lo + rt.W) {
      const size_t ls = (size_t)n * rt.W;
      for (int l = 0; l < rt.L; ++l) rt.p[(size_t)l * ls + (size_t)(s - rt.lo) * n + i] = r[l];
    }
  }
}

template <int L>
__global__ void __launch_bounds__(256) assemble_b_kernel(int n, int D, int Dc, int m, const int32_t *poly_ptr,
                                                         const double *cst, const double *val, double *b, double *tsz,
                                                         const double *vsize, TOut rt, int *clear, int clear_count,
                                                         double *empty, size_t empty_count) {
  assemble_b_block<L>(blockIdx.x, n, D, Dc, m, poly_ptr, cst, val, b, tsz, vsize, rt, clear, clear_count, empty,
                      empty_count);
}

// A[i][j][s] = sum of the derivative series of row i's monomials with respect
// to x_j, in monomial order, for the first Dc coefficients s.  A workgroup
// takes TI consecutive (i, j) and all Dc coefficients (reads and the
// series-major writes along s); with at (nullable) the tile goes through LDS
// so that the coefficient-major copy at[l][s][i][j] (s < at.W, at.L limbs) is
// written along (i, j).
// Coefficients per thread of assemble_A_kernel: with the tiles of
// assemble_tile at most 8, 8, 4, 2 for 1, 2, 4, 8 limbs (MD_MAX_COEFFS = 128).
__host__ __device__ constexpr int asm_a_max_slices(int L) { return L >= 8 ? 2 : (L == 4 ? 4 : 8); }

// Entries of a Jacobian entry's list loaded together by the assemblies of A.
constexpr int ASM_BATCH = 4;

template <int L, int TI>
__device__ __forceinline__ void assemble_A_block(unsigned bid, int n, int D, int Dc, int nnz, const int32_t *asm_ptr,
                                                 const int32_t *asm_ent, const double *der, double *A, TOut at,
                                                 double *tile /* [L][TI][Dc + 1] */) {
  const size_t nn = (size_t)n * n, nnD = nn * D, zD = (size_t)nnz * D;
  const size_t ij0 = (size_t)bid * TI;
  const int Dp = Dc + 1;
  // blockDim / TI threads per (i, j), each the coefficients s = sl + u per,
  // u < NS (at most asm_a_max_slices(L)): the entry list is read once, and the
  // NS values of an entry are loaded together before they are added
  constexpr int MAXS = asm_a_max_slices(L);
  const int per = blockDim.x / TI, il = threadIdx.x / per, sl = threadIdx.x - il * per;
  const int NS = (Dc + per - 1) / per;
  const size_t ij = ij0 + il;
  if (ij < nn) {
    const int lo = asm_ptr[ij], hi = asm_ptr[ij + 1];
    double acc[MAXS][L];
#pragma unroll
    for (int u = 0; u < MAXS; ++u) md::zero<L>(acc[u]);
    // the list in batches of ASM_BATCH entries: a batch's indices, then all
    // its values, are loaded before its values are added in list order (two
    // memory round trips per batch instead of two per entry)
    for (int t0 = lo; t0 < hi; t0 += ASM_BATCH) {
      size_t eo[ASM_BATCH];
#pragma unroll
      for (int e = 0; e < ASM_BATCH; ++e) eo[e] = (t0 + e < hi) ? (size_t)asm_ent[t0 + e] * D : 0;
      double v[ASM_BATCH][MAXS][L];
#pragma unroll
      for (int e = 0; e < ASM_BATCH; ++e)
#pragma unroll
        for (int u = 0; u < MAXS; ++u) {
          const int s = sl + u * per;
          if (t0 + e < hi && u < NS && s < Dc) ld<L>(der, zD, eo[e] + s, v[e][u]);
        }
#pragma unroll
      for (int e = 0; e < ASM_BATCH; ++e)
#pragma unroll
        for (int u = 0; u < MAXS; ++u) {
          const int s = sl + u * per;
          if (t0 + e < hi && u < NS && s < Dc) {
            if (t0 + e == lo) {
              md::copy<L>(v[e][u], acc[u]);
            } else {
              double r[L];
              MD<L>::add(acc[u], v[e][u], r);
              md::copy<L>(r, acc[u]);
            }
          }
        }
    }
#pragma unroll
    for (int u = 0; u < MAXS; ++u) {
      const int s = sl + u * per;
      if (u < NS && s < Dc) {
        st<L>(A, nnD, ij * D + s, acc[u]);
        if (at.p)
#pragma unroll
          for (int l = 0; l < L; ++l) tile[(l * TI + il) * Dp + s] = acc[u][l];
      }
    }
  }
  if (!at.p) return;
  __syncthreads();
  const size_t ls = nn * at.W;
  for (int e = threadIdx.x; e < at.W * TI; e += blockDim.x) {
    const int s = e / TI, il = e - s * TI;
    const size_t ij = ij0 + il;
    if (ij >= nn) continue;
    for (int l = 0; l < at.L; ++l) at.p[(size_t)l * ls + (size_t)s * nn + ij] = tile[(l * TI + il) * Dp + s];
  }
}

template <int L, int TI>
__global__ void __launch_bounds__(256) assemble_A_kernel(int n, int D, int Dc, int nnz, const int32_t *asm_ptr,
                                                         const int32_t *asm_ent, const double *der, double *A,
                                                         TOut at) {
  extern __shared__ double tile[];
  assemble_A_block<L, TI>(blockIdx.x, n, D, Dc, nnz, asm_ptr, asm_ent, der, A, at, tile);
}

// Both assemblies in one launch: workgroups 0 .. GA - 1 form A (as
// assemble_A_kernel), the others b (as assemble_b_kernel); they read disjoint
// inputs and write disjoint outputs.  With wait.ctr, one thread of the first
// workgroup waits for the count after its part, so the launch ends only
// once the count is reached (a wait for another stream that costs no launch
// of its own).
template <int L, int TI>
__global__ void __launch_bounds__(256) assemble_bA_kernel(unsigned GA, int n, int D, int Dc, int m, int nnz,
                                                          const int32_t *poly_ptr, const int32_t *asm_ptr,
                                                          const int32_t *asm_ent, const double *cst,
                                                          const double *val, const double *der, double *b,
                                                          double *A, double *tsz, const double *vsize, TOut rt,
                                                          TOut at, int *clear, int clear_count, double *empty,
                                                          size_t empty_count, CountWait wait) {
  extern __shared__ double tile[];
  if (blockIdx.x < GA)
    assemble_A_block<L, TI>(blockIdx.x, n, D, Dc, nnz, asm_ptr, asm_ent, der, A, at, tile);
  else
    assemble_b_block<L>(blockIdx.x - GA, n, D, Dc, m, poly_ptr, cst, val, b, tsz, vsize, rt, clear, clear_count,
                        empty, empty_count);
  if (wait.ctr && blockIdx.x == 0 && threadIdx.x == 0) wait_count(wait.ctr, wait.target, wait.status);
}

// Coefficient 0 of A into a dense row-major matrix a0 [L][n][n], summed in
// the same order as assemble_A_kernel, so it equals A[i][j][0] bit for bit.
// prep: the hand-over memory of the LDS QR of a0, which follows on this
// stream (flags cleared, scalar slots emptied; none when its pointers are null).
template <int L>
__global__ void assemble_A0_kernel(int n, int D, int nnz, const int32_t *asm_ptr, const int32_t *asm_ent,
                                   const double *der, double *a0, QrPrep prep) {
  __builtin_amdgcn_s_setprio(3);  // on the factorization's chain, as the pre-pass
  const size_t ij = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  qr_prep_item(prep, ij);
  const size_t nn = (size_t)n * n, zD = (size_t)nnz * D;
  if (ij >= nn) return;
  const int lo = asm_ptr[ij], hi = asm_ptr[ij + 1];
  double acc[L];
  md::zero<L>(acc);
  // batches of ASM_BATCH entries, as in assemble_A_block
  for (int t0 = lo; t0 < hi; t0 += ASM_BATCH) {
    size_t eo[ASM_BATCH];
#pragma unroll
    for (int e = 0; e < ASM_BATCH; ++e) eo[e] = (t0 + e < hi) ? (size_t)asm_ent[t0 + e] * D : 0;
    double v[ASM_BATCH][L];
#pragma unroll
    for (int e = 0; e < ASM_BATCH; ++e)
      if (t0 + e < hi) ld<L>(der, zD, eo[e], v[e]);
#pragma unroll
    for (int e = 0; e < ASM_BATCH; ++e) {
      if (t0 + e >= hi) continue;
      if (t0 + e == lo) {
        md::copy<L>(v[e], acc);
      } else {
        double r[L];
        MD<L>::add(acc, v[e], r);
        md::copy<L>(r, acc);
      }
    }
  }
  st<L>(a0, nn, ij, acc);
}

// ------------------------------------------------------------------ launchers

hipError_t launch_assemble_A0(int L, int n, int D, int nnz, const int32_t *asm_ptr, const int32_t *asm_ent,
                              const double *der, double *a0, hipStream_t st, QrPrep prep) {
  const size_t nn = (size_t)n * n;
  const size_t threads = std::max({nn, (size_t)prep.n, (size_t)prep.nt});
  MD_DISPATCH(L, hipLaunchKernelGGL(assemble_A0_kernel<LL>, dim3((threads + 63) / 64), dim3(64), 0, st, n, D, nnz,
                                    asm_ptr, asm_ent, der, a0, prep));
  return hipGetLastError();
}

hipError_t launch_assemble_b(int L, int n, int D, int Dc, int m, const int32_t *poly_ptr, const double *cst,
                             const double *val, double *b, hipStream_t st, double *tsz, const double *vsize,
                             TOut rt, int *clear, int clear_count, double *empty, size_t empty_count) {
  if (Dc < 1 || Dc > D) return hipErrorInvalidValue;
  if (rt.p && (rt.lo < 0 || rt.W < 1 || rt.lo + rt.W > Dc || rt.L < 1 || rt.L > L)) return hipErrorInvalidValue;
  const size_t threads = std::max({(size_t)n * Dc * 4, (size_t)(clear ? clear_count : 0), empty ? empty_count : 0});
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  MD_DISPATCH(L, hipLaunchKernelGGL(assemble_b_kernel<LL>, dim3(blocks), dim3(256), 0, st, n, D, Dc, m, poly_ptr,
                                    cst, val, b, tsz, vsize, rt, clear, clear_count, empty, empty_count));
  return hipGetLastError();
}

// Rows (i, j) per workgroup of assemble_A_kernel: 16 while the LDS tile stays
// within 48 KB and a thread has at most asm_a_max_slices(L) coefficients,
// else fewer.
static int assemble_tile(int L, int Dc) {
  int ti = 16;
  while (ti > 1 && ((size_t)ti * (Dc + 1) * L * sizeof(double) > 48 * 1024 ||
                    (Dc + 256 / ti - 1) / (256 / ti) > asm_a_max_slices(L)))
    ti /= 2;
  return ti;
}

hipError_t launch_assemble_A(int L, int n, int D, int Dc, int nnz, const int32_t *asm_ptr, const int32_t *asm_ent,
                             const double *der, double *A, hipStream_t st, TOut at) {
  if (Dc < 1 || Dc > D) return hipErrorInvalidValue;
  if (at.p && (at.lo != 0 || at.W < 1 || at.W > Dc || at.L < 1 || at.L > L)) return hipErrorInvalidValue;
  const size_t nn = (size_t)n * n;
  const int ti = assemble_tile(L, Dc);
  if ((Dc + 256 / ti - 1) / (256 / ti) > asm_a_max_slices(L)) return hipErrorInvalidValue;
  const size_t lds = at.p ? (size_t)ti * (Dc + 1) * L * sizeof(double) : 0;
  const dim3 grid((unsigned)((nn + ti - 1) / ti));
#define MD_ASM_A(TI)                                                                                            \
  MD_DISPATCH(L, hipLaunchKernelGGL((assemble_A_kernel<LL, TI>), grid, dim3(256), lds, st, n, D, Dc, nnz, asm_ptr, \
                                    asm_ent, der, A, at))
  switch (ti) {
    case 16: MD_ASM_A(16); break;
    case 8: MD_ASM_A(8); break;
    case 4: MD_ASM_A(4); break;
    case 2: MD_ASM_A(2); break;
    default: MD_ASM_A(1); break;
  }
#undef MD_ASM_A
  return hipGetLastError();
}

hipError_t launch_assemble(int L, int n, int D, int Dc, int m, int nnz, const int32_t *poly_ptr,
                           const int32_t *asm_ptr, const int32_t *asm_ent, const double *cst, const double *val,
                           const double *der, double *b, double *A, hipStream_t st, double *tsz,
                           const double *vsize, TOut rt, TOut at, int *clear, int clear_count, double *empty,
                           size_t empty_count, CountWait wait) {
  if (Dc < 1 || Dc > D) return hipErrorInvalidValue;
  if (rt.p && (rt.lo < 0 || rt.W < 1 || rt.lo + rt.W > Dc || rt.L < 1 || rt.L > L)) return hipErrorInvalidValue;
  if (at.p && (at.lo != 0 || at.W < 1 || at.W > Dc || at.L < 1 || at.L > L)) return hipErrorInvalidValue;
  const size_t nn = (size_t)n * n;
  const int ti = assemble_tile(L, Dc);
  if ((Dc + 256 / ti - 1) / (256 / ti) > asm_a_max_slices(L)) return hipErrorInvalidValue;
  const size_t lds = at.p ? (size_t)ti * (Dc + 1) * L * sizeof(double) : 0;
  const unsigned GA = (unsigned)((nn + ti - 1) / ti);
  const size_t bthreads = std::max({(size_t)n * Dc * 4, (size_t)(clear ? clear_count : 0), empty ? empty_count : 0});
  const dim3 grid(GA + (unsigned)((bthreads + 255) / 256));
#define MD_ASM_BA(TI)                                                                                             \
  MD_DISPATCH(L, hipLaunchKernelGGL((assemble_bA_kernel<LL, TI>), grid, dim3(256), lds, st, GA, n, D, Dc, m, nnz, \
                                    poly_ptr, asm_ptr, asm_ent, cst, val, der, b, A, tsz, vsize, rt, at, clear,   \
                                    clear_count, empty, empty_count, wait))
  switch (ti) {
    case 16: MD_ASM_BA(16); break;
    case 8: MD_ASM_BA(8); break;
    case 4: MD_ASM_BA(4); break;
    case 2: MD_ASM_BA(2); break;
    default: MD_ASM_BA(1); break;
  }
#undef MD_ASM_BA
  return hipGetLastError();
}

}  // namespace mdk
