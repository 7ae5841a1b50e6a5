// Assembly of the residual and Jacobian series from the monomial values and
// derivative products (Section 2: b(t) = -p(x(t)), A(t) = p'(x(t))), in a
// fixed monomial order so that results are reproducible, with the size of the
// terms of each residual coefficient for the staggered method's stopping test
// (Section 4).
#include "common.hpp"
#include "kernels.hpp"
#include "md.hpp"

namespace mdk {

// b_i(t) = -(c_{i,0}(t) + sum_{m in P_i} value_m(t)), one thread per (i, s)
// for the first Dc coefficients s.  tsz (nullable, [n][D]) gets the size of
// the terms whose rounding errors reach b_{i,s}, against which the staggered
// method judges it: |c_{i,0,s}| + sum_m vsize_{m,s}, the largest product of
// each monomial's chain (|value_{m,s}| when vsize is null; leading limbs).
template <int L>
__global__ void assemble_b_kernel(int n, int D, int Dc, int m, const int32_t *poly_ptr, const double *cst,
                                  const double *val, double *b, double *tsz, const double *vsize) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nD = (size_t)n * D, mD = (size_t)m * D;
  if (t >= (size_t)n * Dc) return;
  const int i = (int)(t / Dc), s = (int)(t - (size_t)i * Dc);
  const size_t q = (size_t)i * D + s;
  double acc[L];
  ld<L>(cst, nD, q, acc);
  double size = fabs(acc[0]);
  for (int mj = poly_ptr[i]; mj < poly_ptr[i + 1]; ++mj) {
    double v[L], r[L];
    ld<L>(val, mD, (size_t)mj * D + s, v);
    size += vsize ? vsize[(size_t)mj * D + s] : fabs(v[0]);
    MD<L>::add(acc, v, r);
    md::copy<L>(r, acc);
  }
  md::neg<L>(acc, acc);
  st<L>(b, nD, q, acc);
  if (tsz) tsz[q] = size;
}

// A[i][j][s] = sum of the derivative series of row i's monomials with respect
// to x_j, in monomial order; one thread per (i, j, s) for the first Dc
// coefficients s.
template <int L>
__global__ void assemble_A_kernel(int n, int D, int Dc, int nnz, const int32_t *asm_ptr, const int32_t *asm_ent,
                                  const double *der, double *A) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nnD = (size_t)n * n * D, zD = (size_t)nnz * D;
  if (t >= (size_t)n * n * Dc) return;
  const size_t ij = t / Dc;
  const int s = (int)(t - ij * Dc);
  const size_t q = ij * D + s;
  const int lo = asm_ptr[ij], hi = asm_ptr[ij + 1];
  double acc[L];
  md::zero<L>(acc);
  if (lo < hi) {
    ld<L>(der, zD, (size_t)asm_ent[lo] * D + s, acc);
    for (int t = lo + 1; t < hi; ++t) {
      double v[L], r[L];
      ld<L>(der, zD, (size_t)asm_ent[t] * D + s, v);
      MD<L>::add(acc, v, r);
      md::copy<L>(r, acc);
    }
  }
  st<L>(A, nnD, q, acc);
}

// Coefficient 0 of A into a dense row-major matrix a0 [L][n][n], summed in
// the same order as assemble_A_kernel, so it equals A[i][j][0] bit for bit.
template <int L>
__global__ void assemble_A0_kernel(int n, int D, int nnz, const int32_t *asm_ptr, const int32_t *asm_ent,
                                   const double *der, double *a0) {
  const size_t ij = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nn = (size_t)n * n, zD = (size_t)nnz * D;
  if (ij >= nn) return;
  const int lo = asm_ptr[ij], hi = asm_ptr[ij + 1];
  double acc[L];
  md::zero<L>(acc);
  if (lo < hi) {
    ld<L>(der, zD, (size_t)asm_ent[lo] * D, acc);
    for (int t = lo + 1; t < hi; ++t) {
      double v[L], r[L];
      ld<L>(der, zD, (size_t)asm_ent[t] * D, v);
      MD<L>::add(acc, v, r);
      md::copy<L>(r, acc);
    }
  }
  st<L>(a0, nn, ij, acc);
}

// ------------------------------------------------------------------ launchers

hipError_t launch_assemble_A0(int L, int n, int D, int nnz, const int32_t *asm_ptr, const int32_t *asm_ent,
                              const double *der, double *a0, hipStream_t st) {
  const size_t nn = (size_t)n * n;
  switch (L) {
    case 1: hipLaunchKernelGGL(assemble_A0_kernel<1>, dim3((nn + 63) / 64), dim3(64), 0, st, n, D, nnz, asm_ptr, asm_ent, der, a0); break;
    case 2: hipLaunchKernelGGL(assemble_A0_kernel<2>, dim3((nn + 63) / 64), dim3(64), 0, st, n, D, nnz, asm_ptr, asm_ent, der, a0); break;
    case 4: hipLaunchKernelGGL(assemble_A0_kernel<4>, dim3((nn + 63) / 64), dim3(64), 0, st, n, D, nnz, asm_ptr, asm_ent, der, a0); break;
    case 8: hipLaunchKernelGGL(assemble_A0_kernel<8>, dim3((nn + 63) / 64), dim3(64), 0, st, n, D, nnz, asm_ptr, asm_ent, der, a0); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_assemble_b(int L, int n, int D, int Dc, int m, const int32_t *poly_ptr, const double *cst,
                             const double *val, double *b, hipStream_t st, double *tsz, const double *vsize) {
  if (Dc < 1 || Dc > D) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)(((size_t)n * Dc + 255) / 256);
  switch (L) {
    case 1: hipLaunchKernelGGL(assemble_b_kernel<1>, dim3(blocks), dim3(256), 0, st, n, D, Dc, m, poly_ptr, cst, val, b, tsz, vsize); break;
    case 2: hipLaunchKernelGGL(assemble_b_kernel<2>, dim3(blocks), dim3(256), 0, st, n, D, Dc, m, poly_ptr, cst, val, b, tsz, vsize); break;
    case 4: hipLaunchKernelGGL(assemble_b_kernel<4>, dim3(blocks), dim3(256), 0, st, n, D, Dc, m, poly_ptr, cst, val, b, tsz, vsize); break;
    case 8: hipLaunchKernelGGL(assemble_b_kernel<8>, dim3(blocks), dim3(256), 0, st, n, D, Dc, m, poly_ptr, cst, val, b, tsz, vsize); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_assemble_A(int L, int n, int D, int Dc, int nnz, const int32_t *asm_ptr, const int32_t *asm_ent,
                             const double *der, double *A, hipStream_t st) {
  if (Dc < 1 || Dc > D) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)(((size_t)n * n * Dc + 255) / 256);
  switch (L) {
    case 1: hipLaunchKernelGGL(assemble_A_kernel<1>, dim3(blocks), dim3(256), 0, st, n, D, Dc, nnz, asm_ptr, asm_ent, der, A); break;
    case 2: hipLaunchKernelGGL(assemble_A_kernel<2>, dim3(blocks), dim3(256), 0, st, n, D, Dc, nnz, asm_ptr, asm_ent, der, A); break;
    case 4: hipLaunchKernelGGL(assemble_A_kernel<4>, dim3(blocks), dim3(256), 0, st, n, D, Dc, nnz, asm_ptr, asm_ent, der, A); break;
    case 8: hipLaunchKernelGGL(assemble_A_kernel<8>, dim3(blocks), dim3(256), 0, st, n, D, Dc, nnz, asm_ptr, asm_ent, der, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_assemble(int L, int n, int D, int Dc, int m, int nnz, const int32_t *poly_ptr,
                           const int32_t *asm_ptr, const int32_t *asm_ent, const double *cst, const double *val,
                           const double *der, double *b, double *A, hipStream_t st, double *tsz,
                           const double *vsize) {
  hipError_t e = launch_assemble_b(L, n, D, Dc, m, poly_ptr, cst, val, b, st, tsz, vsize);
  if (e != hipSuccess) return e;
  return launch_assemble_A(L, n, D, Dc, nnz, asm_ptr, asm_ent, der, A, st);
}

}  // namespace mdk
