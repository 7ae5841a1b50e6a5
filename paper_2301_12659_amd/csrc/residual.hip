// Residual of the block Toeplitz system of a Newton step, in multiple-double
// precision (the quantity the Newton loop of Section 2 reports; the residual
// kernels of Section 5.4 and Table 4):
//     r_{i,k} = b_{i,k} - sum_{j=0..k} sum_v A_j(i,v) dx_{v,k-j},
// on every equation or on a caller's sample of equations (the paper suggests
// a few random ones instead of all, since the full residual costs as much as
// the staged updates: n^2 D (D+1) / 2 multiply-adds).
//
// One wavefront per (row, k), or a workgroup of four when there are fewer
// than 1024 tasks.  The n (k+1) products of r_{i,k} are dealt to the lanes
// in (v, j) order with j fastest, so that consecutive lanes read consecutive
// coefficients of one series of A (series-major [n][n][D]) and of dx; every
// lane accumulates level sums, then one butterfly per wavefront, the sums of
// the wavefronts through LDS, one subtraction from b.  The 1-norms over
// the rows are formed by a second kernel in a fixed order.
#include "common.hpp"
#include "kernels.hpp"
#include "md.hpp"

namespace mdk {

template <int L, int W>
__global__ void __launch_bounds__(256) residual_kernel(int n, int D, int nrows, const int32_t *rows, const double *A,
                                                       const double *b, const double *dx, double *r,
                                                       int32_t *status) {
  // W wavefronts per (row, k): 1 when there are tasks enough to fill the
  // chip, 4 (the whole workgroup) when there are few, e.g. a sampled row
  __shared__ double part[4][L];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tl = (W == 1) ? lane : (int)threadIdx.x;  // lane within the task's team
  const size_t task = (size_t)blockIdx.x * (4 / W) + (W == 1 ? wv : 0);
  if (task >= (size_t)nrows * D) return;  // whole teams leave together
  const int q = (int)(task / D), k = (int)(task - (size_t)q * D);
  const int i = rows ? rows[q] : q;
  if (i < 0 || i >= n) {
    if (tl == 0 && status) set_status(status, MD_EINVAL);
    return;
  }
  const size_t nD = (size_t)n * D, nnD = (size_t)n * n * D;
  const int kp = k + 1, terms = n * kp, step = 64 * W;
  double acc[L];
  md::zero<L>(acc);
  int v = tl / kp, j = tl - v * kp;  // term t = v (k+1) + j, t = tl first
  for (int t = tl; t < terms; t += step) {
    double a[L], x[L];
    ld<L>(A, nnD, ((size_t)i * n + v) * D + j, a);
    ld<L>(dx, nD, (size_t)v * D + (k - j), x);
    MD<L>::fma_lazy(acc, a, x);
    j += step;
    const int c = j / kp;
    v += c;
    j -= c * kp;
  }
  team_sum_lazy<L>(acc, 64);
  double s[L];
  MD<L>::renorm(acc, s);
  if (W > 1) {
    if (lane == 0)
      for (int l = 0; l < L; ++l) part[wv][l] = s[l];
    __syncthreads();
    if (wv == 0) {
      for (int l = 0; l < L; ++l) s[l] = part[0][l];
      for (int w = 1; w < W; ++w) {
        double o[L], t2[L];
        for (int l = 0; l < L; ++l) o[l] = part[w][l];
        MD<L>::add(s, o, t2);
        md::copy<L>(t2, s);
      }
    }
  }
  if (tl == 0) {
    double bv[L], rv[L];
    ld<L>(b, nD, (size_t)i * D + k, bv);
    MD<L>::sub(bv, s, rv);
    st<L>(r, (size_t)nrows * D, (size_t)q * D + k, rv);
  }
}

// norm1[k] = sum_q |r_{q,k}| on leading limbs: one workgroup per k, a fixed
// tree order over the rows.
__global__ void __launch_bounds__(256) residual_norm_kernel(int nrows, int D, const double *r, double *norm1) {
  __shared__ double part[256];
  const int k = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int q = t; q < nrows; q += blockDim.x) s += fabs(r[(size_t)q * D + k]);
  part[t] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) part[t] += part[t + h];
    __syncthreads();
  }
  if (t == 0) norm1[k] = part[0];
}

hipError_t launch_residual(int L, int n, int D, int nrows, const int32_t *rows, const double *A, const double *b,
                           const double *dx, double *r, double *norm1, int32_t *status, hipStream_t st) {
  if (n < 1 || D < 1 || nrows < 1) return hipErrorInvalidValue;
  const size_t tasks = (size_t)nrows * D;
  if (tasks < 1024) {  // a workgroup per task
    MD_DISPATCH(L, hipLaunchKernelGGL((residual_kernel<LL, 4>), dim3((unsigned)tasks), dim3(256), 0, st, n, D, nrows,
                                      rows, A, b, dx, r, status));
  } else {  // a wavefront per task
    MD_DISPATCH(L, hipLaunchKernelGGL((residual_kernel<LL, 1>), dim3((unsigned)((tasks + 3) / 4)), dim3(256), 0, st,
                                      n, D, nrows, rows, A, b, dx, r, status));
  }
  if (norm1) hipLaunchKernelGGL(residual_norm_kernel, dim3(D), dim3(256), 0, st, nrows, D, r, norm1);
  return hipGetLastError();
}

}  // namespace mdk
