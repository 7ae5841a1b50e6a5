// Linear algebra on multiple-double matrices for the Newton step:
//  * Householder QR of A_0 (Sections 1.1 and 5.3),
//  * Q^T and R^{-1} applied to unit vectors to form M = R^{-1} Q^T once per
//    step (the paper's "Q^H b" and back-substitution kernels, with the
//    triangular solve done column by column with the inverted diagonal,
//    Section 1.1's tiled back substitution with one tile),
//  * the staged right-hand-side updates of the block Toeplitz system
//    (Sections 4 and 5.4), one kernel per stage,
//  * the update x := x + dx and the convergence norms (Section 2).
//
// Stage recurrence.  With M = A_0^{-1} (from the QR factors) and
// N = M A_1, stage k computes
//     dx_k = M r_k - N dx_{k-1},   r_k = b_k - sum_{j=2..k} A_j dx_{k-j},
// which is A_0^{-1} (b_k - sum_{j=1..k} A_j dx_{k-j}) reassociated so that the
// only work that waits for dx_{k-1} is one matrix-vector product per row; in
// the same launch every later right-hand side r_m (m > k) receives its term
// A_{m-k+1} dx_{k-1}.  Every stage is one launch over the whole GPU.
#include "common.hpp"
#include "kernels.hpp"

namespace mdk {

// ----------------------------------------------------------------- status

__global__ void status_init_kernel(int32_t *status) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && status) *status = MD_OK;
}

// ----------------------------------------------------------------- QR

// Unblocked Householder QR in one workgroup; a [L][n][n] row-major in place.
template <int L>
__global__ void __launch_bounds__(256) qr_kernel(int n, double *a, double *tau, int32_t *status) {
  __shared__ double red[4][L];
  __shared__ double sh_tau[L], sh_inv[L];
  __shared__ int sh_skip;
  const size_t nn = (size_t)n * n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  for (int c = 0; c < n; ++c) {
    // squared norm of the column c, rows c..n-1
    double acc[L];
    md::zero<L>(acc);
    for (int i = c + tid; i < n; i += blockDim.x) {
      double xi[L];
      ld<L>(a, nn, (size_t)i * n + c, xi);
      MD<L>::fma(acc, xi, xi);
    }
    team_sum<L>(acc, 64);
    if (lane == 0)
#pragma unroll
      for (int l = 0; l < L; ++l) red[w][l] = acc[l];
    __syncthreads();
    if (tid == 0) {
      double nrm2[L];
#pragma unroll
      for (int l = 0; l < L; ++l) nrm2[l] = red[0][l];
      for (int q = 1; q < nw; ++q) {
        double t[L], s[L];
#pragma unroll
        for (int l = 0; l < L; ++l) t[l] = red[q][l];
        MD<L>::add(nrm2, t, s);
        md::copy<L>(s, nrm2);
      }
      double alpha[L], x0[L];
      md::sqrt<L>(nrm2, alpha);
      ld<L>(a, nn, (size_t)c * n + c, x0);
      if (!(alpha[0] > 0.0)) {  // zero column: R_cc = 0, H_c = I
        sh_skip = 1;
#pragma unroll
        for (int l = 0; l < L; ++l) tau[(size_t)l * n + c] = 0.0;
        set_status(status, MD_ESINGULAR);
      } else {
        sh_skip = 0;
        double beta[L], v0[L], num[L], tc[L], one[L], inv[L];
        if (x0[0] >= 0.0) md::neg<L>(alpha, beta);  // beta = -sign(x0) ||x||, sign(0) = +1
        else md::copy<L>(alpha, beta);
        MD<L>::sub(x0, beta, v0);
        MD<L>::sub(beta, x0, num);
        md::div<L>(num, beta, tc);  // tau = (beta - x0) / beta
        md::zero<L>(one);
        one[0] = 1.0;
        md::div<L>(one, v0, inv);   // v = x / (x0 - beta) below the diagonal
        st<L>(a, nn, (size_t)c * n + c, beta);
        st<L>(tau, n, c, tc);
#pragma unroll
        for (int l = 0; l < L; ++l) {
          sh_tau[l] = tc[l];
          sh_inv[l] = inv[l];
        }
      }
    }
    __syncthreads();
    if (sh_skip) continue;
    double inv[L], tc[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      inv[l] = sh_inv[l];
      tc[l] = sh_tau[l];
    }
    for (int i = c + 1 + tid; i < n; i += blockDim.x) {
      double xi[L], r[L];
      ld<L>(a, nn, (size_t)i * n + c, xi);
      MD<L>::mul(xi, inv, r);
      st<L>(a, nn, (size_t)i * n + c, r);
    }
    __syncthreads();
    // apply H_c to the trailing columns, one wavefront per column
    for (int j = c + 1 + w; j < n; j += nw) {
      double dot[L];
      md::zero<L>(dot);
      for (int i = c + lane; i < n; i += 64) {
        double aij[L];
        ld<L>(a, nn, (size_t)i * n + j, aij);
        if (i == c) {
          double s[L];
          MD<L>::add(dot, aij, s);
          md::copy<L>(s, dot);
        } else {
          double vi[L];
          ld<L>(a, nn, (size_t)i * n + c, vi);
          MD<L>::fma(dot, vi, aij);
        }
      }
      team_sum<L>(dot, 64);
      double wj[L];
      MD<L>::mul(dot, tc, wj);
      for (int i = c + lane; i < n; i += 64) {
        double aij[L];
        ld<L>(a, nn, (size_t)i * n + j, aij);
        if (i == c) {
          double s[L];
          MD<L>::sub(aij, wj, s);
          st<L>(a, nn, (size_t)i * n + j, s);
        } else {
          double vi[L];
          ld<L>(a, nn, (size_t)i * n + c, vi);
          MD<L>::fms(aij, vi, wj);
          st<L>(a, nn, (size_t)i * n + j, aij);
        }
      }
    }
    __syncthreads();
  }
}

// 1 / R_ii for the back substitutions.  A diagonal entry below
// n * 2^(-53 L) times the largest one (leading limbs) means A_0 is singular to
// working precision; it is reported and its inverse set to zero.
template <int L>
__global__ void invdiag_kernel(int n, const double *qr, double *invd, int32_t *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t nn = (size_t)n * n;
  double rmax = 0.0;
  for (int j = 0; j < n; ++j) rmax = fmax(rmax, fabs(qr[(size_t)j * n + j]));
  double r[L], one[L], q[L];
  ld<L>(qr, nn, (size_t)i * n + i, r);
  md::zero<L>(one);
  one[0] = 1.0;
  if (!(fabs(r[0]) > ldexp((double)n, -53 * L) * rmax)) {
    md::zero<L>(q);
    set_status(status, MD_ESINGULAR);
  } else {
    md::div<L>(one, r, q);
  }
  st<L>(invd, n, i, q);
}

// Column c of M = R^{-1} Q^T: y = H_{n-1} ... H_0 e_c (Q^T applied to e_c),
// then z = R^{-1} y by column-oriented back substitution.  One wavefront per
// column, y kept in LDS.
template <int L>
__global__ void __launch_bounds__(64) form_m_kernel(int n, const double *qr, const double *tau, const double *invd,
                                                    double *M) {
  extern __shared__ double y[];  // [L][n]
  const int c = blockIdx.x, lane = threadIdx.x;
  const size_t nn = (size_t)n * n;
  for (int q = lane; q < L * n; q += 64) y[q] = 0.0;
  wave_sync();
  if (lane == 0) y[c] = 1.0;
  wave_sync();
  for (int r = 0; r < n; ++r) {
    double dot[L];
    md::zero<L>(dot);
    for (int i = r + lane; i < n; i += 64) {
      double yi[L];
#pragma unroll
      for (int l = 0; l < L; ++l) yi[l] = y[l * n + i];
      if (i == r) {
        double s[L];
        MD<L>::add(dot, yi, s);
        md::copy<L>(s, dot);
      } else {
        double vi[L];
        ld<L>(qr, nn, (size_t)i * n + r, vi);
        MD<L>::fma(dot, vi, yi);
      }
    }
    team_sum<L>(dot, 64);
    double tr[L], wv[L];
    ld<L>(tau, n, r, tr);
    MD<L>::mul(dot, tr, wv);
    for (int i = r + lane; i < n; i += 64) {
      double yi[L];
#pragma unroll
      for (int l = 0; l < L; ++l) yi[l] = y[l * n + i];
      if (i == r) {
        double s[L];
        MD<L>::sub(yi, wv, s);
        md::copy<L>(s, yi);
      } else {
        double vi[L];
        ld<L>(qr, nn, (size_t)i * n + r, vi);
        MD<L>::fms(yi, vi, wv);
      }
#pragma unroll
      for (int l = 0; l < L; ++l) y[l * n + i] = yi[l];
    }
    wave_sync();
  }
  // back substitution R z = y, z overwrites y
  for (int i = n - 1; i >= 0; --i) {
    double zi[L], yi[L], di[L];
#pragma unroll
    for (int l = 0; l < L; ++l) yi[l] = y[l * n + i];
    ld<L>(invd, n, i, di);
    MD<L>::mul(yi, di, zi);
    wave_sync();
    if (lane == 0)
#pragma unroll
      for (int l = 0; l < L; ++l) y[l * n + i] = zi[l];
    for (int p = lane; p < i; p += 64) {
      double yp[L], rpi[L];
#pragma unroll
      for (int l = 0; l < L; ++l) yp[l] = y[l * n + p];
      ld<L>(qr, nn, (size_t)p * n + i, rpi);
      MD<L>::fms(yp, rpi, zi);
#pragma unroll
      for (int l = 0; l < L; ++l) y[l * n + p] = yp[l];
    }
    wave_sync();
  }
  for (int i = lane; i < n; i += 64) {
    double zi[L];
#pragma unroll
    for (int l = 0; l < L; ++l) zi[l] = y[l * n + i];
    st<L>(M, nn, (size_t)i * n + c, zi);
  }
}

// Dense copy of the series coefficient k of A: out[i][j] = A[i][j][k].
template <int L>
__global__ void extract_coeff_kernel(int n, int D, int k, const double *A, double *out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nn = (size_t)n * n, nnD = nn * D;
  if (q >= nn) return;
  double v[L];
  ld<L>(A, nnD, q * D + k, v);
  st<L>(out, nn, q, v);
}

// N = M B with B given as coefficient kb of the series matrix A; teams of 16
// lanes per output entry.
template <int L>
__global__ void __launch_bounds__(256) gemm_series_kernel(int n, int D, int kb, const double *M, const double *A,
                                                          double *N) {
  const int T = 16;
  const size_t task = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
  const int tl = threadIdx.x & (T - 1);
  const size_t nn = (size_t)n * n, nnD = nn * D;
  const bool live = task < nn;
  const size_t tk = live ? task : 0;
  const int i = (int)(tk / n), j = (int)(tk - (size_t)i * n);
  double acc[L];
  md::zero<L>(acc);
  for (int v = tl; v < n; v += T) {
    double m[L], b[L];
    ld<L>(M, nn, (size_t)i * n + v, m);
    ld<L>(A, nnD, ((size_t)v * n + j) * D + kb, b);
    MD<L>::fma(acc, m, b);
  }
  team_sum<L>(acc, T);
  if (live && tl == 0) st<L>(N, nn, (size_t)i * n + j, acc);
}

// One stage k of the block Toeplitz solve; see the file comment.
template <int L>
__global__ void __launch_bounds__(256) stage_kernel(int n, int D, int k, const double *M, const double *N,
                                                    const double *A, double *r, double *dx) {
  const int T = 16;
  const size_t task = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
  const int tl = threadIdx.x & (T - 1);
  const size_t nn = (size_t)n * n, nD = (size_t)n * D, nnD = nn * D;
  // stage 0 has no previous update to push into later right-hand sides
  const size_t ntask = (k == 0) ? (size_t)n : (size_t)n * (D - k);
  const bool live = task < ntask;
  const size_t tk = live ? task : 0;
  double acc[L];
  md::zero<L>(acc);
  if (tk < (size_t)n) {  // dx_k(i) = M r_k - N dx_{k-1}
    const int i = (int)tk;
    for (int v = tl; v < n; v += T) {
      double m[L], rv[L];
      ld<L>(M, nn, (size_t)i * n + v, m);
      ld<L>(r, nD, (size_t)v * D + k, rv);
      MD<L>::fma(acc, m, rv);
      if (k > 0) {
        double nv[L], xv[L];
        ld<L>(N, nn, (size_t)i * n + v, nv);
        ld<L>(dx, nD, (size_t)v * D + k - 1, xv);
        MD<L>::fms(acc, nv, xv);
      }
    }
    team_sum<L>(acc, T);
    if (live && tl == 0) st<L>(dx, nD, (size_t)i * D + k, acc);
  } else {  // r_m(i) -= A_{m-k+1} dx_{k-1}, m = k+1..D-1
    const size_t t2 = tk - n;
    const int i = (int)(t2 % n), mm = k + 1 + (int)(t2 / n), jj = mm - k + 1;
    for (int v = tl; v < n; v += T) {
      double av[L], xv[L];
      ld<L>(A, nnD, ((size_t)i * n + v) * D + jj, av);
      ld<L>(dx, nD, (size_t)v * D + k - 1, xv);
      MD<L>::fma(acc, av, xv);
    }
    team_sum<L>(acc, T);
    if (live && tl == 0) {
      double rv[L], s[L];
      ld<L>(r, nD, (size_t)i * D + mm, rv);
      MD<L>::sub(rv, acc, s);
      st<L>(r, nD, (size_t)i * D + mm, s);
    }
  }
}

// x := x + dx, one thread per (i, s).
template <int L>
__global__ void update_kernel(int n, int D, const double *dx, double *x) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nD = (size_t)n * D;
  if (q >= nD) return;
  double a[L], b[L], s[L];
  ld<L>(x, nD, q, a);
  ld<L>(dx, nD, q, b);
  MD<L>::add(a, b, s);
  st<L>(x, nD, q, s);
}

// norms[k] = max_i |b_{i,k}|, norms[D+k] = max_i |dx_{i,k}| (leading limbs);
// a non-finite update is reported.
__global__ void norms_kernel(int n, int D, const double *b, const double *dx, double *norms, int32_t *status) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D) return;
  double nb = 0.0, nx = 0.0;
  bool finite = true;
  for (int i = 0; i < n; ++i) {
    const double bi = b[(size_t)i * D + k], xi = dx[(size_t)i * D + k];
    finite = finite && isfinite(bi) && isfinite(xi);
    nb = fmax(nb, fabs(bi));
    nx = fmax(nx, fabs(xi));
  }
  if (norms) {
    norms[k] = nb;
    norms[D + k] = nx;
  }
  if (!finite) set_status(status, MD_ENONFINITE);
}

template <int L>
__global__ void arith_kernel(int op, int64_t count, const double *a, const double *b, double *c) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  double x[L], y[L], r[L];
  ld<L>(a, count, q, x);
  if (op != 4) ld<L>(b, count, q, y);
  switch (op) {
    case 0: MD<L>::add(x, y, r); break;
    case 1: MD<L>::sub(x, y, r); break;
    case 2: MD<L>::mul(x, y, r); break;
    case 3: md::div<L>(x, y, r); break;
    case 4: md::sqrt<L>(x, r); break;
    default:
      ld<L>(c, count, q, r);
      MD<L>::fma(r, x, y);
      break;
  }
  st<L>(c, count, q, r);
}

// ------------------------------------------------------------------ launchers

#define MD_DISPATCH(L, ...)                          \
  switch (L) {                                       \
    case 2: { constexpr int LL = 2; __VA_ARGS__; } break; \
    case 4: { constexpr int LL = 4; __VA_ARGS__; } break; \
    case 8: { constexpr int LL = 8; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_status_init(int32_t *status, hipStream_t st) {
  hipLaunchKernelGGL(status_init_kernel, dim3(1), dim3(64), 0, st, status);
  return hipGetLastError();
}

hipError_t launch_qr(int L, int n, double *a, double *tau, int32_t *status, hipStream_t st) {
  MD_DISPATCH(L, hipLaunchKernelGGL(qr_kernel<LL>, dim3(1), dim3(256), 0, st, n, a, tau, status));
  return hipGetLastError();
}

hipError_t launch_form_m(int L, int n, const double *qr, const double *tau, double *invd, double *M, int32_t *status,
                         hipStream_t st) {
  MD_DISPATCH(L, {
    hipLaunchKernelGGL(invdiag_kernel<LL>, dim3((n + 63) / 64), dim3(64), 0, st, n, qr, invd, status);
    hipLaunchKernelGGL(form_m_kernel<LL>, dim3(n), dim3(64), (size_t)LL * n * sizeof(double), st, n, qr, tau,
                       (const double *)invd, M);
  });
  return hipGetLastError();
}

hipError_t launch_extract(int L, int n, int D, int k, const double *A, double *out, hipStream_t st) {
  const size_t nn = (size_t)n * n;
  MD_DISPATCH(L, hipLaunchKernelGGL(extract_coeff_kernel<LL>, dim3((nn + 255) / 256), dim3(256), 0, st, n, D, k, A,
                                    out));
  return hipGetLastError();
}

hipError_t launch_gemm_series(int L, int n, int D, int kb, const double *M, const double *A, double *N,
                              hipStream_t st) {
  const size_t threads = (size_t)n * n * 16;
  MD_DISPATCH(L, hipLaunchKernelGGL(gemm_series_kernel<LL>, dim3((threads + 255) / 256), dim3(256), 0, st, n, D, kb,
                                    M, A, N));
  return hipGetLastError();
}

hipError_t launch_stages(int L, int n, int D, const double *M, const double *N, const double *A, double *r,
                         double *dx, hipStream_t st) {
  for (int k = 0; k < D; ++k) {
    const size_t threads = (size_t)n * (k == 0 ? 1 : D - k) * 16;
    MD_DISPATCH(L, hipLaunchKernelGGL(stage_kernel<LL>, dim3((threads + 255) / 256), dim3(256), 0, st, n, D, k, M, N,
                                      A, r, dx));
  }
  return hipGetLastError();
}

hipError_t launch_update(int L, int n, int D, const double *b, const double *dx, double *x, double *norms,
                         int32_t *status, hipStream_t st) {
  const size_t nD = (size_t)n * D;
  MD_DISPATCH(L, hipLaunchKernelGGL(update_kernel<LL>, dim3((nD + 255) / 256), dim3(256), 0, st, n, D, dx, x));
  hipLaunchKernelGGL(norms_kernel, dim3((D + 63) / 64), dim3(64), 0, st, n, D, b, dx, norms, status);
  return hipGetLastError();
}

hipError_t launch_arith(int L, int op, int64_t count, const double *a, const double *b, double *c, hipStream_t st) {
  const int64_t blocks = (count + 255) / 256;
  MD_DISPATCH(L, hipLaunchKernelGGL(arith_kernel<LL>, dim3((unsigned)blocks), dim3(256), 0, st, op, count, a, b, c));
  return hipGetLastError();
}

}  // namespace mdk
