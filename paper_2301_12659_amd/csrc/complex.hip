// Complex data (Section 5.2): evaluation and differentiation at complex
// power series with the 4M products computed side by side, and the pieces
// of a complex Newton step around the real linear-algebra kernels.
//
// A complex multiple-double array is [2][L][...]: the real plane, then the
// imaginary plane, each limb-major like a real array.  A complex truncated
// product W = U * V is, per coefficient s,
//     Re W_s = sum_i Re U_i Re V_{s-i} - Im U_i Im V_{s-i},
//     Im W_s = sum_i Re U_i Im V_{s-i} + Im U_i Re V_{s-i},
// the four real products of the 4M method.  A complex worker has 2G lanes:
// lanes [0, G) form the real part and lanes [G, 2G) the imaginary part of
// every output at the same time, each lane adding both of its part's products
// into one level-sum accumulator, with the term layout of the real
// convolution (outputs paired s and D-1-s, halves on lanes p and p + G2).
// With 2G <= 64 several workers share a wavefront and synchronize as a
// wavefront; with 2G = 128 (D > 32) a worker is a workgroup of two
// wavefronts and uses workgroup barriers.  Exponents 1 and 2 (no power
// table: the common factor of an exponent 2 is the variable itself).
//
// The complex block system A(t) dx(t) = b(t) is solved through its real form
// of dimension 2n, [[Re A, -Im A], [Im A, Re A]] [Re dx; Im dx] = [Re b; Im b],
// with the real QR, M and stage kernels.
#include "common.hpp"
#include "evaldiff_dev.hpp"
#include "kernels.hpp"
#include "md.hpp"

namespace mdk {

struct SyncWave {
  __device__ void operator()() const { wave_sync(); }
};
struct SyncBlock {
  __device__ void operator()() const { __syncthreads(); }
};

// Complex truncated product W = scale * (U * V) in LDS; part 0 (lanes < G)
// writes Re W, part 1 writes Im W.
template <int L>
__device__ void conv_c(const double *U, const double *V, double *W, int D, int lane2, int G, int scale) {
  const int Dp = D + 1, G2 = pair_lanes(D), S = split_factor(D);
  const int part = lane2 >= G, lane = lane2 - part * G;
  const size_t P = (size_t)L * Dp;  // offset of the imaginary part of a series
  // part 0: Re U Re V - Im U Im V; part 1: Re U Im V + Im U Re V
  const double *A1 = U, *B1 = part ? V + P : V, *A2 = U + P, *B2 = part ? V : V + P;
  const double sgn = part ? 1.0 : -1.0;
  double *Wp = W + part * P;
  const int h = lane / G2, p = lane - h * G2;
  const bool act = p < (D + 1) / 2;
  const int o1 = p, o2 = D - 1 - p;
  const int H = (D + S) / S;
  const int t0 = h * H;
  // the first output's level sums are parked in acc1 when its last term is
  // in and renormalized after the loop by all lanes together
  double acc0[L], acc1[L];
  md::zero<L>(acc0);
  md::zero<L>(acc1);
  for (int tt = 0; tt < H; ++tt) {
    const int t = t0 + tt;
    const bool ph1 = t <= o1;
    int i = ph1 ? t : t - o1 - 1;
    int j = (ph1 ? o1 : o2) - i;
    if (!act || t > D) {  // reads the zero padding
      i = D;
      j = 0;
    }
    double u[L], v[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      u[l] = A1[l * Dp + i];
      v[l] = B1[l * Dp + j];
    }
    MD<L>::fma_lazy(acc0, u, v);
#pragma unroll
    for (int l = 0; l < L; ++l) {
      u[l] = sgn * A2[l * Dp + i];
      v[l] = B2[l * Dp + j];
    }
    MD<L>::fma_lazy(acc0, u, v);
    if (t == o1) {
      md::copy<L>(acc0, acc1);
      md::zero<L>(acc0);
    }
  }
  if (h == 0 && act) {
    double r[L];
    MD<L>::renorm(acc1, r);
    md::mul_int<L>(r, scale);
#pragma unroll
    for (int l = 0; l < L; ++l) Wp[l * Dp + o1] = r[l];
  }
  if (S == 2) {  // lanes p and p + G2 of the same part hold the two halves
    double o[L];
#pragma unroll
    for (int l = 0; l < L; ++l) o[l] = __shfl_xor(acc0[l], G2, 64);
    MD<L>::add_lazy(acc0, o);
  }
  double r[L];
  MD<L>::renorm(acc0, r);
  if (h == 0 && act && o2 > o1) {
    md::mul_int<L>(r, scale);
#pragma unroll
    for (int l = 0; l < L; ++l) Wp[l * Dp + o2] = r[l];
  }
}

// W = scale * c * V for a complex scalar c = cr + i ci (W must not alias V).
template <int L>
__device__ void scal_c(const double (&cr)[L], const double (&ci)[L], const double *V, double *W, int D, int lane2,
                       int G, int scale) {
  const int Dp = D + 1;
  const int part = lane2 >= G, lane = lane2 - part * G;
  const size_t P = (size_t)L * Dp;
  double ci_s[L];
#pragma unroll
  for (int l = 0; l < L; ++l) ci_s[l] = part ? ci[l] : -ci[l];
  const double *B1 = part ? V + P : V, *B2 = part ? V : V + P;
  for (int s = lane; s < D; s += G) {
    double acc[L], v[L], r[L];
    md::zero<L>(acc);
#pragma unroll
    for (int l = 0; l < L; ++l) v[l] = B1[l * Dp + s];
    MD<L>::fma_lazy(acc, cr, v);
#pragma unroll
    for (int l = 0; l < L; ++l) v[l] = B2[l * Dp + s];
    MD<L>::fma_lazy(acc, ci_s, v);
    MD<L>::renorm(acc, r);
    md::mul_int<L>(r, scale);
#pragma unroll
    for (int l = 0; l < L; ++l) W[part * P + l * Dp + s] = r[l];
  }
}

// Complex series between global memory ([2] planes, imaginary plane at
// element offset plane) and LDS ([2][L][D + 1]).
__device__ __forceinline__ void load_c(double *S, const double *g, size_t gstride, size_t plane, size_t off, int L,
                                       int D, int lane2, int G2L) {
  load_series(S, g, gstride, off, L, D, lane2, G2L);
  load_series(S + (size_t)L * (D + 1), g + plane, gstride, off, L, D, lane2, G2L);
}

__device__ __forceinline__ void store_c(double *g, size_t gstride, size_t plane, size_t off, const double *S, int L,
                                        int D, int lane2, int G2L) {
  store_series(g, gstride, off, S, L, D, lane2, G2L);
  store_series(g + plane, gstride, off, S + (size_t)L * (D + 1), L, D, lane2, G2L);
}

// One complex monomial c * prod_j x_{v_j}^{a_j} (a_j in {1, 2}) by the
// reverse-mode products of eval_monomial: common factor, backward chain
// parked in the derivative slots, forward chain with the cross products.
template <int L, class Sync>
__device__ void eval_monomial_c(const EvalArgs &a, int mono, int lane2, int G, double *buf0, Sync sync) {
  const int D = a.D, Dc = a.Dc, Dp = Dc + 1, G2L = 2 * G;
  const size_t CS = 2 * (size_t)L * Dp;  // one complex series in LDS
  double *buf[3] = {buf0, buf0 + CS, buf0 + 2 * CS};
  for (int q = lane2; q < 6 * L; q += G2L) buf0[(size_t)q * Dp + Dc] = 0.0;
  const int e0 = a.mon_ptr[mono], k = a.mon_ptr[mono + 1] - e0;
  const size_t nD = (size_t)a.n * D, mD = (size_t)a.m * D, zD = (size_t)a.nnz * D;
  const size_t xp = (size_t)L * nD, vp = (size_t)L * mD, dp = (size_t)L * zD, cp = (size_t)L * a.m;
  double cr[L], ci[L];
  ld<L>(a.cff, (size_t)a.m, mono, cr);
  ld<L>(a.cff + cp, (size_t)a.m, mono, ci);
  auto xoff = [&](int v) { return (size_t)v * D; };
  auto der_off = [&](int j) { return (size_t)(e0 + j) * D; };
  const int part = lane2 >= G, lane = lane2 - part * G;
  if (k == 0) {  // constant monomial
    for (int s = lane; s < Dc; s += G) {
#pragma unroll
      for (int l = 0; l < L; ++l)
        a.val[part * vp + (size_t)l * mD + (size_t)mono * D + s] = (s == 0) ? (part ? ci[l] : cr[l]) : 0.0;
    }
    return;
  }
  sync();
  // backward chain: b_1 = x_{v_k}, b_q = b_{q-1} * x_{v_{k-q+1}}, parked in
  // the slot of entry k - q - 1
  if (k >= 3) {
    double *B = buf[0], *X = buf[1], *Wb = buf[2];
    load_c(B, a.x, nD, xp, xoff(a.var[e0 + k - 1]), L, Dc, lane2, G2L);
    for (int q = 2; q <= k - 1; ++q) {
      load_c(X, a.x, nD, xp, xoff(a.var[e0 + k - q]), L, Dc, lane2, G2L);
      sync();
      conv_c<L>(B, X, Wb, Dc, lane2, G, 1);
      sync();
      store_c(a.der, zD, dp, der_off(k - q - 1), Wb, L, Dc, lane2, G2L);
      double *t = B;
      B = Wb;
      Wb = t;
      sync();
    }
  }
  // common factor (exponent-2 variables) and f_0 = c * CF
  double *U = buf[0], *V = buf[1], *W = buf[2];
  bool f0_scalar = true;
  for (int j = 0; j < k; ++j) {
    if (a.exp[e0 + j] < 2) continue;
    const int v = a.var[e0 + j];
    if (f0_scalar) {
      load_c(U, a.x, nD, xp, xoff(v), L, Dc, lane2, G2L);
      f0_scalar = false;
      sync();
    } else {
      load_c(V, a.x, nD, xp, xoff(v), L, Dc, lane2, G2L);
      sync();
      conv_c<L>(U, V, W, Dc, lane2, G, 1);
      sync();
      double *t = U;
      U = W;
      W = t;
    }
  }
  if (!f0_scalar) {
    scal_c<L>(cr, ci, U, W, Dc, lane2, G, 1);
    sync();
    double *t = U;
    U = W;
    W = t;
  }
  // forward chain with the cross products
  for (int j = 1; j <= k; ++j) {
    const int ej = j - 1;
    const int aj = a.exp[e0 + ej];
    if (j < k) {
      if (k - j == 1)
        load_c(V, a.x, nD, xp, xoff(a.var[e0 + k - 1]), L, Dc, lane2, G2L);
      else
        load_c(V, a.der, zD, dp, der_off(ej), L, Dc, lane2, G2L);
      sync();
      if (f0_scalar && j == 1)
        scal_c<L>(cr, ci, V, W, Dc, lane2, G, aj);
      else
        conv_c<L>(U, V, W, Dc, lane2, G, aj);
      sync();
      store_c(a.der, zD, dp, der_off(ej), W, L, Dc, lane2, G2L);
    } else {  // d/dx_{v_k} = a_k f_{k-1}
      for (int s = lane; s < Dc; s += G) {
        double r[L];
#pragma unroll
        for (int l = 0; l < L; ++l)
          r[l] = (f0_scalar && j == 1) ? ((s == 0) ? (part ? ci[l] : cr[l]) : 0.0) : U[part * L * Dp + l * Dp + s];
        md::mul_int<L>(r, aj);
#pragma unroll
        for (int l = 0; l < L; ++l) a.der[part * dp + (size_t)l * zD + der_off(ej) + s] = r[l];
      }
    }
    sync();
    load_c(V, a.x, nD, xp, xoff(a.var[e0 + ej]), L, Dc, lane2, G2L);
    sync();
    if (f0_scalar && j == 1)
      scal_c<L>(cr, ci, V, W, Dc, lane2, G, 1);
    else
      conv_c<L>(U, V, W, Dc, lane2, G, 1);
    sync();
    double *t = U;
    U = W;
    W = t;
  }
  store_c(a.val, mD, vp, (size_t)mono * D, U, L, Dc, lane2, G2L);
}

// Workers of 2G lanes; WIDE: one worker per workgroup of 2G = 128 threads,
// else workgroups of one wavefront holding 64 / (2G) workers.
template <int L, bool WIDE>
__global__ void __launch_bounds__(128) evaldiff_complex_kernel(EvalArgs a) {
  extern __shared__ double lds[];
  const int G = worker_lanes(a.Dc), G2L = 2 * G;
  const size_t per = 6 * (size_t)L * (a.Dc + 1);
  if (WIDE) {
    eval_monomial_c<L>(a, a.order[blockIdx.x], (int)threadIdx.x, G, lds, SyncBlock{});
  } else {
    const int wpb = 64 / G2L, wid = threadIdx.x / G2L, lane2 = threadIdx.x - wid * G2L;
    const int widx = blockIdx.x * wpb + wid;
    if (widx >= a.m) return;  // whole workers leave together
    eval_monomial_c<L>(a, a.order[widx], lane2, G, lds + wid * per, SyncWave{});
  }
}

template <int L>
static hipError_t launch_evaldiff_complex_T(const EvalArgs &a, hipStream_t st) {
  const int G = worker_lanes(a.Dc), G2L = 2 * G;
  const size_t per = 6 * (size_t)L * (a.Dc + 1) * sizeof(double);
  if (a.m <= 0) return hipSuccess;
  if (G2L > 64) {
    hipLaunchKernelGGL((evaldiff_complex_kernel<L, true>), dim3(a.m), dim3(G2L), per, st, a);
  } else {
    const int wpb = 64 / G2L;
    hipLaunchKernelGGL((evaldiff_complex_kernel<L, false>), dim3((a.m + wpb - 1) / wpb), dim3(64), per * wpb, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_evaldiff_complex(int L, const EvalArgs &a, hipStream_t st) {
  switch (L) {
    case 2: return launch_evaldiff_complex_T<2>(a, st);
    case 4: return launch_evaldiff_complex_T<4>(a, st);
    case 8: return launch_evaldiff_complex_T<8>(a, st);
  }
  return hipErrorInvalidValue;
}

// The real form of the complex block system: At [L][2n][2n][D] with blocks
// [[Re A, -Im A], [Im A, Re A]] (series-major like A [2][L][n][n][D]), and
// bt [L][2n][D] = [Re b; Im b].  One thread per entry of At.
__global__ void __launch_bounds__(256) complex_embed_kernel(int L, int n, int D, const double *A, const double *b,
                                                            double *At, double *bt) {
  const size_t N = 2 * (size_t)n, q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = N * N * D, nnD = (size_t)n * n * D, nD = (size_t)n * D;
  if (q < (size_t)L * per) {
    const size_t l = q / per, r = q - l * per;
    const size_t I = r / (N * D), rem = r - I * N * D, J = rem / D, k = rem - J * D;
    const size_t i = I % n, j = J % n;
    const bool im = (I >= (size_t)n) != (J >= (size_t)n);  // off-diagonal blocks hold Im A
    double v = A[(im ? (size_t)L * nnD : 0) + l * nnD + (i * n + j) * D + k];
    if (I < (size_t)n && J >= (size_t)n) v = -v;
    At[q] = v;
  }
  if (q < (size_t)L * N * D) {
    const size_t l = q / (N * D), r = q - l * N * D, I = r / D, k = r - I * D;
    const size_t i = I % n;
    bt[q] = b[(I >= (size_t)n ? (size_t)L * nD : 0) + l * nD + i * D + k];
  }
}

// dx [2][L][n][D] from the real solution dxt [L][2n][D].
__global__ void __launch_bounds__(256) complex_unpack_kernel(int L, int n, int D, const double *dxt, double *dx) {
  const size_t nD = (size_t)n * D, q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 2 * (size_t)L * nD) return;
  const size_t part = q / ((size_t)L * nD), r = q - part * L * nD, l = r / nD, e = r - l * nD;
  dx[q] = dxt[l * 2 * nD + part * nD + e];
}

// a[q] = max(a[q], b[q]): norms of the two parts.
__global__ void __launch_bounds__(256) max_kernel(int count, const double *b, double *a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < count) a[q] = fmax(a[q], b[q]);
}

hipError_t launch_complex_embed(int L, int n, int D, const double *A, const double *b, double *At, double *bt,
                                hipStream_t st) {
  const size_t tot = (size_t)L * 4 * n * n * D;
  hipLaunchKernelGGL(complex_embed_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, n, D, A, b, At,
                     bt);
  return hipGetLastError();
}

hipError_t launch_complex_unpack(int L, int n, int D, const double *dxt, double *dx, hipStream_t st) {
  const size_t tot = 2 * (size_t)L * n * D;
  hipLaunchKernelGGL(complex_unpack_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L, n, D, dxt, dx);
  return hipGetLastError();
}

hipError_t launch_max(int count, const double *b, double *a, hipStream_t st) {
  hipLaunchKernelGGL(max_kernel, dim3((count + 255) / 256), dim3(256), 0, st, count, b, a);
  return hipGetLastError();
}

}  // namespace mdk
