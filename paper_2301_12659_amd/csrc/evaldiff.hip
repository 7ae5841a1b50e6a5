// Evaluation and differentiation of a polynomial system at a power series
// (Section 5.1: reverse mode of algorithmic differentiation with power-series
// products; Section 6: operands staged through shared memory into registers).
// The sums into b(t) = -p(x(t)) and the Jacobian series A(t) are in
// assemble.hip.
//
// Work decomposition.  A "worker" is a group of G lanes of one wavefront; it
// evaluates and differentiates one whole monomial, product after product,
// with three series buffers in LDS.  In a truncated product
// c_s = sum_{i<=s} a_i b_{s-i} the outputs are paired, s and D-1-s, so every
// pair has exactly D+1 multiply-adds: the triangular work is balanced without
// the zero padding of the paper's kernels (which pad to D^2 multiplications,
// Section 5.1).  Each pair is split over S = 2 lanes (S = 1 when D > 64) that
// take the first and second half of its D+1 terms; the halves of the second
// output are added at the end.  G = S * (smallest power of two >= ceil(D/2)).
// Each lane accumulates its terms as multiple-double level sums and
// renormalizes once per output.
//
// Per monomial c * prod_j x_{v_j}^{a_j} with support v_1 < ... < v_k:
//   common factor   CF = prod_{a_j >= 2} x_{v_j}^{a_j - 1}   (the paper's systems
//                   have exponent one only; this reading keeps every derivative a
//                   single cross product), f_0 = c * CF (or the scalar c);
//   backward        b_1 = x_{v_k}, b_q = b_{q-1} * x_{v_{k-q+1}}, q = 2..k-1;
//   forward         f_j = f_{j-1} * x_{v_j}, j = 1..k, value = f_k;
//   cross           d/dx_{v_j} = a_j f_{j-1} * b_{k-j} (j < k), d/dx_{v_k} = a_k f_{k-1}.
// With exponents one and a scalar f_0 this is the paper's 3k-5 convolutions.
// The backward products are parked in the derivative slots of the entries
// that consume them, so no extra memory is needed.
#include "evaldiff_dev.hpp"

namespace mdk {

// Two wavefronts per monomial when a worker fills a wavefront (worker width
// 64: orders 33 and up).  Wavefront B forms the backward chain while
// wavefront A forms the common factor; then at every forward step A forms
// f_j = f_{j-1} * x_{v_j} while B forms the cross product f_{j-1} * b_{k-j}
// of the same f_{j-1}, so the chain of dependent products shortens from
// 3k - 5 to about 2k - 2 and every monomial has two wavefronts to interleave.
// One workgroup of 128 threads per monomial, a workgroup barrier per step;
// the products are the single-wavefront routines of eval_monomial.
template <int L>
__device__ void eval_monomial_pair(const EvalArgs &a, int mono, double *buf0) {
  const int D = a.D, Dc = a.Dc, Dp = Dc + 1, G = 64;
  const int tid = threadIdx.x, lane = tid & 63;
  const bool isA = tid < 64;
  for (int q = tid; q < 6 * L; q += 128) buf0[(size_t)q * Dp + Dc] = 0.0;
  // one monomial per workgroup: its index range is uniform and kept in
  // scalar registers, so the index tables are read through the scalar cache
  // (not so in the kernels with several workers per wavefront)
  const int e0 = __builtin_amdgcn_readfirstlane(a.mon_ptr[mono]);
  const int k = __builtin_amdgcn_readfirstlane(a.mon_ptr[mono + 1]) - e0;
  const size_t nD = (size_t)a.n * D, mD = (size_t)a.m * D, zD = (size_t)a.nnz * D;
  const size_t xls = a.x_ls ? a.x_ls : nD;
  double c[L];
  ld<L>(a.cff, a.cff_ls ? a.cff_ls : (size_t)a.m, mono, c);
  if (k == 0) {  // constant monomial (the whole workgroup leaves)
    if (isA)
      for (int s = lane; s < Dc; s += G) {
#pragma unroll
        for (int l = 0; l < L; ++l) a.val[(size_t)l * mD + (size_t)mono * D + s] = (s == 0) ? c[l] : 0.0;
        if (a.vsize) a.vsize[(size_t)mono * D + s] = (s == 0) ? fabs(c[0]) : 0.0;
      }
    return;
  }
  auto xoff = [&](int v) { return (size_t)v * D; };
  auto der_off = [&](int j) { return (size_t)(e0 + j) * D; };
  const bool derivs = a.values_only == 0;
  double *U = buf0, *V = buf0 + (size_t)L * Dp, *W = buf0 + 2 * (size_t)L * Dp;  // A's buffers
  double *Bq = buf0 + 3 * (size_t)L * Dp, *Xq = buf0 + 4 * (size_t)L * Dp, *Wq = buf0 + 5 * (size_t)L * Dp;  // B's
  bool f0_scalar = true;
  for (int j = 0; j < k; ++j) f0_scalar = f0_scalar && a.exp[e0 + j] < 2;
  __syncthreads();
  if (!isA) {
    // backward chain: b_1 = x_{v_k}, b_q = b_{q-1} * x_{v_{k-q+1}}, parked in the slot of entry k - q - 1
    if (derivs && k >= 3) {
      double *B = Bq, *X = Xq, *Wb = Wq;
      load_series_t<L>(B, a.x, xls, xoff(a.var[e0 + k - 1]), Dc, lane, G);
      for (int q = 2; q <= k - 1; ++q) {
        load_series_t<L>(X, a.x, xls, xoff(a.var[e0 + k - q]), Dc, lane, G);
        wave_sync();
        conv_any<L>(B, X, Wb, Dc, lane, 1);
        wave_sync();
        store_series_t<L>(a.der, zD, der_off(k - q - 1), Wb, Dc, lane, G);
        double *t = B;
        B = Wb;
        Wb = t;
        wave_sync();
      }
    }
  } else if (!f0_scalar) {
    // common factor and f_0 = c * CF
    bool first = true;
    for (int j = 0; j < k; ++j) {
      const int p = a.exp[e0 + j] - 1;
      if (p < 1) continue;
      const int v = a.var[e0 + j];
      const double *src = (p == 1) ? a.x : a.pw + (size_t)(p - 2) * L * nD;
      const size_t sls = (p == 1) ? xls : nD;
      if (first) {
        load_series_t<L>(U, src, sls, xoff(v), Dc, lane, G);
        first = false;
        wave_sync();
      } else {
        load_series_t<L>(V, src, sls, xoff(v), Dc, lane, G);
        wave_sync();
        conv_any<L>(U, V, W, Dc, lane, 1);
        wave_sync();
        double *t = U;
        U = W;
        W = t;
      }
    }
    scal<L>(c, U, U, Dc, lane, G, 1);
    wave_sync();
  }
  // A's buffer rotation above happened in A only: share the result's place
  __shared__ int sh_u;
  if (tid == 0) sh_u = (int)((U - buf0) / ((size_t)L * Dp));
  __syncthreads();
  U = buf0 + (size_t)sh_u * L * Dp;
  V = buf0 + (size_t)((sh_u + 1) % 3) * L * Dp;
  W = buf0 + (size_t)((sh_u + 2) % 3) * L * Dp;
  const bool track = a.vsize != nullptr;
  double vmax[2] = {0.0, 0.0};
  auto track_max = [&](const double *F, bool scalar) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int s = lane + q * G;
      if (s < Dc) vmax[q] = fmax(vmax[q], scalar ? (s == 0 ? fabs(c[0]) : 0.0) : fabs(F[s]));
    }
  };
  if (track && isA) track_max(U, f0_scalar);
  // forward chain (A) beside the cross products (B)
  for (int j = 1; j <= k; ++j) {
    const int ej = j - 1;
    const int aj = a.exp[e0 + ej];
    if (isA) {
      load_series_t<L>(V, a.x, xls, xoff(a.var[e0 + ej]), Dc, lane, G);
      wave_sync();
      if (f0_scalar && j == 1)
        scal<L>(c, V, W, Dc, lane, G, 1);
      else
        conv_any<L>(U, V, W, Dc, lane, 1);
    } else if (derivs) {
      if (j < k) {
        if (k - j == 1)
          load_series_t<L>(Xq, a.x, xls, xoff(a.var[e0 + k - 1]), Dc, lane, G);  // b_1 = x_{v_k}
        else
          load_series_t<L>(Xq, a.der, zD, der_off(ej), Dc, lane, G);  // b_{k-j}
        wave_sync();
        if (f0_scalar && j == 1)
          scal<L>(c, Xq, Wq, Dc, lane, G, aj);
        else
          conv_any<L>(U, Xq, Wq, Dc, lane, aj);
        wave_sync();
        store_series_t<L>(a.der, zD, der_off(ej), Wq, Dc, lane, G);
      } else {  // d/dx_{v_k} = a_k f_{k-1}
        for (int s = lane; s < Dc; s += G) {
          double r[L];
#pragma unroll
          for (int l = 0; l < L; ++l) r[l] = (f0_scalar && j == 1) ? ((s == 0) ? c[l] : 0.0) : U[l * Dp + s];
          md::mul_int<L>(r, aj);
#pragma unroll
          for (int l = 0; l < L; ++l) a.der[(size_t)l * zD + der_off(ej) + s] = r[l];
        }
      }
    }
    __syncthreads();  // f_{j-1} read by both, f_j complete
    double *t = U;
    U = W;
    W = t;
    if (track && isA) track_max(U, false);
  }
  if (isA) {
    store_series_t<L>(a.val, mD, (size_t)mono * D, U, Dc, lane, G);
    if (track)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int s = lane + q * G;
        if (s < Dc) a.vsize[(size_t)mono * D + s] = vmax[q];
      }
  }
}

template <int L>
__global__ void __launch_bounds__(128) evaldiff_pair_kernel(EvalArgs a) {
  extern __shared__ double lds[];
  eval_monomial_pair<L>(a, __builtin_amdgcn_readfirstlane(a.order[blockIdx.x]), lds);
}

template <int L>
__global__ void __launch_bounds__(256, (L == 8) ? 1 : 2) evaldiff_kernel(EvalArgs a) {
  extern __shared__ double lds[];
  const int G = worker_lanes(a.Dc);
  const int wpb = blockDim.x / G;  // workers per block
  const int wid = threadIdx.x / G, lane = threadIdx.x - wid * G;
  const int widx = blockIdx.x * wpb + wid;
  if (widx >= a.m) return;  // whole worker exits together
  eval_monomial<L>(a, a.order[widx], lane, lds + (size_t)wid * 3 * L * (a.Dc + 1));
}

// Coefficient 0 of every derivative product (the entries of A_0), one
// thread per monomial, for supports of at most EVAL0_MAXK variables.  The
// same products as evaldiff_kernel restricted to the constant coefficients,
// which are plain multiple-double products: f_0 = c * CF(0), forward
// products f_j = f_{j-1} x_{v_j}(0) kept in registers, then the backward
// products b formed on the way back, d/dx_{v_j} = a_j f_{j-1} b_{k-j}.  The
// loads of the k constant coefficients are issued before the products, so
// the thread waits for memory once.
constexpr int EVAL0_MAXK = 8;

template <int L>
__global__ void __launch_bounds__(256) evaldiff0_kernel(EvalArgs a) {
  // it opens the factorization's chain, which runs beside the staged solve
  // and the evaluation: the highest issue priority on a shared CU
  __builtin_amdgcn_s_setprio(3);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  // the step's status word, reset by its first launch (every launch that can
  // report into it comes later in stream order; no evaluation kernel does)
  if (t == 0 && a.reset_status) *a.reset_status = MD_OK;
  // the monomial's support, exponents and coefficient do not depend on x:
  // their loads are issued before any wait for x
  const bool live = t < a.m;
  const int mono = live ? t : 0;
  int e0 = 0, k = 0;
  int vv[EVAL0_MAXK], ex[EVAL0_MAXK];
  double f[EVAL0_MAXK][L];  // f[j] = f_j for j < k (f_0 = c CF)
  if (live) {
    e0 = a.mon_ptr[mono];
    k = a.mon_ptr[mono + 1] - e0;
    ld<L>(a.cff, a.m, mono, f[0]);
  }
#pragma unroll
  for (int j = 0; j < EVAL0_MAXK; ++j) {
    vv[j] = 0;
    ex[j] = 1;
    if (j < k) {
      vv[j] = a.var[e0 + j];
      ex[j] = a.exp[e0 + j];
    }
  }
  if (a.wait_ctr) {
    __shared__ int ok;
    if (threadIdx.x == 0) ok = wait_count(a.wait_ctr, a.wait_target, a.wait_status) ? 1 : 0;
    __syncthreads();
    if (!ok) return;
  }
  if (!live || k == 0) return;  // k == 0: no derivatives
  const size_t nD = (size_t)a.n * a.D, zD = (size_t)a.nnz * a.D;
  double xs[EVAL0_MAXK][L];
#pragma unroll
  for (int j = 0; j < EVAL0_MAXK; ++j) {
    md::zero<L>(xs[j]);
    if (j < k) {
      if (a.wait_ctr) ld_agent<L>(a.x, nD, (size_t)vv[j] * a.D, xs[j]);
      else ld<L>(a.x, nD, (size_t)vv[j] * a.D, xs[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < EVAL0_MAXK; ++j) {  // common factor: x^(a-1) for exponents >= 2
    if (j < k)
      for (int p = 1; p < ex[j]; ++p) {
        double r[L];
        MD<L>::mul(f[0], xs[j], r);
        md::copy<L>(r, f[0]);
      }
  }
#pragma unroll
  for (int j = 1; j < EVAL0_MAXK; ++j)
    if (j < k) MD<L>::mul(f[j - 1], xs[j - 1], f[j]);
  double b[L];  // backward product b_{k-j}, b_0 = 1
  md::zero<L>(b);
  b[0] = 1.0;
#pragma unroll
  for (int j = EVAL0_MAXK; j >= 1; --j) {
    if (j > k) continue;
    double d[L];
    if (j == k) md::copy<L>(f[j - 1], d);
    else MD<L>::mul(f[j - 1], b, d);
    md::mul_int<L>(d, ex[j - 1]);
#pragma unroll
    for (int l = 0; l < L; ++l) a.der[(size_t)l * zD + (size_t)(e0 + j - 1) * a.D] = d[l];
    if (j > 1) {
      double r[L];
      if (j == k) md::copy<L>(xs[j - 1], r);
      else MD<L>::mul(b, xs[j - 1], r);
      md::copy<L>(r, b);
    }
  }
}

hipError_t launch_evaldiff0(int L, const EvalArgs &a, hipStream_t st) {
  // one wavefront per workgroup: the few thousand monomials spread over as
  // many CUs as possible (each thread is a chain of dependent products)
  const dim3 grid((a.m + 63) / 64);
  switch (L) {
    case 1: hipLaunchKernelGGL(evaldiff0_kernel<1>, grid, dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL(evaldiff0_kernel<2>, grid, dim3(64), 0, st, a); break;
    case 4: hipLaunchKernelGGL(evaldiff0_kernel<4>, grid, dim3(64), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Octo doubles would spill the registers of this kernel: they take the
// general kernel with one coefficient.
int evaldiff0_max_support(int L) { return L <= 4 ? EVAL0_MAXK : 0; }

// Powers x_v^p, p = 2..maxexp-1, for the common factors of exponents >= 3.
template <int L>
__global__ void __launch_bounds__(256, (L == 8) ? 1 : 2) power_kernel(int n, int D, int Dc, int maxp, const double *x, double *pw) {
  extern __shared__ double lds[];
  const int G = worker_lanes(Dc);
  const int wpb = blockDim.x / G;
  const int wid = threadIdx.x / G, lane = threadIdx.x - wid * G;
  const int v = blockIdx.x * wpb + wid;
  if (v >= n) return;
  double *U = lds + (size_t)wid * 3 * L * (Dc + 1), *X = U + L * (Dc + 1), *W = X + L * (Dc + 1);
  zero_pads(U, L, Dc, lane, G);
  const size_t nD = (size_t)n * D;
  load_series_t<L>(X, x, nD, (size_t)v * D, Dc, lane, G);
  load_series_t<L>(U, x, nD, (size_t)v * D, Dc, lane, G);
  wave_sync();
  for (int p = 2; p <= maxp; ++p) {
    conv_any<L>(U, X, W, Dc, lane, 1);
    wave_sync();
    store_series_t<L>(pw + (size_t)(p - 2) * L * nD, nD, (size_t)v * D, W, Dc, lane, G);
    double *t = U;
    U = W;
    W = t;
    wave_sync();
  }
}

// ------------------------------------------------------------------ launchers

template <int L>
hipError_t launch_evaldiff_T(const EvalArgs &a, int maxexp, double *pw_mut, hipStream_t st) {
  const int G = worker_lanes(a.Dc);
  const int wpb = 256 / G;
  const size_t lds = (size_t)wpb * 3 * L * (a.Dc + 1) * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {  // dynamic LDS above 64 KB needs the attribute
    (void)hipFuncSetAttribute((const void *)power_kernel<L>, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)hipFuncSetAttribute((const void *)evaldiff_kernel<L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              150 * 1024);
    (void)hipGetLastError();  // an attribute the runtime refuses must not be reported by the launch
    attr_set = true;
  }
  if (maxexp >= 3) {
    const int blocks = (a.n + wpb - 1) / wpb;
    hipLaunchKernelGGL(power_kernel<L>, dim3(blocks), dim3(256), lds, st, a.n, a.D, a.Dc, maxexp - 1, a.x, pw_mut);
  }
  if (a.m > 0) {
    if (G == 64 && !a.beside_qr) {  // two wavefronts per monomial
      hipLaunchKernelGGL(evaldiff_pair_kernel<L>, dim3(a.m), dim3(128), (size_t)6 * L * (a.Dc + 1) * sizeof(double),
                         st, a);
    } else {
      const int blocks = (a.m + wpb - 1) / wpb;
      hipLaunchKernelGGL(evaldiff_kernel<L>, dim3(blocks), dim3(256), lds, st, a);
    }
  }
  return hipGetLastError();
}

hipError_t launch_evaldiff(int L, const EvalArgs &a, int maxexp, double *pw, hipStream_t st) {
  switch (L) {
    case 1: return launch_evaldiff_T<1>(a, maxexp, pw, st);
    case 2: return launch_evaldiff_T<2>(a, maxexp, pw, st);
    case 4: return launch_evaldiff_T<4>(a, maxexp, pw, st);
    case 8: return launch_evaldiff_T<8>(a, maxexp, pw, st);
  }
  return hipErrorInvalidValue;
}

int evaldiff_workers_per_block(int D) { return worker_lanes(D) == 64 ? 1 : 256 / worker_lanes(D); }

size_t evaldiff_lds_bytes(int L, int D) {
  const int G = worker_lanes(D);
  return (size_t)(256 / G) * 3 * L * (D + 1) * sizeof(double);
}

}  // namespace mdk
