// Device routines of the evaluation and differentiation by convolutions,
// shared by the single-system kernels (evaldiff.hip) and the batched Newton
// step (batch.hip).  The method and the work decomposition are described at
// the top of evaldiff.hip.
#pragma once
#include "common.hpp"
#include "kernels.hpp"

namespace mdk {

// Lanes per output pair (S) and per half (G2) of a worker for D coefficients.
__host__ __device__ inline int pair_lanes(int D) {
  int h = (D + 1) / 2, g = 1;
  while (g < h) g <<= 1;
  return g;
}
__host__ __device__ inline int split_factor(int D) { return 2 * pair_lanes(D) <= 64 ? 2 : 1; }
__host__ __device__ inline int worker_lanes(int D) { return split_factor(D) * pair_lanes(D); }

// LDS series layout: [L][D + 1]; entry D of every limb is zero and is what
// masked terms read.

// Truncated product W = scale * (U * V) (all in LDS).  DP > 0: the buffers'
// limb stride D + 1 known at compile time (the limb offsets of the LDS reads
// become immediates); the operand pointers move by one entry per term.
template <int L, int DP = 0>
__device__ void conv(const double *U, const double *V, double *W, int D, int lane, int scale) {
  const int Dp = DP > 0 ? DP : D + 1, G2 = pair_lanes(D), S = split_factor(D);
  const int h = lane / G2, p = lane - h * G2;
  const bool act = p < (D + 1) / 2;
  const int o1 = p, o2 = D - 1 - p;
  const int H = (D + S) / S;  // terms per half: ceil((D + 1) / S)
  const int t0 = h * H;
  // acc0 accumulates the current output; the first one's level sums are
  // parked in acc1 when its last term is in (a different iteration in
  // every lane) and renormalized after the loop, by all lanes together
  double acc0[L], acc1[L];
  md::zero<L>(acc0);
  md::zero<L>(acc1);
  // term t multiplies u_i v_j with i + j = o1 for t <= o1 and i + j = o2
  // after (i = t - o1 - 1); masked terms read the zero padding (entry D)
  int i, j;
  {
    const bool ph1 = t0 <= o1;
    i = ph1 ? t0 : t0 - o1 - 1;
    j = (ph1 ? o1 : o2) - i;
    if (!act || t0 > D) {
      i = D;
      j = 0;
    }
  }
  for (int tt = 0; tt < H; ++tt) {
    const int t = t0 + tt;
    double u[L], v[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      u[l] = U[l * Dp + i];
      v[l] = V[l * Dp + j];
    }
    // the next term's indices
    if (t == o1) {
      i = 0;
      j = o2;
    } else {
      ++i;
      --j;
    }
    if (!act || t + 1 > D) {
      i = D;
      j = 0;
    }
    MD<L>::fma_lazy(acc0, u, v);
    if (t == o1) {  // first output complete (always in the first half)
      md::copy<L>(acc0, acc1);
      md::zero<L>(acc0);
    }
  }
  if (h == 0 && act) {
    double r[L];
    MD<L>::renorm(acc1, r);
    md::mul_int<L>(r, scale);
#pragma unroll
    for (int l = 0; l < L; ++l) W[l * Dp + o1] = r[l];
  }
  if (S == 2) {  // add the second half's part of the second output, still as level sums
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
    for (int l = 0; l < L; ++l) W[l * Dp + o2] = r[l];
  }
}

// conv with the limb stride fixed at compile time for the orders of the
// workloads (16, 32, 64, 128 coefficients), the runtime stride otherwise.
template <int L>
__device__ __forceinline__ void conv_any(const double *U, const double *V, double *W, int D, int lane, int scale) {
  switch (D) {
    case 16: conv<L, 17>(U, V, W, D, lane, scale); break;
    case 32: conv<L, 33>(U, V, W, D, lane, scale); break;
    case 64: conv<L, 65>(U, V, W, D, lane, scale); break;
    case 128: conv<L, 129>(U, V, W, D, lane, scale); break;
    default: conv<L>(U, V, W, D, lane, scale);
  }
}

// W = scale * c * V for a scalar c (registers) and a series V.
template <int L>
__device__ void scal(const double (&c)[L], const double *V, double *W, int D, int lane, int G, int scale) {
  const int Dp = D + 1;
  for (int s = lane; s < D; s += G) {
    double v[L], r[L];
#pragma unroll
    for (int l = 0; l < L; ++l) v[l] = V[l * Dp + s];
    MD<L>::mul(c, v, r);
    md::mul_int<L>(r, scale);
#pragma unroll
    for (int l = 0; l < L; ++l) W[l * Dp + s] = r[l];
  }
}

// LDS <- global series (limb stride gstride, element offset off), D entries.
__device__ __forceinline__ void load_series(double *S, const double *g, size_t gstride, size_t off, int L, int D,
                                            int lane, int G) {
  for (int q = lane; q < L * D; q += G) {
    const int l = q / D, s = q - l * D;
    S[l * (D + 1) + s] = g[(size_t)l * gstride + off + s];
  }
}

__device__ __forceinline__ void store_series(double *g, size_t gstride, size_t off, const double *S, int L, int D,
                                             int lane, int G) {
  for (int q = lane; q < L * D; q += G) {
    const int l = q / D, s = q - l * D;
    g[(size_t)l * gstride + off + s] = S[l * (D + 1) + s];
  }
}

// The same with the limb count known at compile time: lane takes the
// coefficients s = lane + c G, every limb of each, and issues all loads of a
// block of two coefficients per lane before it writes any of them to LDS, so
// a series costs one round trip to memory instead of one per element (and no
// integer division).
template <int L>
__device__ __forceinline__ void load_series_t(double *S, const double *g, size_t gstride, size_t off, int D, int lane,
                                              int G) {
  for (int s0 = 0; s0 < D; s0 += 2 * G) {
    double r[2][L];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int s = s0 + lane + c * G;
#pragma unroll
      for (int l = 0; l < L; ++l) r[c][l] = s < D ? g[(size_t)l * gstride + off + s] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int s = s0 + lane + c * G;
      if (s < D)
#pragma unroll
        for (int l = 0; l < L; ++l) S[l * (D + 1) + s] = r[c][l];
    }
  }
}

template <int L>
__device__ __forceinline__ void store_series_t(double *g, size_t gstride, size_t off, const double *S, int D, int lane,
                                               int G) {
  for (int s = lane; s < D; s += G)
#pragma unroll
    for (int l = 0; l < L; ++l) g[(size_t)l * gstride + off + s] = S[l * (D + 1) + s];
}

// Zero the padding entries of a worker's three buffers.
__device__ __forceinline__ void zero_pads(double *buf0, int L, int D, int lane, int G) {
  for (int q = lane; q < 3 * L; q += G) buf0[q * (D + 1) + D] = 0.0;
}

// One worker (G lanes of one wavefront, worker_lanes(a.Dc) of them) evaluates
// and differentiates monomial `mono` with the three LDS series buffers at
// buf0 (3 L (Dc + 1) doubles).  The products are described at the top of
// evaldiff.hip.
template <int L>
__device__ void eval_monomial(const EvalArgs &a, int mono, int lane, double *buf0) {
  const int D = a.D;    // coefficients stored per series (global stride)
  const int Dc = a.Dc;  // coefficients computed: the order of a truncated problem (1: the A_0 pre-pass)
  const int G = worker_lanes(Dc);
  const int Dp = Dc + 1;
  double *buf[3] = {buf0, buf0 + L * Dp, buf0 + 2 * L * Dp};
  zero_pads(buf[0], L, Dc, lane, G);
  const int e0 = a.mon_ptr[mono], k = a.mon_ptr[mono + 1] - e0;
  const size_t nD = (size_t)a.n * D, mD = (size_t)a.m * D, zD = (size_t)a.nnz * D;
  const size_t xls = a.x_ls ? a.x_ls : nD;  // limb stride of x
  double c[L];
  ld<L>(a.cff, a.cff_ls ? a.cff_ls : (size_t)a.m, mono, c);

  if (k == 0) {  // constant monomial
    for (int s = lane; s < Dc; s += G) {
#pragma unroll
      for (int l = 0; l < L; ++l) a.val[(size_t)l * mD + (size_t)mono * D + s] = (s == 0) ? c[l] : 0.0;
      if (a.vsize) a.vsize[(size_t)mono * D + s] = (s == 0) ? fabs(c[0]) : 0.0;
    }
    return;
  }
  auto xoff = [&](int v) { return (size_t)v * D; };
  auto der_off = [&](int j) { return (size_t)(e0 + j) * D; };  // j: 0-based entry

  const bool derivs = a.values_only == 0;
  // ---- backward chain: b_q for q = 2..k-1 parked in the slot of entry k-q (0-based k-q-1+... )
  if (derivs && k >= 3) {
    double *B = buf[0], *X = buf[1], *Wb = buf[2];
    load_series_t<L>(B, a.x, xls, xoff(a.var[e0 + k - 1]), Dc, lane, G);  // b_1 = x_{v_k}
    for (int q = 2; q <= k - 1; ++q) {
      load_series_t<L>(X, a.x, xls, xoff(a.var[e0 + k - q]), Dc, lane, G);  // x_{v_{k-q+1}}
      wave_sync();
      conv_any<L>(B, X, Wb, Dc, lane, 1);
      wave_sync();
      // b_q is consumed by the cross product of forward step j = k - q (1-based),
      // i.e. entry k - q - 1 (0-based)
      store_series_t<L>(a.der, zD, der_off(k - q - 1), Wb, Dc, lane, G);
      double *t = B;
      B = Wb;
      Wb = t;
      wave_sync();
    }
  }

  // ---- common factor and f_0
  double *U = buf[0], *V = buf[1], *W = buf[2];
  bool f0_scalar = true;
  for (int j = 0; j < k; ++j) {
    const int p = a.exp[e0 + j] - 1;
    if (p < 1) continue;
    const int v = a.var[e0 + j];
    const double *src = (p == 1) ? a.x : a.pw + (size_t)(p - 2) * L * nD;
    const size_t sls = (p == 1) ? xls : nD;
    if (f0_scalar) {
      load_series_t<L>(U, src, sls, xoff(v), Dc, lane, G);
      f0_scalar = false;
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
  if (!f0_scalar) {  // f_0 = c * CF in place
    scal<L>(c, U, U, Dc, lane, G, 1);
    wave_sync();
  }
  // With vsize: the largest |f_j| of the forward chain at each coefficient
  // (a lane owns s = lane and s = lane + G; G >= Dc / 2 for Dc <= 128): the
  // size of the terms whose rounding errors reach the value.
  const bool track = a.vsize != nullptr;
  double vmax[2] = {0.0, 0.0};
  auto track_max = [&](const double *F, bool scalar) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int s = lane + q * G;
      if (s < Dc) vmax[q] = fmax(vmax[q], scalar ? (s == 0 ? fabs(c[0]) : 0.0) : fabs(F[s]));
    }
  };
  if (track) track_max(U, f0_scalar);

  // ---- forward chain with the cross products
  for (int j = 1; j <= k; ++j) {
    const int ej = j - 1;  // 0-based entry of v_j
    const int aj = a.exp[e0 + ej];
    if (!derivs) {
      // values only: the forward product below
    } else if (j < k) {
      if (k - j == 1)
        load_series_t<L>(V, a.x, xls, xoff(a.var[e0 + k - 1]), Dc, lane, G);  // b_1 = x_{v_k}
      else
        load_series_t<L>(V, a.der, zD, der_off(ej), Dc, lane, G);  // b_{k-j}
      wave_sync();
      if (f0_scalar && j == 1)
        scal<L>(c, V, W, Dc, lane, G, aj);
      else
        conv_any<L>(U, V, W, Dc, lane, aj);
      wave_sync();
      store_series_t<L>(a.der, zD, der_off(ej), W, Dc, lane, G);
    } else {  // d/dx_{v_k} = a_k f_{k-1}
      if (f0_scalar && j == 1) {
        for (int s = lane; s < Dc; s += G) {
          double r[L];
#pragma unroll
          for (int l = 0; l < L; ++l) r[l] = (s == 0) ? c[l] : 0.0;
          md::mul_int<L>(r, aj);
#pragma unroll
          for (int l = 0; l < L; ++l) a.der[(size_t)l * zD + der_off(ej) + s] = r[l];
        }
      } else {
        for (int s = lane; s < Dc; s += G) {
          double r[L];
#pragma unroll
          for (int l = 0; l < L; ++l) r[l] = U[l * Dp + s];
          md::mul_int<L>(r, aj);
#pragma unroll
          for (int l = 0; l < L; ++l) a.der[(size_t)l * zD + der_off(ej) + s] = r[l];
        }
      }
    }
    wave_sync();
    // f_j = f_{j-1} * x_{v_j}
    load_series_t<L>(V, a.x, xls, xoff(a.var[e0 + ej]), Dc, lane, G);
    wave_sync();
    if (f0_scalar && j == 1)
      scal<L>(c, V, W, Dc, lane, G, 1);
    else
      conv_any<L>(U, V, W, Dc, lane, 1);
    wave_sync();
    double *t = U;
    U = W;
    W = t;
    if (track) track_max(U, false);
  }
  store_series_t<L>(a.val, mD, (size_t)mono * D, U, Dc, lane, G);
  if (track)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int s = lane + q * G;
      if (s < Dc) a.vsize[(size_t)mono * D + s] = vmax[q];
    }
}


}  // namespace mdk
