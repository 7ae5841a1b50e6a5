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
// A_{m-k+1} dx_{k-1}.  Every stage is one launch over the whole GPU; for
// n <= 64 in double and quad double one persistent launch runs all stages
// with the recurrence reassociated further (stages_persistent_kernel).
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace mdk {

// ----------------------------------------------------------------- status

__global__ void status_init_kernel(int32_t *status, int *counter, int *counter2) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && status) *status = MD_OK;
  if (threadIdx.x == 0 && blockIdx.x == 0 && counter) *counter = 0;
  if (threadIdx.x == 0 && blockIdx.x == 0 && counter2) *counter2 = 0;
}

// ----------------------------------------------------------------- QR

// Householder reflector of a column with squared norm nrm2 and leading entry
// x0: beta = -sign(x0) ||x|| (sign(0) = +1), v = x / (x0 - beta) with v_0 = 1,
// tau = (beta - x0) / beta.  Division-free: y = 1/||x|| and 1/(x0 - beta) by
// the shortened Newton doublings (the reflector is on the chain of every
// column of the factorization).
template <int L>
__device__ void reflector(const double (&nrm2)[L], const double (&x0)[L], double (&beta)[L], double (&tau)[L],
                          double (&inv)[L]) {
  double y[L];
  md::rsqrt_short<L>(nrm2, y);
  double alpha[L], v0[L];
  MD<L>::mul(nrm2, y, alpha);  // ||x||
  const bool nonneg = x0[0] >= 0.0;
  if (nonneg) md::neg<L>(alpha, beta);
  else md::copy<L>(alpha, beta);
  MD<L>::sub(x0, beta, v0);
  MD<L>::mul(v0, y, tau);      // tau = -v0 / beta and 1/beta = -+ y
  if (!nonneg) md::neg<L>(tau, tau);
  md::recip_short<L>(v0, inv);
}

// Unblocked Householder QR in one workgroup of 1024 threads; a [L][n][n]
// row-major in place (R on and above the diagonal, v below it).  When qt is
// not null it starts as the identity and receives every reflector too, so it
// ends as Q^T = H_{n-1} ... H_0 (the augmented matrix [A_0 | I]).  The trailing
// update gives each column to a team of 16 lanes.
template <int L> struct QrThreads {
  static constexpr int value = 256;
};

// Grid-wide barrier among the workgroups of one launch: a monotone counter
// in device memory, agent-scope release/acquire.  The spin is bounded; on
// time-out the launch records MD_EHIP in the status word and the caller's
// result is garbage (every workgroup still exits).
__device__ __forceinline__ bool grid_barrier(unsigned *counter, unsigned target, int32_t *status) {
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 1;
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    // relaxed polling (an acquire load would invalidate the caches on every
    // poll), one acquire fence once the count is reached
    long spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1L << 22)) {
        set_status(status, MD_EHIP);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
}

__global__ void zero_u32_kernel(unsigned *p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}

// Householder QR of A_0 by G workgroups (a [L][n][n] row-major in place, R
// on and above the diagonal, v below it).  For every column c each workgroup
// computes the same reflector from the same data, so no workgroup waits for
// another to publish it; the columns of the trailing matrix are dealt out
// cyclically (column j to workgroup j mod G), each to a team of 16 lanes.  When
// qt is not null it starts as the identity and receives every reflector too,
// ending as Q^T = H_{n-1} ... H_0 (the augmented matrix [A_0 | I]).  One grid
// barrier per column makes the updated column c+1 visible to all.
template <int L>
__global__ void __launch_bounds__(256) qr_kernel(int n, double *a, double *tau, double *qt, int32_t *status,
                                                 unsigned *bar) {
  extern __shared__ double vsh[];  // the current reflector v, [L][n]
  __shared__ double red[4][L];
  __shared__ double sh_tau[L], sh_inv[L], sh_beta[L];
  __shared__ int sh_skip;
  constexpr int T = 16;
  const size_t nn = (size_t)n * n;
  const int G = gridDim.x, g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  const int team = tid / T, tl = tid % T, nteams = blockDim.x / T;
  if (qt)  // columns of Q^T owned by this workgroup start as the identity
    for (int j = g; j < n; j += G)
      for (int i = tid; i < n; i += blockDim.x) {
#pragma unroll
        for (int l = 0; l < L; ++l) qt[(size_t)l * nn + (size_t)i * n + j] = (l == 0 && i == j) ? 1.0 : 0.0;
      }
  bool alive = true;
  for (int c = 0; c < n && alive; ++c) {
    // squared norm of column c, rows c..n-1
    double acc[L];
    md::zero<L>(acc);
    for (int i = c + tid; i < n; i += blockDim.x) {
      double xi[L];
      ld<L>(a, nn, (size_t)i * n + c, xi);
      MD<L>::fma(acc, xi, xi);
    }
    if (n - c <= 64) {  // one wavefront holds the whole column
      if (w == 0) team_sum<L>(acc, 64);
    } else {
      team_sum<L>(acc, 64);
      if (lane == 0)
#pragma unroll
        for (int l = 0; l < L; ++l) red[w][l] = acc[l];
      __syncthreads();
      if (w == 0) {
#pragma unroll
        for (int l = 0; l < L; ++l) acc[l] = (lane < nw) ? red[lane][l] : 0.0;
        team_sum<L>(acc, 64);
      }
    }
    if (tid == 0) {
      double x0[L];
      ld<L>(a, nn, (size_t)c * n + c, x0);
      if (!(acc[0] > 0.0)) {  // zero column: R_cc = 0, H_c = I
        sh_skip = 1;
#pragma unroll
        for (int l = 0; l < L; ++l) sh_beta[l] = x0[l];
        if (g == 0) {
#pragma unroll
          for (int l = 0; l < L; ++l) tau[(size_t)l * n + c] = 0.0;
          set_status(status, MD_ESINGULAR);
        }
      } else {
        double beta[L], tc[L], inv[L];
        reflector<L>(acc, x0, beta, tc, inv);
        sh_skip = 0;
        if (g == 0) st<L>(tau, n, c, tc);
#pragma unroll
        for (int l = 0; l < L; ++l) {
          sh_tau[l] = tc[l];
          sh_inv[l] = inv[l];
          sh_beta[l] = beta[l];
        }
      }
    }
    __syncthreads();
    const bool skip = sh_skip != 0;
    double inv[L], tc[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      inv[l] = sh_inv[l];
      tc[l] = sh_tau[l];
    }
    for (int i = c + tid; i < n; i += blockDim.x) {
      double vi[L];
      if (i == c) {
        md::zero<L>(vi);
        vi[0] = 1.0;
      } else if (skip) {
        md::zero<L>(vi);
      } else {
        double xi[L];
        ld<L>(a, nn, (size_t)i * n + c, xi);
        MD<L>::mul(xi, inv, vi);
      }
#pragma unroll
      for (int l = 0; l < L; ++l) vsh[l * n + i] = vi[l];
    }
    __syncthreads();
    if (!skip) {
      // this workgroup's trailing columns of A (j > c, j mod G == g) and of Q^T (j mod G == g)
      const int first_a = c + 1 + ((g - (c + 1)) % G + G) % G;
      const int na = (first_a < n) ? (n - 1 - first_a) / G + 1 : 0;
      const int nq = qt ? ((g < n) ? (n - 1 - g) / G + 1 : 0) : 0;
      for (int col = team; col < na + nq; col += nteams) {
        double *base = (col < na) ? a : qt;
        const int j = (col < na) ? first_a + col * G : g + (col - na) * G;
        double dot[L];
        md::zero<L>(dot);
        for (int i = c + tl; i < n; i += T) {
          double vi[L], x[L];
#pragma unroll
          for (int l = 0; l < L; ++l) vi[l] = vsh[l * n + i];
          ld<L>(base, nn, (size_t)i * n + j, x);
          MD<L>::fma(dot, vi, x);
        }
        team_sum<L>(dot, T);
        double wj[L];
        MD<L>::mul(dot, tc, wj);
        for (int i = c + tl; i < n; i += T) {
          double vi[L], x[L];
#pragma unroll
          for (int l = 0; l < L; ++l) vi[l] = vsh[l * n + i];
          ld<L>(base, nn, (size_t)i * n + j, x);
          MD<L>::fms(x, vi, wj);
          st<L>(base, nn, (size_t)i * n + j, x);
        }
      }
    }
    // every workgroup has read column c: workgroup 0 may now store R_cc and v
    alive = grid_barrier(bar, (unsigned)G * (unsigned)(c + 1), status);
    if (g == 0) {
      for (int i = c + tid; i < n; i += blockDim.x) {
        double vi[L];
        if (i == c) {
#pragma unroll
          for (int l = 0; l < L; ++l) vi[l] = sh_beta[l];
        } else {
#pragma unroll
          for (int l = 0; l < L; ++l) vi[l] = vsh[l * n + i];
        }
        st<L>(a, nn, (size_t)i * n + c, vi);
      }
    }
  }
}

// Lanes of a butterfly over `rows` values held one per lane from lane 0
// (at most 64; more rows than lanes use all 64): the smallest power of two
// that covers them, so that short columns take fewer levels.
__device__ __forceinline__ int red_width(int rows) {
  int w = 1;
  while (w < rows && w < 64) w <<= 1;
  return w;
}

// Bounded wait for a published flag (agent scope).  Returns false on time-out
// (the status word then holds MD_EHIP and the caller's result is garbage).
// The flag is polled with relaxed loads and a short sleep (an acquire load
// would invalidate the caches on every poll, and a busy loop takes issue
// slots from the waves sharing the CU); one acquire fence follows, so that
// the board is then read with plain loads.  The writer stores the board
// with agent-scope stores and waits for them before raising the flag: a
// release fence would write back the whole L2 of its chiplet at every
// column, and beside the evaluation that L2 holds megabytes of its output.
__device__ __forceinline__ bool wait_flag(const int *flag, int32_t *status, int target = 1) {
  long spins = 0;
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > (1L << 22)) {
      set_status(status, MD_EHIP);
      return false;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Consecutive columns of [A_0 | I] owned by one workgroup of the LDS QR.
constexpr int QR_GROUP = 2;

// Householder QR of A_0 with Q^T, columns resident in LDS.  Column J of the
// augmented matrix [A_0 | I] (J < 2n) belongs to workgroup (J / QR_GROUP) mod G and
// stays in its LDS for the whole factorization.  Reflector c is published by
// the owner of column c in two parts: first the column x below the diagonal
// as it is (flags[c] = 1), then, after its norm and the reflector scalars,
// tau and 1/(x_0 - beta) into slots that an earlier launch on the stream
// emptied (QrPrep), which the readers poll themselves: one round trip, and
// no wait for the stores on the owner's chain.  With v = x / (x_0 - beta) below the
// diagonal and v_c = 1, H_c y = y - tau (v^T y) v needs of y only
//     S = sum_{i>c} x_i y_i,  d = y_c + S / (x_0 - beta),
// so every workgroup forms S for all its columns from the first part while
// the owner still computes the scalars, and the second part only leaves one
// multiply-add per row: y_c -= tau d, y_i -= (tau d / (x_0 - beta)) x_i.  The
// owner of column c+1 updates that column first and publishes reflector c+1
// from one wavefront while its other wavefronts update the rest (look-ahead).
// Every column is written back at the end: R on and above the diagonal, v
// below it for the A_0 part; Q^T for the identity part.
template <int L>
__global__ void __launch_bounds__(256) qr_lds_kernel(int n, double *a, double *tau, double *qt, int32_t *status,
                                                     int *flags, double *vboard, double *tboard) {
  extern __shared__ double lds[];
  // this launch runs beside the evaluation kernel and is on the critical
  // path: its wavefronts get the highest issue priority on a shared CU
  __builtin_amdgcn_s_setprio(3);
  const int G = gridDim.x, g = blockIdx.x;
  const int ncols_total = qt ? 2 * n : n;  // [A_0 | I] or A_0 alone
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int T = 16;
  const int team = tid / T, tl = tid % T;
  const size_t nn = (size_t)n * n;
  // columns are owned in groups of QR_GROUP: J belongs to workgroup
  // (J / QR_GROUP) mod G, so that of QR_GROUP consecutive reflectors all but
  // the first are used by the workgroup that computed them, from its LDS,
  // without a hand-over
  constexpr int OG = QR_GROUP;
  auto owner = [&](int J) { return (J / OG) % G; };
  auto gcol = [&](int q) { return OG * (g + (q / OG) * G) + (q % OG); };  // local index -> J
  auto lcol = [&](int J) { return OG * ((J / OG) / G) + (J % OG); };       // J -> local index
  int ncol = 0;
  while (gcol(ncol) < ncols_total) ++ncol;
  double *cols = lds;                          // [ncol][L][n]
  double *vsh = lds + (size_t)ncol * L * n;    // [L][n] column c below the diagonal (another workgroup's)
  double *own_inv = vsh + (size_t)L * n;       // [ncol][L] 1 / (x_0 - beta) of the owned columns
  double *ssum = own_inv + (size_t)ncol * L;   // [ncol][L] S of every owned column for the current reflector
  __shared__ double sh_tau[L], sh_inv[L], sh_tau_own[L];
  __shared__ int sh_ok;
  auto col = [&](int q) { return cols + (size_t)q * L * n; };
  // load the owned columns of [A_0 | I]
  for (int q = 0; q < ncol; ++q) {
    const int J = gcol(q);
    double *cq = col(q);
    for (int i = tid; i < n; i += blockDim.x)
#pragma unroll
      for (int l = 0; l < L; ++l)
        cq[l * n + i] = (J < n) ? a[(size_t)l * nn + (size_t)i * n + J] : ((l == 0 && i == J - n) ? 1.0 : 0.0);
  }
  __syncthreads();

  // reflector of owned column q (global column c), by one wavefront: the
  // column below the diagonal to the board and flags[c] = 1, its norm, the
  // scalars (beta into the column as R_cc), tau and 1 / (x_0 - beta) into
  // their slots
  auto publish = [&](int q, int c) {
    double *cq = col(q);
    for (int i = c + 1 + lane; i < n; i += 64) {
      double xi[L];
#pragma unroll
      for (int l = 0; l < L; ++l) xi[l] = cq[l * n + i];
      st_agent<L>(vboard + (size_t)c * L * n, n, i, xi);
    }
    double acc[L];
    {
      double u[L];
      md::zero<L>(u);
      for (int i = c + lane; i < n; i += 64) {
        double xi[L];
#pragma unroll
        for (int l = 0; l < L; ++l) xi[l] = cq[l * n + i];
        MD<L>::fma_lazy(u, xi, xi);
      }
      team_sum_lazy<L>(u, red_width(n - c));
      MD<L>::renorm(u, acc);
    }
    if (lane == 0) {
      wait_vm();  // the board stores are performed before the flag
      __hip_atomic_store(&flags[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    double x0[L], beta[L], tc[L], inv[L];
#pragma unroll
    for (int l = 0; l < L; ++l) x0[l] = cq[l * n + c];
    const bool zero = !(acc[0] > 0.0);
    if (zero) {
      md::copy<L>(x0, beta);
      md::zero<L>(tc);
      md::zero<L>(inv);
      if (lane == 0) set_status(status, MD_ESINGULAR);
    } else {
      reflector<L>(acc, x0, beta, tc, inv);  // every lane computes the same scalars
    }
    if (lane == 0) {
#pragma unroll
      for (int l = 0; l < L; ++l) {
        __hip_atomic_store(&tboard[(size_t)c * 2 * L + l], tc[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&tboard[(size_t)c * 2 * L + L + l], inv[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tau[(size_t)l * n + c] = tc[l];
        sh_tau_own[l] = tc[l];
        own_inv[q * L + l] = inv[l];
        cq[l * n + c] = beta[l];  // R_cc
      }
    }
    wave_sync();
  };

  // S = sum_{i>c} x_i y_i for owned column q (x in xs), team of `width` lanes
  auto partial_dot = [&](int q, int c, const double *xs, int tlane, int width, double (&S)[L]) {
    const double *cq = col(q);
    double u[L];
    md::zero<L>(u);
    for (int i = c + 1 + tlane; i < n; i += width) {
      double xi[L], y[L];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        xi[l] = xs[l * n + i];
        y[l] = cq[l * n + i];
      }
      MD<L>::fma_lazy(u, xi, y);
    }
    team_sum_lazy<L>(u, width == 64 ? red_width(n - c - 1) : width);
    MD<L>::renorm(u, S);
  };

  // H_c on owned column q given its S (tau tc, 1 / (x_0 - beta) inv)
  auto finish_apply = [&](int q, int c, const double *xs, const double (&S)[L], const double (&tc)[L],
                          const double (&inv)[L], int tlane, int width) {
    double *cq = col(q);
    double yc[L], t[L], d[L], wj[L], wi[L];
#pragma unroll
    for (int l = 0; l < L; ++l) yc[l] = cq[l * n + c];
    MD<L>::mul(S, inv, t);
    MD<L>::add(yc, t, d);
    MD<L>::mul(d, tc, wj);
    MD<L>::mul(wj, inv, wi);
    if (tlane == 0) {
      double r[L];
      MD<L>::sub(yc, wj, r);
#pragma unroll
      for (int l = 0; l < L; ++l) cq[l * n + c] = r[l];
    }
    for (int i = c + 1 + tlane; i < n; i += width) {
      double xi[L], y[L];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        xi[l] = xs[l * n + i];
        y[l] = cq[l * n + i];
      }
      MD<L>::fms(y, xi, wi);
#pragma unroll
      for (int l = 0; l < L; ++l) cq[l * n + i] = y[l];
    }
  };

  if (g == 0 && w == 0) publish(0, 0);  // column 0 belongs to workgroup 0
  bool ok = true;
  int q0 = 0;  // owned columns J <= c: a prefix of the local order
  for (int c = 0; c < n; ++c) {
    const bool own = owner(c) == g;
    // 1. the column below the diagonal: this workgroup's own, or from the board
    if (!own) {
      if (tid == 0) sh_ok = wait_flag(&flags[c], status, 1) ? 1 : 0;
      __syncthreads();
      if (!sh_ok) {
        ok = false;
        break;
      }
      for (int e = c + 1 + tid; e < n; e += blockDim.x)
#pragma unroll
        for (int l = 0; l < L; ++l) vsh[l * n + e] = vboard[(size_t)c * L * n + (size_t)l * n + e];
    }
    __syncthreads();
    const double *xs = own ? col(lcol(c)) : vsh;
    while (q0 < ncol && gcol(q0) <= c) ++q0;
    const bool ahead = (c + 1 < n) && owner(c + 1) == g;
    const int qa = ahead ? lcol(c + 1) : -1;
    // 2. S of every live column: owned A columns J > c (a suffix q >= q0 of
    // the owned ones) and every owned Q^T column; the look-ahead column by
    // wavefront 0 with all its lanes, the others by teams 4.. (or 0..) of
    // T lanes, team t0 taking the live columns t0, t0 + nt, ...
    const int t0 = ahead ? team - 4 : team, nt = ahead ? (blockDim.x / T) - 4 : blockDim.x / T;
    const int nlive = ncol - q0 - (ahead ? 1 : 0);
    auto live_col = [&](int k) {
      int q = q0 + k;
      if (ahead && q >= qa) ++q;
      return q;
    };
    double Sa[L];
    if (ahead && w == 0) {
      partial_dot(qa, c, xs, lane, 64, Sa);
    } else {
      for (int k = t0; k < nlive; k += nt) {
        const int q = live_col(k);
        double S[L];
        partial_dot(q, c, xs, tl, T, S);
        if (tl == 0)
#pragma unroll
          for (int l = 0; l < L; ++l) ssum[q * L + l] = S[l];
      }
    }
    // 2. tau and 1 / (x_0 - beta)
    if (tid == 0) {
      if (own) {
#pragma unroll
        for (int l = 0; l < L; ++l) {
          sh_tau[l] = sh_tau_own[l];
          sh_inv[l] = own_inv[lcol(c) * L + l];
        }
        sh_ok = 1;
      } else {
        // poll the 2 L slots (agent scope: the emptied value, or the owner's)
        // until none holds SLOT_EMPTY; bounded, MD_EHIP on time-out
        double ts[2 * L];
        long spins = 0;
        sh_ok = 1;
        while (true) {
          bool full = true;
#pragma unroll
          for (int l = 0; l < 2 * L; ++l) {
            ts[l] = __hip_atomic_load(&tboard[(size_t)c * 2 * L + l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            full = full && __double_as_longlong(ts[l]) != SLOT_EMPTY;
          }
          if (full) break;
          __builtin_amdgcn_s_sleep(1);
          if (++spins > (1L << 22)) {
            set_status(status, MD_EHIP);
            sh_ok = 0;
            break;
          }
        }
#pragma unroll
        for (int l = 0; l < L; ++l) {
          sh_tau[l] = ts[l];
          sh_inv[l] = ts[L + l];
        }
      }
    }
    __syncthreads();
    if (!sh_ok) {
      ok = false;
      break;
    }
    double tc[L], inv[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      tc[l] = sh_tau[l];
      inv[l] = sh_inv[l];
    }
    // 3. the updates; the look-ahead column first, then its reflector
    if (ahead && w == 0) {
      finish_apply(qa, c, xs, Sa, tc, inv, lane, 64);
      wave_sync();
      publish(qa, c + 1);
    } else {
      for (int k = t0; k < nlive; k += nt) {
        const int q = live_col(k);
        double S[L];
#pragma unroll
        for (int l = 0; l < L; ++l) S[l] = ssum[q * L + l];
        finish_apply(q, c, xs, S, tc, inv, tl, T);
      }
    }
    __syncthreads();
  }
  if (ok) {  // write back the owned columns, v = x / (x_0 - beta) below the diagonal
    for (int q = 0; q < ncol; ++q) {
      const int J = gcol(q);
      const double *cq = col(q);
      for (int i = tid; i < n; i += blockDim.x) {
        double x[L];
#pragma unroll
        for (int l = 0; l < L; ++l) x[l] = cq[l * n + i];
        if (J < n && i > J) {
          double inv[L], v[L];
#pragma unroll
          for (int l = 0; l < L; ++l) inv[l] = own_inv[q * L + l];
          MD<L>::mul(x, inv, v);
          md::copy<L>(v, x);
        }
#pragma unroll
        for (int l = 0; l < L; ++l) {
          if (J < n) a[(size_t)l * nn + (size_t)i * n + J] = x[l];
          else qt[(size_t)l * nn + (size_t)i * n + (J - n)] = x[l];
        }
      }
    }
  }
}

__global__ void qr_prep_kernel(QrPrep q) { qr_prep_item(q, (size_t)blockIdx.x * blockDim.x + threadIdx.x); }

// The persistent staged solve's counters cleared and its dx slots emptied.
__global__ void stages_prep_kernel(int *sync, int nsync, double *dxT, size_t ndx) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (size_t)nsync) sync[t] = 0;
  if (t < ndx) dxT[t] = __longlong_as_double(SLOT_EMPTY);
}

__global__ void zero_i32_kernel(int *p, int count) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < count) p[q] = 0;
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

// Back substitution R z = y in place on y [L][n] in LDS, one wavefront:
// column-oriented, z_i = y_i / R_ii with the precomputed reciprocal, then
// y_p -= R_pi z_i for p < i.
template <int L>
__device__ void back_subst(int n, const double *qr, const double *invd, double *y, int lane) {
  const size_t nn = (size_t)n * n;
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
}

// Column c of M = R^{-1} Q^T: y = H_{n-1} ... H_0 e_c (Q^T applied to e_c),
// then z = R^{-1} y by column-oriented back substitution.  One wavefront per
// column, y kept in LDS.
template <int L>
__global__ void __launch_bounds__(64, 1) form_m_kernel(int n, const double *qr, const double *tau, const double *invd,
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
  back_subst<L>(n, qr, invd, y, lane);
  for (int i = lane; i < n; i += 64) {
    double zi[L];
#pragma unroll
    for (int l = 0; l < L; ++l) zi[l] = y[l * n + i];
    st<L>(M, nn, (size_t)i * n + c, zi);
  }
}

// Column c of M = R^{-1} Q^T from an explicit Q^T (rows of the QR kernel's
// augmented part): one wavefront per column.
template <int L>
__global__ void __launch_bounds__(64, 1) m_from_qt_kernel(int n, const double *qr, const double *qt, const double *invd,
                                                       double *M) {
  extern __shared__ double y[];  // [L][n]
  const int c = blockIdx.x, lane = threadIdx.x;
  const size_t nn = (size_t)n * n;
  for (int i = lane; i < n; i += 64) {
    double v[L];
    ld<L>(qt, nn, (size_t)i * n + c, v);
#pragma unroll
    for (int l = 0; l < L; ++l) y[l * n + i] = v[l];
  }
  wave_sync();
  back_subst<L>(n, qr, invd, y, lane);
  for (int i = lane; i < n; i += 64) {
    double zi[L];
#pragma unroll
    for (int l = 0; l < L; ++l) zi[l] = y[l * n + i];
    st<L>(M, nn, (size_t)i * n + c, zi);
  }
}

// Lane i's double in every lane (i uniform over the wavefront).
__device__ __forceinline__ double read_lane(double x, int i) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, i);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), i);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The rows of R scaled by their diagonal entries, for the back substitution
// of M: dq[p] = 1 / R_pp and rs(p, j) = R_pj / R_pp for j > p ([L][n][n],
// row-major), one wavefront per row p.  A diagonal entry below n 2^(-53 L)
// times the largest one (leading limbs) means A_0 is singular to working
// precision: MD_ESINGULAR, and the row's 1 / R_pp is zero.
template <int L>
__global__ void __launch_bounds__(64) rscale_kernel(int n, const double *qr, double *rs, double *dq, int32_t *status) {
  const int p = blockIdx.x, lane = threadIdx.x;
  const size_t nn = (size_t)n * n;
  double rmax = 0.0;
  for (int j = lane; j < n; j += 64) {
    double d[L];
    ld<L>(qr, nn, (size_t)j * n + j, d);
    rmax = fmax(rmax, fabs(d[0]));
  }
  for (int off = 32; off > 0; off >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, off, 64));
  double rpp[L], d[L];
  ld<L>(qr, nn, (size_t)p * n + p, rpp);
  const bool sing = !(fabs(rpp[0]) > ldexp((double)n, -53 * L) * rmax);
  if (sing) md::zero<L>(d);
  else md::recip_newton<L>(rpp, d);
  if (lane == 0) {
    st<L>(dq, n, p, d);
    if (sing) set_status(status, MD_ESINGULAR);
  }
  for (int j = p + 1 + lane; j < n; j += 64) {
    double r[L], q[L];
    ld<L>(qr, nn, (size_t)p * n + j, r);
    MD<L>::mul(r, d, q);
    st<L>(rs, nn, (size_t)p * n + j, q);
  }
}

// Column c of M = R^{-1} Q^T for n <= 64, one wavefront per column with
// row p in lane p, on the scaled rows of rscale_kernel: with y~_p = y_p / R_pp
// and R~_pi = R_pi / R_pp, back substitution takes z_i = y~_i and then
// y~_p -= R~_pi z_i for p < i, so a step of the dependent chain is one lane
// read and one multiply-add.  The columns of R~ are loaded four steps before
// they are used (they were just written by another kernel: their loads come
// from memory, not the L2).
template <int L>
__global__ void __launch_bounds__(64, 1) m_from_qt_small_kernel(int n, const double *rs, const double *dq,
                                                             const double *qt, double *M, int *done) {
  // raised wave priority: the kernel runs beside the evaluation, whose
  // wavefronts fill the CUs (M beside it: 47 against 180 us)
  __builtin_amdgcn_s_setprio(3);
  const int c = blockIdx.x, lane = threadIdx.x;
  const size_t nn = (size_t)n * n;
  const bool on = lane < n;
  const int p = on ? lane : 0;
  double y[L];
  md::zero<L>(y);
  if (on) {
    double y0[L], d[L];
    ld<L>(qt, nn, (size_t)p * n + c, y0);
    ld<L>(dq, n, p, d);
    MD<L>::mul(y0, d, y);
  }
  // R~(p, j) for p < j
  auto ldcol = [&](int j, double (&r)[L]) {
    md::zero<L>(r);
    if (j >= 0 && lane < j) ld<L>(rs, nn, (size_t)p * n + j, r);
  };
  double r0[L], r1[L], r2[L], r3[L];
  ldcol(n - 1, r0);
  ldcol(n - 2, r1);
  ldcol(n - 3, r2);
  ldcol(n - 4, r3);
  // step i with column i of R~ in rc, which then receives column i - 4
  auto step = [&](int i, double (&rc)[L]) {
    double z[L];
#pragma unroll
    for (int l = 0; l < L; ++l) z[l] = read_lane(y[l], i);
    if (lane < i) MD<L>::fms(y, rc, z);
    ldcol(i - 4, rc);
  };
  int i = n - 1;
  for (; i >= 3; i -= 4) {  // four steps a round: the four registers rotate by name, not by copies
    step(i, r0);
    step(i - 1, r1);
    step(i - 2, r2);
    step(i - 3, r3);
  }
  if (i >= 0) step(i, r0);
  if (i >= 1) step(i - 1, r1);
  if (i >= 2) step(i - 2, r2);
  if (!done) {
    if (on) st<L>(M, nn, (size_t)p * n + c, y);
    return;
  }
  // a reader on another stream polls *done (one count per column)
  if (on) st_agent<L>(M, nn, (size_t)p * n + c, y);
  wait_vm();
  if (lane == 0) __hip_atomic_fetch_add(done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// out[l][c][r] = in[l][r][c] for r < rows, c < cols (row strides in_ld,
// out_ld; limb strides in_ls, out_ls): series-major arrays [..][D] to
// coefficient-major [D][..] and back, also for a window of the coefficients,
// through a 32 x 32 LDS tile so that reads and writes are both coalesced.
__global__ void __launch_bounds__(256) transpose_kernel(const double *in, double *out, size_t rows, int cols,
                                                        size_t in_ld, size_t out_ld, size_t in_ls, size_t out_ls) {
  __shared__ double tile[32][33];
  const int l = blockIdx.z;
  const size_t r0 = (size_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const size_t r = r0 + yy;
    const int c = c0 + tx;
    if (r < rows && c < cols) tile[yy][tx] = in[(size_t)l * in_ls + r * in_ld + c];
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int c = c0 + yy;
    const size_t r = r0 + tx;
    if (r < rows && c < cols) out[(size_t)l * out_ls + (size_t)c * out_ld + r] = tile[tx][yy];
  }
}

// N = M B for dense n x n matrices (B with limb stride b_ls); teams of 16
// lanes per output entry, level-sum accumulation.  Product y: B + y n^2 (the
// next series coefficient) into N + y L n^2.
template <int L>
__device__ __forceinline__ void gemm_block(int n, const double *M, const double *B, size_t b_ls, double *N, int y) {
  const int T = 16;
  B += (size_t)y * n * n;
  N += (size_t)y * L * n * n;
  const size_t task = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
  const int tl = threadIdx.x & (T - 1);
  const size_t nn = (size_t)n * n;
  const bool live = task < nn;
  const size_t tk = live ? task : 0;
  const int i = (int)(tk / n), j = (int)(tk - (size_t)i * n);
  double acc[L], r[L];
  md::zero<L>(acc);
  for (int v = tl; v < n; v += T) {
    double m[L], b[L];
    ld<L>(M, nn, (size_t)i * n + v, m);
    ld<L>(B, b_ls, (size_t)v * n + j, b);
    MD<L>::fma_lazy(acc, m, b);
  }
  team_sum_lazy<L>(acc, T);
  MD<L>::renorm(acc, r);
  if (live && tl == 0) st<L>(N, nn, (size_t)i * n + j, r);
}

template <int L>
__global__ void __launch_bounds__(256) gemm_kernel(int n, const double *M, const double *B, size_t b_ls, double *N) {
  gemm_block<L>(n, M, B, b_ls, N, blockIdx.y);
}

// One stage k of the block Toeplitz solve (see the file comment), on
// coefficient-major arrays: At [L][D][n][n] (At[k] = A_k), rT, dxT [L][D][n].
// Blocks 0 .. ceil(n/4)-1: one wavefront per row i computes
//     dx_k(i) = sum_v M(i,v) r_k(v) - N(i,v) dx_{k-1}(v);
// the other blocks: teams of 16 lanes per (m, i), m = k+1..D-1, push
//     r_m(i) -= sum_v A_{m-k+1}(i,v) dx_{k-1}(v).
template <int L>
__global__ void __launch_bounds__(256) stage_kernel(int n, int D, int k, const double *M, const double *N,
                                                    const double *At, double *rT, double *dxT) {
  const size_t nn = (size_t)n * n, nD = (size_t)n * D, nnD = nn * D;
  const int crit_blocks = (n + 3) / 4;
  double acc[L], r[L];
  md::zero<L>(acc);
  if ((int)blockIdx.x < crit_blocks) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int i = row < n ? row : 0;
    for (int v = lane; v < n; v += 64) {
      double m[L], rv[L];
      ld<L>(M, nn, (size_t)i * n + v, m);
      ld<L>(rT, nD, (size_t)k * n + v, rv);
      MD<L>::fma_lazy(acc, m, rv);
      if (k > 0) {
        double nv[L], xv[L];
        ld<L>(N, nn, (size_t)i * n + v, nv);
        ld<L>(dxT, nD, (size_t)(k - 1) * n + v, xv);
        md::neg<L>(nv, nv);
        MD<L>::fma_lazy(acc, nv, xv);
      }
    }
    team_sum_lazy<L>(acc, 64);
    MD<L>::renorm(acc, r);
    if (row < n && lane == 0) st<L>(dxT, nD, (size_t)k * n + i, r);
    return;
  }
  if (k == 0) return;  // stage 0 has no previous update to push
  const int T = 16;
  const size_t task = ((size_t)(blockIdx.x - crit_blocks) * blockDim.x + threadIdx.x) / T;
  const int tl = threadIdx.x & (T - 1);
  const size_t ntask = (size_t)n * (D - k - 1);
  const bool live = task < ntask;
  const size_t tk = live ? task : 0;
  const int mm = k + 1 + (int)(tk / n), i = (int)(tk % n), jj = mm - k + 1;
  if (live) {
    for (int v = tl; v < n; v += T) {
      double av[L], xv[L];
      ld<L>(At, nnD, (size_t)jj * nn + (size_t)i * n + v, av);
      ld<L>(dxT, nD, (size_t)(k - 1) * n + v, xv);
      MD<L>::fma_lazy(acc, av, xv);
    }
  }
  team_sum_lazy<L>(acc, T);
  MD<L>::renorm(acc, r);
  if (live && tl == 0) {
    double rv[L], s2[L];
    ld<L>(rT, nD, (size_t)mm * n + i, rv);
    MD<L>::sub(rv, r, s2);
    st<L>(rT, nD, (size_t)mm * n + i, s2);
  }
}

// Bounded wait until *ctr >= target (relaxed polling with a short sleep, one
// agent-scope acquire fence after).  On time-out the status word gets MD_EHIP.
template <int SLEEP = 1>
__device__ __forceinline__ bool wait_geq(const int *ctr, int target, int32_t *status) {
  long spins = 0;
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(SLEEP);
    if (++spins > (1L << 22)) {
      set_status(status, MD_EHIP);
      return false;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Coefficient 0 of the next iterate, x_0 + dx_0 with dx_0 = M r_0, by the
// operations the persistent staged solve and finish_kernel apply to it: one
// wavefront per row i, lane v accumulates M(i, v) r_0(v) into zeroed level
// sums, one 64-lane butterfly of level sums, one renormalization (the first
// stage of stages_persistent_kernel), then the addition of finish_kernel.
// The result is therefore the x_0 that the next step reads, bit for bit,
// available before the staged solve has run; xn [L][n].  This and the two
// kernels must keep these operations in step.
template <int L>
__device__ __forceinline__ void next_x0_block(int n, int D, const double *M, const double *rT, const double *x,
                                              double *xn, int *done) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i = blockIdx.x * 4 + wv;
  const bool row = i < n, col = lane < n;
  const int ii = row ? i : 0, v = col ? lane : 0;
  const size_t nn = (size_t)n * n, nD = (size_t)n * D;
  double acc[L], r[L];
  md::zero<L>(acc);
  if (col) {
    double m[L], a[L];
    ld<L>(M, nn, (size_t)ii * n + v, m);
    ld<L>(rT, nD, (size_t)v, a);
    MD<L>::fma_lazy(acc, m, a);
  }
  team_sum_lazy<L>(acc, 64);
  MD<L>::renorm(acc, r);
  if (row && lane == 0) {
    double a[L], sum[L];
    ld<L>(x, nD, (size_t)i * D, a);
    MD<L>::add(a, r, sum);
    if (done) st_agent<L>(xn, n, i, sum);
    else st<L>(xn, n, i, sum);
  }
  if (done) {  // a reader on another stream polls *done (one count per workgroup)
    wait_vm();
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Coefficient 0 of the next iterate (next_x0_block) in the first row of
// blocks and the products of gemm_kernel (product blockIdx.y - 1) in the
// others: one launch where the caller's stream has both ready (M and r_0),
// so that the update of x later in that stream comes after every read of
// x_0.  The xn workgroups are dispatched first: the factorization on the
// second stream waits for them.  done (nullable): each of the ceil(n / 4)
// workgroups of xn adds one to it once its stores are performed.
template <int L>
__global__ void __launch_bounds__(256) gemm_next_x0_kernel(int n, int D, const double *M, const double *B, size_t b_ls,
                                                           double *N, const double *rT, const double *x, double *xn,
                                                           int *done) {
  if (blockIdx.y > 0) {
    gemm_block<L>(n, M, B, b_ls, N, blockIdx.y - 1);
  } else if ((int)blockIdx.x * 4 < n) {
    next_x0_block<L>(n, D, M, rT, x, xn, done);
  }
}

// Counters of the persistent staged solve: the updaters' counters one per
// 256 bytes, the solvers' flags packed into the second block of 256 bytes.
constexpr int SYNC_STRIDE = 64;

// Products of M with the leading Jacobian coefficients that the persistent
// staged solve takes as a whole: N = M A_1, P = M A_2, Q = M A_3.
constexpr int STAGE_PRODUCTS = 3;

// The whole staged solve in one launch, for n <= 64.  With P = M A_2 and
// Q = M A_3 the recurrence is reassociated twice more,
//     dx_k = M r''_k - N dx_{k-1} - P dx_{k-2} - Q dx_{k-3},
//     r''_k = b_k - sum_{j>=4} A_j dx_{k-j},
// so that a stage only needs right-hand-side terms at least three stages
// old.  Solver workgroup s (s < Gs = ceil(n/2)) owns rows i = 2 s + w, w = 0, 1,
// with two wavefronts per row (lane v holds column v):
//   * the critical wavefront of row i keeps N(i,.) in registers; at stage k it
//     waits for every solver's dx_{k-1}, adds N(i,.) dx_{k-1} to the level
//     sums pre_k(i) left in LDS by its companion, reduces them over the 64
//     lanes, renormalizes and stores dx_k(i);
//   * the companion wavefront keeps M(i,.), P(i,.), Q(i,.) and forms, while
//     stage k runs, pre_{k+1}(i) = M r''_{k+1} - Q dx_{k-2} - P dx_{k-1} in
//     lane-wise level sums: r''_{k+1} once its updaters have published it,
//     dx_{k-2} from its registers, dx_{k-1} from the LDS copy that the
//     critical wavefront made at the start of stage k.
// So a stage's critical path holds one multiply-add per lane, one butterfly
// and the hand-over.  One workgroup barrier per stage separates the two
// wavefronts' uses of the LDS slots (pre_k in slot k mod 2).  dx itself is
// the hand-over: its slots are emptied (SLOT_EMPTY) by the launch ahead of
// this one on the stream, every dx_k(i) is written once with agent-scope
// stores, and a reader polls the entries it needs with agent-scope loads
// until no limb is empty (no flag, no wait for the stores, one round trip).
// Updater (g, b) owns the rows 16 b .. 16 b + 15 (one team of 16
// lanes per row) of coefficient m = 4 + g (and m + Gm when there are more than
// 64 coefficients from 4 on): in round q, once dx_q is out, every lane adds
// its four terms of A_{m-q}(i,.) dx_q to level sums kept in registers across
// the rounds; after round m - 4 the team reduces them, renormalizes,
// stores r''_m(i) = b_m(i) - sum and counts itself done for m, so r''_m is
// written once, by its owner.  Everything handed between workgroups (dx,
// r'', counters) goes through agent-scope loads and stores (r'' with a wait
// for the stores before its counter), never through fences: a fence would
// write back or invalidate a whole L2 at every hand-over, hundreds of them
// per stage.  All
// workgroups must be resident together; waits are bounded and report
// MD_EHIP, after which every wavefront of a workgroup leaves at the same
// barrier.
template <int L>
__global__ void __launch_bounds__(256) stages_persistent_kernel(int n, int D, int Gs, int Gm, const double *M,
                                                                const double *NP, const double *At, double *rT,
                                                                double *dxT, int *sync, int32_t *status) {
  __shared__ int sh_dead[2];               // a wait of stage k timed out (slot k mod 2)
  __shared__ int sh_ok;                    // an updater round may start
  __shared__ int sh_x1[2];                 // stage k whose dx_{k-1} is in x1s[w]
  __shared__ double x1s[2][L * 64];        // dx_{k-1}, critical -> companion wavefront of row slot w
  __shared__ double pres[2][2][L * 64];    // pre_k level sums of row slot w in slot k mod 2
  __shared__ double xq[L * 64];            // dx_q of an updater round
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const size_t nn = (size_t)n * n, nD = (size_t)n * D, nnD = nn * D;
  const int Bm = (n + 15) / 16;
  auto rounds = [&](int m) { return sync + (size_t)(2 + m) * SYNC_STRIDE; };
  auto poll = [&](const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
  // wavefront-wide poll of dx_k (lane v: dx_k(v), its L limbs) until no limb
  // is empty; lanes v >= n get zeros.  Bounded: false and MD_EHIP on time-out.
  auto poll_dx = [&](int k, double (&x)[L]) {
    long spins = 0;
    while (true) {
      bool full = true;
      md::zero<L>(x);
      if (lane < n) {
        ld_agent<L>(dxT, nD, (size_t)k * n + lane, x);
#pragma unroll
        for (int l = 0; l < L; ++l) full = full && !slot_empty(x[l]);
      }
      if (__all(full)) return true;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1L << 22)) {
        if (lane == 0) set_status(status, MD_EHIP);
        return false;
      }
    }
  };
  if ((int)blockIdx.x < Gs) {
    const int w = wv & 1;              // row slot
    const bool crit = wv < 2;          // critical wavefront (else the companion)
    const int i = blockIdx.x * 2 + w;
    const bool row = i < n, col = lane < n;
    const int ii = row ? i : 0, v = col ? lane : 0;
    if (tid < 2) {
      sh_dead[tid] = 0;
      sh_x1[tid] = 0;
    }
    double *const slot0 = &pres[w][0][0], *const slot1 = &pres[w][1][0];
    if (crit) {
      double nv[L];
      md::zero<L>(nv);
      if (row && col && D > 1) {
        ld<L>(NP, nn, (size_t)ii * n + v, nv);
        md::neg<L>(nv, nv);
      }
      __syncthreads();  // pre_0 is in slot 0
      for (int k = 0; k < D; ++k) {
        double acc[L], r[L], x1[L];
        const double *slot = (k & 1) ? slot1 : slot0;
#pragma unroll
        for (int l = 0; l < L; ++l) acc[l] = slot[l * 64 + lane];
        if (k >= 1) {
          md::zero<L>(x1);
          const bool ok = row ? poll_dx(k - 1, x1) : true;
          if (!ok && lane == 0) sh_dead[k & 1] = 1;
#pragma unroll
          for (int l = 0; l < L; ++l) x1s[w][l * 64 + lane] = x1[l];
          __hip_atomic_store(&sh_x1[w], k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
          MD<L>::fma_lazy(acc, nv, x1);
        }
        if (row) {
          team_sum_lazy<L>(acc, 64);
          MD<L>::renorm(acc, r);
          if (lane == 0) st_agent<L>(dxT, nD, (size_t)k * n + i, r);  // the readers poll these slots
        }
        __syncthreads();  // pre_{k+1} is in its slot
        if (sh_dead[k & 1]) return;
      }
      return;
    }
    // companion wavefront
    double m[L], pv[L], qv[L], x2[L], pre[L];
    md::zero<L>(m);
    md::zero<L>(pv);
    md::zero<L>(qv);
    md::zero<L>(x2);
    md::zero<L>(pre);
    if (row && col) {
      ld<L>(M, nn, (size_t)ii * n + v, m);
      if (D > 2) ld<L>(NP + (size_t)L * nn, nn, (size_t)ii * n + v, pv);
      if (D > 3) ld<L>(NP + (size_t)2 * L * nn, nn, (size_t)ii * n + v, qv);
      md::neg<L>(pv, pv);
      md::neg<L>(qv, qv);
      double a[L];
      ld_agent<L>(rT, nD, (size_t)v, a);
      MD<L>::fma_lazy(pre, m, a);
    }
#pragma unroll
    for (int l = 0; l < L; ++l) slot0[l * 64 + lane] = pre[l];
    __syncthreads();  // pre_0 is in slot 0
    for (int k = 0; k < D; ++k) {
      if (k + 1 < D && row) {  // pre_{k+1} while stage k runs
        bool ok = true;
        if (k + 1 > STAGE_PRODUCTS) {  // r''_{k+1} published by its Bm updaters
          long spins = 0;
          while (true) {
            const int f = poll(rounds(k + 1));
            if (__all(f >= Bm)) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1L << 22)) {
              if (lane == 0) set_status(status, MD_EHIP);
              ok = false;
              break;
            }
          }
        }
        md::zero<L>(pre);
        if (ok && col) {
          double a[L];
          ld_agent<L>(rT, nD, (size_t)(k + 1) * n + v, a);
          MD<L>::fma_lazy(pre, m, a);
          if (k >= 2) MD<L>::fma_lazy(pre, qv, x2);
        }
        if (k >= 1) {  // dx_{k-1} from the critical wavefront of this row
          long spins = 0;
          while (__hip_atomic_load(&sh_x1[w], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < k) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1L << 22)) {
              if (lane == 0) set_status(status, MD_EHIP);
              ok = false;
              break;
            }
          }
          double x1[L];
#pragma unroll
          for (int l = 0; l < L; ++l) x1[l] = x1s[w][l * 64 + lane];
          if (ok && col) MD<L>::fma_lazy(pre, pv, x1);
          md::copy<L>(x1, x2);
        }
        if (!ok && lane == 0) sh_dead[k & 1] = 1;
        double *slot = ((k + 1) & 1) ? slot1 : slot0;
#pragma unroll
        for (int l = 0; l < L; ++l) slot[l * 64 + lane] = pre[l];
      }
      __syncthreads();
      if (sh_dead[k & 1]) return;
    }
    return;
  }
  // updater (g, b): rows 16 b .. 16 b + 15, coefficients m0 and m1 (if below D)
  const int u = blockIdx.x - Gs, g = u / Bm, b = u - g * Bm;
  const int team = tid / 16, tl = tid & 15;
  const int i = b * 16 + team;
  const bool live = i < n;
  const int m0 = STAGE_PRODUCTS + 1 + g, m1 = m0 + Gm;
  const int qlast = (m1 < D ? m1 : m0) - STAGE_PRODUCTS - 1;
  double acc0[L], acc1[L];  // lane-wise level sums of sum_q A_{m-q}(i, v) dx_q(v)
  md::zero<L>(acc0);
  md::zero<L>(acc1);
  // r''_m(i) = b_m(i) - (the team's sum of acc) once every round q <= m - 4 is in
  auto publish = [&](int mm, const double (&acc)[L]) {
    double t[L], r[L];
    md::copy<L>(acc, t);
    team_sum_lazy<L>(t, 16);
    MD<L>::renorm(t, r);
    if (live && tl == 0) {
      double rv[L], s2[L];
      ld_agent<L>(rT, nD, (size_t)mm * n + i, rv);
      MD<L>::sub(rv, r, s2);
      st_agent<L>(rT, nD, (size_t)mm * n + i, s2);
    }
    wait_vm();
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(rounds(mm), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  // the row's four terms A_{m0-q}(i, tl + 16 j) of the coming round, loaded
  // while the previous round waits (they do not depend on dx)
  double an[4][L];
  auto fetch0 = [&](int q) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int vv = tl + 16 * j;
      if (live && vv < n && q + STAGE_PRODUCTS + 1 <= m0)
        ld<L>(At + (size_t)(m0 - q) * nn, nnD, (size_t)i * n + vv, an[j]);
      else
        md::zero<L>(an[j]);
    }
  };
  fetch0(0);
  for (int q = 0; q <= qlast; ++q) {
    // dx_q: every thread polls its entries until they are written (bounded)
    int bad = 0;
    for (int e = tid; e < L * n; e += blockDim.x) {
      const int l = e / n, vv = e - l * n;
      const double *src = dxT + (size_t)l * nD + (size_t)q * n + vv;
      double val;
      long spins = 0;
      while (true) {
        val = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!slot_empty(val)) break;
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1L << 22)) {
          set_status(status, MD_EHIP);
          bad = 1;
          break;
        }
      }
      xq[l * 64 + vv] = val;
    }
    if (__syncthreads_or(bad)) return;
    const bool use0 = q + STAGE_PRODUCTS + 1 <= m0, use1 = m1 < D && q + STAGE_PRODUCTS + 1 <= m1;
    if (live && use0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int vv = tl + 16 * j;
        if (vv < n) {
          double x[L];
#pragma unroll
          for (int l = 0; l < L; ++l) x[l] = xq[l * 64 + vv];
          MD<L>::fma_lazy(acc0, an[j], x);
        }
      }
    }
    fetch0(q + 1);
    if (live && use1) {
      for (int vv = tl; vv < n; vv += 16) {
        double a[L], x[L];
#pragma unroll
        for (int l = 0; l < L; ++l) x[l] = xq[l * 64 + vv];
        ld<L>(At + (size_t)(m1 - q) * nn, nnD, (size_t)i * n + vv, a);
        MD<L>::fma_lazy(acc1, a, x);
      }
    }
    if (q + STAGE_PRODUCTS + 1 == m0) publish(m0, acc0);
    if (m1 < D && q + STAGE_PRODUCTS + 1 == m1) publish(m1, acc1);
    __syncthreads();  // xq is rewritten by the next round
  }
}

// out[l][s][i] = in[l][i][D-1-s] and back (coefficients in reverse order):
// the transposed block Toeplitz system runs the stage recurrence from the
// last coefficient to the first.
__global__ void series_to_rev_kernel(int n, int D, int L, const double *in, double *out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nD = (size_t)n * D;
  if (q >= nD * L) return;
  const size_t l = q / nD, r = q - l * nD;
  const int s = (int)(r / n), i = (int)(r - (size_t)s * n);
  out[q] = in[l * nD + (size_t)i * D + (D - 1 - s)];
}

__global__ void rev_to_series_kernel(int n, int D, int L, const double *in, double *out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nD = (size_t)n * D;
  if (q >= nD * L) return;
  const size_t l = q / nD, r = q - l * nD;
  const int i = (int)(r / D), k = (int)(r - (size_t)i * D);
  out[q] = in[l * nD + (size_t)(D - 1 - k) * n + i];
}

// grad[m] = -sum_k lambda_{row(m),k} val_m[k] (val: coefficient-free monomial
// values [L][m][D]), one thread per monomial, fixed order.
template <int L>
__global__ void coef_grad_kernel(int n, int D, int m, const int32_t *row_of, const double *lambda, const double *val,
                                 double *grad) {
  const int mj = blockIdx.x * blockDim.x + threadIdx.x;
  if (mj >= m) return;
  const size_t nD = (size_t)n * D, mD = (size_t)m * D;
  const int i = row_of[mj];
  double acc[L], r[L];
  md::zero<L>(acc);
  for (int k = 0; k < D; ++k) {
    double a[L], b[L];
    ld<L>(lambda, nD, (size_t)i * D + k, a);
    ld<L>(val, mD, (size_t)mj * D + k, b);
    MD<L>::fma_lazy(acc, a, b);
  }
  MD<L>::renorm(acc, r);
  md::neg<L>(r, r);
  st<L>(grad, m, mj, r);
}

// c = [1, 0, ..., 0] in every element (unit coefficients).
__global__ void unit_md_kernel(int L, int m, double *c) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < L * m) c[q] = (q < m) ? 1.0 : 0.0;
}

// c = sum_q a[q] * b[q] over count elements (one workgroup, fixed order).
template <int L>
__global__ void __launch_bounds__(256) dot_kernel(int64_t count, const double *a, const double *b, double *c) {
  __shared__ double part[256][L];
  double acc[L], r[L];
  md::zero<L>(acc);
  for (int64_t q = threadIdx.x; q < count; q += blockDim.x) {
    double x[L], y[L];
    ld<L>(a, count, q, x);
    ld<L>(b, count, q, y);
    MD<L>::fma_lazy(acc, x, y);
  }
  MD<L>::renorm(acc, r);
#pragma unroll
  for (int l = 0; l < L; ++l) part[threadIdx.x][l] = r[l];
  __syncthreads();
  for (int half = 128; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half) {
      double u[L], v[L], s[L];
#pragma unroll
      for (int l = 0; l < L; ++l) {
        u[l] = part[threadIdx.x][l];
        v[l] = part[threadIdx.x + half][l];
      }
      MD<L>::add(u, v, s);
#pragma unroll
      for (int l = 0; l < L; ++l) part[threadIdx.x][l] = s[l];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int l = 0; l < L; ++l) c[l] = part[0][l];
}

// x := x + dx for the coefficients lo .. lo + W - 1 of every series, one
// thread per (i, s), dx with Ldx <= L limbs (the complex step updates its
// two planes with it; the real step uses finish_kernel below).
template <int L, int Ldx = L>
__global__ void update_kernel(int n, int D, int lo, int W, const double *dx, double *x) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nD = (size_t)n * D;
  if (t >= (size_t)n * W) return;
  const size_t i = t / W;
  const size_t q = i * D + lo + (t - i * W);
  double a[L], b[L], s[L], d[Ldx];
  ld<L>(x, nD, q, a);
  ld<Ldx>(dx, nD, q, d);
  md::widen<Ldx>(d, b);
  MD<L>::add(a, b, s);
  st<L>(x, nD, q, s);
}

// The end of a step on the window lo..hi-1 in one launch, one workgroup
// per coefficient k: dx_k from the coefficient-major output of the staged
// solve (dxT [Ldx][W][n]) into the series-major dx, x_k += dx_k at L limbs
// (dx may carry fewer limbs), and the norms of norms_kernel below from the
// same values (the transpose, update_kernel and norms_kernel fused).
template <int L, int Ldx = L>
__global__ void __launch_bounds__(256) finish_kernel(int n, int D, int lo, int hi, const double *dxT, double *dx,
                                                     double *x, const double *b, double *norms, int32_t *status,
                                                     const double *tsz, double *rel) {
  __shared__ double sb[256], sx[256], ss[256];
  __shared__ int sf[256];
  const int k = blockIdx.x, t = threadIdx.x;
  const bool has_b = k < hi, has_dx = k >= lo && k < hi;
  const size_t nD = (size_t)n * D, nW = (size_t)n * (hi - lo);
  double nb = 0.0, nx = 0.0, ns = 0.0;
  int finite = 1;
  for (int i = t; i < n; i += blockDim.x) {
    const size_t q = (size_t)i * D + k;
    double xi = 0.0;
    if (has_dx) {
      double d[Ldx], w[L], a[L], sum[L];
      ld<Ldx>(dxT, nW, (size_t)(k - lo) * n + i, d);
      st<Ldx>(dx, nD, q, d);
      md::widen<Ldx>(d, w);
      ld<L>(x, nD, q, a);
      MD<L>::add(a, w, sum);
      st<L>(x, nD, q, sum);
      xi = d[0];
    }
    const double bi = has_b ? b[q] : 0.0;
    finite &= (isfinite(bi) && isfinite(xi)) ? 1 : 0;
    nb = fmax(nb, fabs(bi));
    nx = fmax(nx, fabs(xi));
    if (tsz && has_b) {  // |b_{i,k}| relative to the size of its own terms (0/0 = 0)
      const double tz = tsz[q], ab = fabs(bi);
      ns = fmax(ns, tz > 0.0 ? ab / tz : (ab > 0.0 ? INFINITY : 0.0));
    }
  }
  sb[t] = nb;
  sx[t] = nx;
  ss[t] = ns;
  sf[t] = finite;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) {
      sb[t] = fmax(sb[t], sb[t + h]);
      sx[t] = fmax(sx[t], sx[t + h]);
      ss[t] = fmax(ss[t], ss[t + h]);
      sf[t] &= sf[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (norms) {
      norms[k] = sb[0];
      norms[D + k] = sx[0];
    }
    if (tsz && rel) rel[k] = ss[0];
    if (!sf[0]) set_status(status, MD_ENONFINITE);
  }
}

// norms[k] = max_i |b_{i,k}| for k < hi, norms[D+k] = max_i |dx_{i,k}| for
// lo <= k < hi (leading limbs), zero elsewhere; with the term sizes tsz of
// the assembly, rel[k] = max_i |b_{i,k}| / tsz_{i,k} for k < hi (every
// equation judged against its own terms).  A non-finite residual or update
// is reported.  One workgroup of 256 threads per coefficient k, rows strided
// over the threads, maxima reduced in LDS.
__global__ void __launch_bounds__(256) norms_kernel(int n, int D, int lo, int hi, const double *b, const double *dx,
                                                    double *norms, int32_t *status, const double *tsz,
                                                    double *rel) {
  __shared__ double sb[256], sx[256], ss[256];
  __shared__ int sf[256];
  const int k = blockIdx.x, t = threadIdx.x;
  const bool has_b = k < hi, has_dx = k >= lo && k < hi;
  double nb = 0.0, nx = 0.0, ns = 0.0;
  int finite = 1;
  for (int i = t; i < n; i += blockDim.x) {
    const double bi = has_b ? b[(size_t)i * D + k] : 0.0, xi = has_dx ? dx[(size_t)i * D + k] : 0.0;
    finite &= (isfinite(bi) && isfinite(xi)) ? 1 : 0;
    nb = fmax(nb, fabs(bi));
    nx = fmax(nx, fabs(xi));
    if (tsz && has_b) {  // |b_{i,k}| relative to the size of its own terms (0/0 = 0)
      const double t = tsz[(size_t)i * D + k], ab = fabs(bi);
      ns = fmax(ns, t > 0.0 ? ab / t : (ab > 0.0 ? INFINITY : 0.0));
    }
  }
  sb[t] = nb;
  sx[t] = nx;
  ss[t] = ns;
  sf[t] = finite;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) {
      sb[t] = fmax(sb[t], sb[t + h]);
      sx[t] = fmax(sx[t], sx[t + h]);
      ss[t] = fmax(ss[t], ss[t + h]);
      sf[t] &= sf[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (norms) {
      norms[k] = sb[0];
      norms[D + k] = sx[0];
    }
    if (tsz && rel) rel[k] = ss[0];
    if (!sf[0]) set_status(status, MD_ENONFINITE);
  }
}

// out[0..2D) = norms, out[2D..3D) = scale, out[3D] = status; one workgroup.
__global__ void __launch_bounds__(256) report_kernel(int D, const double *norms, const double *scale,
                                                     const int32_t *status, double *out) {
  for (int t = threadIdx.x; t <= 3 * D; t += blockDim.x)
    out[t] = (t < 2 * D) ? norms[t] : (t < 3 * D) ? scale[t - 2 * D] : (double)status[0];
}

template <int L>
__global__ void __launch_bounds__(256) arith_kernel(int op, int64_t count, const double *a, const double *b, double *c) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  double x[L], y[L], r[L];
  ld<L>(a, count, q, x);
  if (op != 4) ld<L>(b, count, q, y);
  switch (op) {
    case 0: MD<L>::add_acc(x, y, r); break;
    case 1: MD<L>::sub_acc(x, y, r); break;
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

hipError_t launch_status_init(int32_t *status, hipStream_t st, int *counter, int *counter2) {
  hipLaunchKernelGGL(status_init_kernel, dim3(1), dim3(64), 0, st, status, counter, counter2);
  return hipGetLastError();
}

// Workgroups of the QR: a team of 16 lanes per trailing column, at most 16
// workgroups while that suffices (a cheap grid barrier) and up to 128 for the
// large systems this kernel serves (n = 1024: 2048 columns of [A_0 | I]);
// all of them must be resident at once, one per CU at most.
int qr_workgroups(int n, bool with_qt) {
  const int cols = n + (with_qt ? n : 0);
  int G = (cols + 15) / 16;
  return G < 1 ? 1 : (G > 128 ? 128 : G);
}

// Dynamic LDS above 64 KB (an octo-double column of 1024 entries) needs the
// attribute; set once per kernel.
template <typename K>
static void allow_large_lds(K kernel) {
  (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
  (void)hipGetLastError();  // an attribute the runtime refuses must not be reported by the launch
}

hipError_t launch_qr(int L, int n, double *a, double *tau, double *qt, int32_t *status, unsigned *bar,
                     hipStream_t st) {
  const int G = qr_workgroups(n, qt != nullptr);
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, st, bar);
  MD_DISPATCH(L, {
    static bool attr = false;
    if (!attr) {
      allow_large_lds(qr_kernel<LL>);
      attr = true;
    }
    hipLaunchKernelGGL(qr_kernel<LL>, dim3(G), dim3(256), (size_t)LL * n * sizeof(double), st, n, a, tau, qt, status,
                       bar);
  });
  return hipGetLastError();
}

// Workgroups of the LDS-resident QR: at most 8 (large systems 16) columns and
// about 140 KB of columns per workgroup; 0 if that needs more than 64.
size_t qr_lds_bytes(int L, int n, int G, bool with_qt);

int qr_lds_workgroups(int L, int n, bool with_qt) {
  const int cols = with_qt ? 2 * n : n;
  // about 8 columns per workgroup (n = 64 with Q^T: 16 workgroups, 563 us
  // beside the evaluation against 570 with 8 and 584 with 4), about 16 for
  // the large systems
  int G = std::max(1, (cols + 7) / 8);
  if (G > 64) G = std::max(1, (cols + 15) / 16);
  while (G <= 64 && qr_lds_bytes(L, n, G, with_qt) > 140 * 1024) ++G;
  return G > 64 ? 0 : G;
}

size_t qr_lds_bytes(int L, int n, int G, bool with_qt) {
  const int cols = with_qt ? 2 * n : n;
  const int groups = (cols + QR_GROUP - 1) / QR_GROUP;
  const int ncol = QR_GROUP * ((groups + G - 1) / G);  // columns are owned in groups
  // the owned columns, the current reflector's column, 1 / (x_0 - beta) and
  // the partial dot product S per owned column
  return (((size_t)ncol + 1) * L * n + 2 * (size_t)ncol * L) * sizeof(double);
}

hipError_t launch_qr_lds(int L, int n, double *a, double *tau, double *qt, int32_t *status, int *flags,
                         double *vboard, double *tboard, hipStream_t st, bool prepared) {
  const int G = qr_lds_workgroups(L, n, qt != nullptr);
  if (G == 0) return hipErrorInvalidValue;
  const size_t lds = qr_lds_bytes(L, n, G, qt != nullptr);
  if (!prepared) {
    QrPrep q;
    q.flags = flags;
    q.tboard = tboard;
    q.n = n;
    q.nt = 2 * L * n;
    hipLaunchKernelGGL(qr_prep_kernel, dim3((q.nt + 255) / 256), dim3(256), 0, st, q);
  }
  MD_DISPATCH(L, {
    static bool attr = false;
    if (!attr) {
      // the kernel also has static LDS: leave room for it below the 160 KB of a CU
      (void)hipFuncSetAttribute((const void *)qr_lds_kernel<LL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                150 * 1024);
      (void)hipGetLastError();
      attr = true;
    }
    hipLaunchKernelGGL(qr_lds_kernel<LL>, dim3(G), dim3(256), lds, st, n, a, tau, qt, status, flags, vboard, tboard);
  });
  return hipGetLastError();
}

hipError_t launch_m_from_qt(int L, int n, const double *qr, const double *qt, double *invd, double *M,
                            int32_t *status, hipStream_t st, double *rs, int *done) {
  if (n <= 64 && rs) {
    MD_DISPATCH(L, {
      hipLaunchKernelGGL(rscale_kernel<LL>, dim3(n), dim3(64), 0, st, n, qr, rs, invd, status);
      hipLaunchKernelGGL(m_from_qt_small_kernel<LL>, dim3(n), dim3(64), 0, st, n, (const double *)rs,
                         (const double *)invd, qt, M, done);
    });
    return hipGetLastError();
  }
  MD_DISPATCH(L, {
    static bool attr = false;
    if (!attr) {
      allow_large_lds(m_from_qt_kernel<LL>);
      attr = true;
    }
    hipLaunchKernelGGL(invdiag_kernel<LL>, dim3((n + 63) / 64), dim3(64), 0, st, n, qr, invd, status);
    hipLaunchKernelGGL(m_from_qt_kernel<LL>, dim3(n), dim3(64), (size_t)LL * n * sizeof(double), st, n, qr, qt,
                       (const double *)invd, M);
  });
  return hipGetLastError();
}

hipError_t launch_form_m(int L, int n, const double *qr, const double *tau, double *invd, double *M, int32_t *status,
                         hipStream_t st) {
  MD_DISPATCH(L, {
    static bool attr = false;
    if (!attr) {
      allow_large_lds(form_m_kernel<LL>);
      attr = true;
    }
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

hipError_t launch_transpose_ld(int L, const double *in, size_t in_ld, double *out, size_t out_ld, size_t rows,
                               int cols, size_t in_ls, size_t out_ls, hipStream_t st) {
  // L counts batches: limbs, or limbs times coefficients for per-coefficient matrices
  if (rows == 0 || cols <= 0) return hipSuccess;
  dim3 grid((unsigned)((rows + 31) / 32), (unsigned)((cols + 31) / 32), (unsigned)L);
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, in, out, rows, cols, in_ld, out_ld, in_ls, out_ls);
  return hipGetLastError();
}

hipError_t launch_transpose(int L, const double *in, double *out, size_t rows, int cols, size_t in_ls,
                            size_t out_ls, hipStream_t st) {
  return launch_transpose_ld(L, in, (size_t)cols, out, rows, rows, cols, in_ls, out_ls, st);
}

hipError_t launch_gemm(int L, int n, const double *M, const double *B, size_t b_ls, double *N, int count,
                       hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const size_t threads = (size_t)n * n * 16;
  MD_DISPATCH(L, hipLaunchKernelGGL(gemm_kernel<LL>, dim3((threads + 255) / 256, count), dim3(256), 0, st, n, M, B,
                                    b_ls, N));
  return hipGetLastError();
}

bool stages_persistent(int L, int n, int D) { return (L == 2 || L == 4) && n <= 64 && D >= 1; }

int stages_sync_ints(int D) { return (D + 2 + 64) * SYNC_STRIDE; }

int stages_products(int L, int n, int D) {
  return stages_persistent(L, n, D) ? std::min(STAGE_PRODUCTS, D - 1) : std::min(1, D - 1);
}

// The counters of the persistent staged solve cleared ahead of it (a caller
// may issue this before it waits for the factorization, off the critical
// path, and then launch_stages with sync_ready).
hipError_t launch_stages_sync(int L, int n, int D, int *sync, double *dxT, hipStream_t st) {
  if (stages_persistent(L, n, D)) {
    const size_t cnt = std::max((size_t)stages_sync_ints(D), (size_t)L * n * D);
    hipLaunchKernelGGL(stages_prep_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, sync,
                       stages_sync_ints(D), dxT, (size_t)L * n * D);
  }
  return hipGetLastError();
}

hipError_t launch_stages(int L, int n, int D, const double *M, const double *NP, const double *At, double *rT,
                         double *dxT, int *sync, int32_t *status, hipStream_t st, bool sync_ready) {
  if (stages_persistent(L, n, D)) {
    const int Gs = (n + 1) / 2, Bm = (n + 15) / 16;
    // coefficient groups of the updaters: coefficients STAGE_PRODUCTS + 1 .. D - 1,
    // one per group up to 64 of them, else two
    const int C = D > STAGE_PRODUCTS + 1 ? D - STAGE_PRODUCTS - 1 : 0;
    const int Gm = C <= 64 ? C : (C + 1) / 2;
    const int G = Gs + Gm * Bm;  // at most 32 + 256 workgroups of 256 threads
    if (!sync_ready) {
      const hipError_t e = launch_stages_sync(L, n, D, sync, dxT, st);
      if (e != hipSuccess) return e;
    }
    if (L == 2)
      hipLaunchKernelGGL(stages_persistent_kernel<2>, dim3(G), dim3(256), 0, st, n, D, Gs, Gm, M, NP, At, rT, dxT,
                         sync, status);
    else
      hipLaunchKernelGGL(stages_persistent_kernel<4>, dim3(G), dim3(256), 0, st, n, D, Gs, Gm, M, NP, At, rT, dxT,
                         sync, status);
    return hipGetLastError();
  }
  const int crit_blocks = (n + 3) / 4;
  for (int k = 0; k < D; ++k) {
    const size_t bulk = (k == 0) ? 0 : (size_t)n * (D - k - 1) * 16;
    const unsigned blocks = (unsigned)(crit_blocks + (bulk + 255) / 256);
    MD_DISPATCH(L, hipLaunchKernelGGL(stage_kernel<LL>, dim3(blocks), dim3(256), 0, st, n, D, k, M, NP, At, rT, dxT));
  }
  return hipGetLastError();
}

hipError_t launch_gemm_next_x0(int L, int n, int D, const double *M, const double *B, size_t b_ls, double *N,
                               int count, const double *rT, const double *x, double *xn, int *done, hipStream_t st) {
  if (!stages_persistent(L, n, D) || count < 0) return hipErrorInvalidValue;
  const size_t threads = (size_t)n * n * 16;
  const unsigned bx = (unsigned)std::max<size_t>((threads + 255) / 256, (size_t)(n + 3) / 4);
  const dim3 grid(bx, count + 1), block(256);
  if (L == 2)
    hipLaunchKernelGGL(gemm_next_x0_kernel<2>, grid, block, 0, st, n, D, M, B, b_ls, N, rT, x, xn, done);
  else
    hipLaunchKernelGGL(gemm_next_x0_kernel<4>, grid, block, 0, st, n, D, M, B, b_ls, N, rT, x, xn, done);
  return hipGetLastError();
}

hipError_t launch_update(int L, int n, int D, int lo, int hi, const double *b, const double *dx, double *x,
                         double *norms, int32_t *status, hipStream_t st, const double *tsz, double *scale) {
  if (lo < 0 || hi > D || lo >= hi) return hipErrorInvalidValue;
  const int W = hi - lo;
  const size_t nW = (size_t)n * W;
  MD_DISPATCH(L, hipLaunchKernelGGL(update_kernel<LL>, dim3((nW + 255) / 256), dim3(256), 0, st, n, D, lo, W, dx, x));
  hipLaunchKernelGGL(norms_kernel, dim3(D), dim3(256), 0, st, n, D, lo, hi, b, dx, norms, status, tsz,
                     scale);
  return hipGetLastError();
}

hipError_t launch_finish(int L, int Ldx, int n, int D, int lo, int hi, const double *dxT, double *dx, double *x,
                         const double *b, double *norms, int32_t *status, hipStream_t st, const double *tsz,
                         double *rel) {
  if (lo < 0 || hi > D || lo >= hi || n < 1) return hipErrorInvalidValue;
  const dim3 grid(D), block(256);
  if (Ldx == L) {
    MD_DISPATCH(L, hipLaunchKernelGGL((finish_kernel<LL, LL>), grid, block, 0, st, n, D, lo, hi, dxT, dx, x, b, norms,
                                      status, tsz, rel));
  } else if (L == 4 && Ldx == 2) {
    hipLaunchKernelGGL((finish_kernel<4, 2>), grid, block, 0, st, n, D, lo, hi, dxT, dx, x, b, norms, status, tsz, rel);
  } else if (L == 8 && Ldx == 2) {
    hipLaunchKernelGGL((finish_kernel<8, 2>), grid, block, 0, st, n, D, lo, hi, dxT, dx, x, b, norms, status, tsz, rel);
  } else if (L == 8 && Ldx == 4) {
    hipLaunchKernelGGL((finish_kernel<8, 4>), grid, block, 0, st, n, D, lo, hi, dxT, dx, x, b, norms, status, tsz, rel);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_report(int D, const double *norms, const double *scale, const int32_t *status, double *out,
                         hipStream_t st) {
  hipLaunchKernelGGL(report_kernel, dim3(1), dim3(256), 0, st, D, norms, scale, status, out);
  return hipGetLastError();
}

hipError_t launch_series_to_rev(int L, int n, int D, const double *in, double *out, hipStream_t st) {
  const size_t tot = (size_t)L * n * D;
  hipLaunchKernelGGL(series_to_rev_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, D, L, in, out);
  return hipGetLastError();
}

hipError_t launch_rev_to_series(int L, int n, int D, const double *in, double *out, hipStream_t st) {
  const size_t tot = (size_t)L * n * D;
  hipLaunchKernelGGL(rev_to_series_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, D, L, in, out);
  return hipGetLastError();
}

hipError_t launch_coef_grad(int L, int n, int D, int m, const int32_t *row_of, const double *lambda, const double *val,
                            double *grad, hipStream_t st) {
  MD_DISPATCH(L, hipLaunchKernelGGL(coef_grad_kernel<LL>, dim3((m + 63) / 64), dim3(64), 0, st, n, D, m, row_of,
                                    lambda, val, grad));
  return hipGetLastError();
}

hipError_t launch_unit_md(int L, int m, double *c, hipStream_t st) {
  hipLaunchKernelGGL(unit_md_kernel, dim3((L * m + 255) / 256), dim3(256), 0, st, L, m, c);
  return hipGetLastError();
}

hipError_t launch_dot(int L, int64_t count, const double *a, const double *b, double *c, hipStream_t st) {
  MD_DISPATCH(L, hipLaunchKernelGGL(dot_kernel<LL>, dim3(1), dim3(256), 0, st, count, a, b, c));
  return hipGetLastError();
}

hipError_t launch_arith(int L, int op, int64_t count, const double *a, const double *b, double *c, hipStream_t st) {
  const int64_t blocks = (count + 255) / 256;
  MD_DISPATCH(L, hipLaunchKernelGGL(arith_kernel<LL>, dim3((unsigned)blocks), dim3(256), 0, st, op, count, a, b, c));
  return hipGetLastError();
}

}  // namespace mdk
