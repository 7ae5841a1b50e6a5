// Newton steps for a batch of independent polynomial systems ("paths") of
// uneven size in one persistent launch.  The paper tracks many solution
// paths of a homotopy (Section 1); each path is one system p(x; c) = 0 with
// its own n, truncation degree d and monomials, and one step of every path
// is the Newton step of Section 2.
//
// Work decomposition.  A grid of G workgroups (G <= 2 per CU) takes paths
// from a queue, most expensive first, and runs the whole step of a path
// itself: the evaluation and differentiation by convolutions (the workers
// of evaldiff_dev.hpp), the assembly of b(t) and of the Jacobian series
// (coefficient-major, A_k contiguous), the Householder QR of A_0 with Q^T,
// M = R^{-1} Q^T, N = M A_1, the stages dx_k = M r_k - N dx_{k-1} with the
// later right-hand sides pushed r_m -= A_{m-k} dx_k, and x := x + dx.  Each
// workgroup has its own slot of device memory for the intermediates of one
// path, so the workspace is G slots, not one per path.  The phases of a path
// are separated by workgroup barriers only; no workgroup waits for another,
// and every workgroup leaves when the queue is empty.
//
// Mixed precision (Section 1): the residual and the update at L limbs, the
// Jacobian, the QR and the stages at Ls <= L limbs (the leading limb planes
// of x, cff and b).
//
// Tiles.  The multiply-add reductions of the QR updates, N and the stages
// use teams of T lanes per dot product, T in {4, 8, 16} chosen per size
// bucket of (n, D) by md_batch_autotune (default 8).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "evaldiff_dev.hpp"

namespace mdk {

struct PathMeta {
  int n, D, m, nnz;
  int poly_off, mon_off, ent_off, asm_off, asment_off;  // offsets into the packed tables
  long long x_off, cff_off;                              // offsets within a limb plane of x (cst) and cff
  int bucket;
};

struct BatchArgs {
  int P;                                   // paths to run (entries of order)
  const PathMeta *meta;
  const int32_t *order;
  const int32_t *poly_ptr, *mon_ptr, *var, *exp, *asm_ptr, *asm_ent;
  const int32_t *tile;                     // team lanes per bucket
  const double *cff, *cst;
  double *x;
  size_t x_ls, cff_ls;                     // limb strides of x (cst) and cff
  int32_t *status;                         // per path
  double *norms;                           // per path: max |b|, max |dx|
  char *slots;
  size_t slot_bytes;
  int *queue;
};

constexpr int BATCH_NT = 256;
constexpr int BATCH_MAXN = 128;  // rows per lane <= 2 in the back substitution

__host__ __device__ inline int size_bucket(int n, int D) {
  const int bn = n <= 32 ? 0 : (n <= 64 ? 1 : 2);
  const int bd = D <= 16 ? 0 : (D <= 32 ? 1 : 2);
  return bn * 3 + bd;
}
constexpr int BATCH_BUCKETS = 9;

// Sum of an accumulator over the whole workgroup (four wavefronts), the
// renormalized total in every thread.
template <int L>
__device__ void block_sum_lazy(double (&u)[L], double (&r)[L], double *sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  team_sum_lazy<L>(u, 64);
  __syncthreads();  // sh may still be read from the previous call
  if (lane == 0)
#pragma unroll
    for (int l = 0; l < L; ++l) sh[wv * L + l] = u[l];
  __syncthreads();
  double t[L];
#pragma unroll
  for (int l = 0; l < L; ++l) t[l] = sh[l];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
    double o[L];
#pragma unroll
    for (int l = 0; l < L; ++l) o[l] = sh[w * L + l];
    MD<L>::add_lazy(t, o);
  }
  MD<L>::renorm(t, r);
}

__device__ double block_max(double v, double *sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, sh[w]);
  return r;
}

template <int L, int Ls>
__device__ void path_step(const BatchArgs &B, const PathMeta &pm, int p, double *slot, double *lds, double *shr,
                          int &sh_sing) {
  const int tid = threadIdx.x, NT = blockDim.x;
  const int n = pm.n, D = pm.D, m = pm.m, nnz = pm.nnz;
  const int T = B.tile[pm.bucket];
  const int team = tid / T, tl = tid % T, nteams = NT / T;
  const size_t nn = (size_t)n * n, nD = (size_t)n * D, nnD = nn * D;
  size_t off = 0;
  auto take = [&](size_t cnt) {
    double *q = slot + off;
    off += (cnt + 31) & ~(size_t)31;
    return q;
  };
  double *val = take((size_t)L * m * D), *der = take((size_t)L * nnz * D), *b = take((size_t)L * nD);
  double *At = take((size_t)Ls * nnD), *qr = take((size_t)Ls * nn), *qt = take((size_t)Ls * nn);
  double *tau = take((size_t)Ls * n), *invd = take((size_t)Ls * n), *M = take((size_t)Ls * nn);
  double *N = take((size_t)Ls * nn), *r = take((size_t)Ls * nD), *dx = take((size_t)Ls * nD);
  const int32_t *poly_ptr = B.poly_ptr + pm.poly_off, *asm_ptr = B.asm_ptr + pm.asm_off;
  const int32_t *asm_ent = B.asm_ent + pm.asment_off;
  const double *cst = B.cst + pm.x_off;
  double *x = B.x + pm.x_off;
  if (tid == 0) sh_sing = 0;

  // 1. evaluation: values at L limbs (with the derivatives when Ls == L)
  EvalArgs a;
  a.n = n;
  a.D = D;
  a.Dc = D;
  a.m = m;
  a.nnz = nnz;
  a.mon_ptr = B.mon_ptr + pm.mon_off;
  a.var = B.var + pm.ent_off;
  a.exp = B.exp + pm.ent_off;
  a.order = a.mon_ptr;  // not read: monomials are addressed directly
  a.cff = B.cff + pm.cff_off;
  a.x = x;
  a.pw = x;  // not read: batched paths have exponents of at most 2, no power table
  a.val = val;
  a.der = der;
  a.x_ls = B.x_ls;
  a.cff_ls = B.cff_ls;
  a.values_only = (Ls == L) ? 0 : 1;
  {
    const int Gw = worker_lanes(D), wpb = NT / Gw, wid = tid / Gw, wl = tid - wid * Gw;
    double *wbuf = lds + (size_t)wid * 3 * L * (D + 1);
    for (int mono = wid; mono < m; mono += wpb) eval_monomial<L>(a, mono, wl, wbuf);
  }
  __syncthreads();
  // 2. b = -(c_0 + sum of the row's monomial values), L limbs
  for (int q = tid; q < (int)nD; q += NT) {
    const int i = q / D, s = q - i * D;
    double acc[L];
    ld<L>(cst, B.x_ls, (size_t)q, acc);
    for (int mj = poly_ptr[i]; mj < poly_ptr[i + 1]; ++mj) {
      double v[L], t[L];
      ld<L>(val, (size_t)m * D, (size_t)mj * D + s, v);
      MD<L>::add(acc, v, t);
      md::copy<L>(t, acc);
    }
    md::neg<L>(acc, acc);
    st<L>(b, nD, q, acc);
  }
  __syncthreads();
  if (Ls != L) {  // the derivatives at Ls limbs
    a.values_only = 0;
    const int Gw = worker_lanes(D), wpb = NT / Gw, wid = tid / Gw, wl = tid - wid * Gw;
    double *wbuf = lds + (size_t)wid * 3 * Ls * (D + 1);
    for (int mono = wid; mono < m; mono += wpb) eval_monomial<Ls>(a, mono, wl, wbuf);
    __syncthreads();
  }
  // 3. the Jacobian series, coefficient-major At[k][i][j]; A_0 into qr, I into qt
  for (size_t q = tid; q < nnD; q += NT) {
    const size_t ij = q / D;
    const int s = (int)(q - ij * D);
    double acc[Ls];
    md::zero<Ls>(acc);
    const int lo = asm_ptr[ij], hi = asm_ptr[ij + 1];
    if (lo < hi) {
      ld<Ls>(der, (size_t)nnz * D, (size_t)asm_ent[lo] * D + s, acc);
      for (int t = lo + 1; t < hi; ++t) {
        double v[Ls], w[Ls];
        ld<Ls>(der, (size_t)nnz * D, (size_t)asm_ent[t] * D + s, v);
        MD<Ls>::add(acc, v, w);
        md::copy<Ls>(w, acc);
      }
    }
    st<Ls>(At, nnD, (size_t)s * nn + ij, acc);
    if (s == 0) {
      st<Ls>(qr, nn, ij, acc);
      const int i = (int)(ij / n), j = (int)(ij - (size_t)i * n);
#pragma unroll
      for (int l = 0; l < Ls; ++l) qt[(size_t)l * nn + ij] = (l == 0 && i == j) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  // 4. Householder QR of A_0 (row-major, in place) with Q^T
  for (int c = 0; c < n; ++c) {
    double u[Ls], nrm2[Ls];
    md::zero<Ls>(u);
    for (int i = c + tid; i < n; i += NT) {
      double xi[Ls];
      ld<Ls>(qr, nn, (size_t)i * n + c, xi);
      MD<Ls>::fma_lazy(u, xi, xi);
    }
    block_sum_lazy<Ls>(u, nrm2, shr);
    if (tid == 0) {
      double x0[Ls], beta[Ls], tc[Ls], inv[Ls];
      ld<Ls>(qr, nn, (size_t)c * n + c, x0);
      if (!(nrm2[0] > 0.0)) {
        md::copy<Ls>(x0, beta);
        md::zero<Ls>(tc);
        md::zero<Ls>(inv);
        sh_sing = 1;
      } else {
        double y[Ls], alpha[Ls], v0[Ls];
        md::rsqrt_newton<Ls>(nrm2, y);
        MD<Ls>::mul(nrm2, y, alpha);
        const bool nonneg = x0[0] >= 0.0;
        if (nonneg) md::neg<Ls>(alpha, beta);
        else md::copy<Ls>(alpha, beta);
        MD<Ls>::sub(x0, beta, v0);
        MD<Ls>::mul(v0, y, tc);
        if (!nonneg) md::neg<Ls>(tc, tc);
        md::recip_newton<Ls>(v0, inv);
      }
#pragma unroll
      for (int l = 0; l < Ls; ++l) {
        shr[8 * 8 + l] = inv[l];
        shr[8 * 8 + 8 + l] = tc[l];
        tau[(size_t)l * n + c] = tc[l];
      }
      st<Ls>(qr, nn, (size_t)c * n + c, beta);
    }
    __syncthreads();
    double inv[Ls], tc[Ls];
#pragma unroll
    for (int l = 0; l < Ls; ++l) {
      inv[l] = shr[8 * 8 + l];
      tc[l] = shr[8 * 8 + 8 + l];
    }
    for (int i = c + 1 + tid; i < n; i += NT) {  // v below the diagonal
      double xi[Ls], vi[Ls];
      ld<Ls>(qr, nn, (size_t)i * n + c, xi);
      MD<Ls>::mul(xi, inv, vi);
      st<Ls>(qr, nn, (size_t)i * n + c, vi);
    }
    __syncthreads();
    // apply H_c to the trailing columns of A_0 and to every column of Q^T
    const int na = n - 1 - c;
    for (int col = team; col < na + n; col += nteams) {
      double *base = col < na ? qr : qt;
      const int j = col < na ? c + 1 + col : col - na;
      double acc[Ls], dot[Ls], w[Ls];
      md::zero<Ls>(acc);
      for (int i = c + tl; i < n; i += T) {
        double vi[Ls], xv[Ls];
        if (i == c) {
          md::zero<Ls>(vi);
          vi[0] = 1.0;
        } else {
          ld<Ls>(qr, nn, (size_t)i * n + c, vi);
        }
        ld<Ls>(base, nn, (size_t)i * n + j, xv);
        MD<Ls>::fma_lazy(acc, vi, xv);
      }
      team_sum_lazy<Ls>(acc, T);
      MD<Ls>::renorm(acc, dot);
      MD<Ls>::mul(dot, tc, w);
      for (int i = c + tl; i < n; i += T) {
        double vi[Ls], xv[Ls];
        if (i == c) {
          md::zero<Ls>(vi);
          vi[0] = 1.0;
        } else {
          ld<Ls>(qr, nn, (size_t)i * n + c, vi);
        }
        ld<Ls>(base, nn, (size_t)i * n + j, xv);
        MD<Ls>::fms(xv, vi, w);
        st<Ls>(base, nn, (size_t)i * n + j, xv);
      }
    }
    __syncthreads();
  }
  // 5. reciprocals of diag(R), with the singularity test of the single-system path
  {
    double dmax = 0.0;
    for (int i = tid; i < n; i += NT) dmax = fmax(dmax, fabs(qr[(size_t)i * n + i]));
    dmax = block_max(dmax, shr);
    for (int i = tid; i < n; i += NT) {
      double rii[Ls], q[Ls];
      ld<Ls>(qr, nn, (size_t)i * n + i, rii);
      if (!(fabs(rii[0]) > ldexp((double)n, -53 * Ls) * dmax)) {
        md::zero<Ls>(q);
        sh_sing = 1;
      } else {
        md::recip_newton<Ls>(rii, q);
      }
      st<Ls>(invd, n, i, q);
    }
  }
  __syncthreads();
  // 6. M = R^{-1} Q^T: one wavefront per column, rows in lanes (p and p + 64)
  {
    const int lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
    for (int c = wv; c < n; c += nw) {
      double y0[Ls], y1[Ls];
      md::zero<Ls>(y0);
      md::zero<Ls>(y1);
      if (lane < n) ld<Ls>(qt, nn, (size_t)lane * n + c, y0);
      if (lane + 64 < n) ld<Ls>(qt, nn, (size_t)(lane + 64) * n + c, y1);
      for (int i = n - 1; i >= 0; --i) {
        double z[Ls], zi[Ls];
        md::zero<Ls>(z);
        const bool hi = i >= 64;
        const int src = hi ? i - 64 : i;
        if (lane == src) {
          double d[Ls];
          ld<Ls>(invd, n, i, d);
          if (hi) {
            MD<Ls>::mul(y1, d, z);
            md::copy<Ls>(z, y1);
          } else {
            MD<Ls>::mul(y0, d, z);
            md::copy<Ls>(z, y0);
          }
        }
#pragma unroll
        for (int l = 0; l < Ls; ++l) zi[l] = __shfl(z[l], src, 64);
        if (lane < i) {
          double rp[Ls];
          ld<Ls>(qr, nn, (size_t)lane * n + i, rp);
          MD<Ls>::fms(y0, rp, zi);
        }
        if (lane + 64 < i) {
          double rp[Ls];
          ld<Ls>(qr, nn, (size_t)(lane + 64) * n + i, rp);
          MD<Ls>::fms(y1, rp, zi);
        }
      }
      if (lane < n) st<Ls>(M, nn, (size_t)lane * n + c, y0);
      if (lane + 64 < n) st<Ls>(M, nn, (size_t)(lane + 64) * n + c, y1);
    }
  }
  __syncthreads();
  // 7. N = M A_1
  if (D > 1)
    for (int task = team; task < (int)nn; task += nteams) {
      const int i = task / n, j = task - i * n;
      double acc[Ls], s2[Ls];
      md::zero<Ls>(acc);
      for (int v = tl; v < n; v += T) {
        double mv[Ls], av[Ls];
        ld<Ls>(M, nn, (size_t)i * n + v, mv);
        ld<Ls>(At, nnD, nn + (size_t)v * n + j, av);
        MD<Ls>::fma_lazy(acc, mv, av);
      }
      team_sum_lazy<Ls>(acc, T);
      MD<Ls>::renorm(acc, s2);
      if (tl == 0) st<Ls>(N, nn, (size_t)i * n + j, s2);
    }
  // right-hand sides, coefficient-major r[k][i] (leading Ls limbs of b)
  for (int q = tid; q < (int)nD; q += NT) {
    const int i = q / D, s = q - i * D;
#pragma unroll
    for (int l = 0; l < Ls; ++l) r[(size_t)l * nD + (size_t)s * n + i] = b[(size_t)l * nD + q];
  }
  __syncthreads();
  // 8. stages
  for (int k = 0; k < D; ++k) {
    for (int i = team; i < n; i += nteams) {
      double acc[Ls], s2[Ls];
      md::zero<Ls>(acc);
      for (int v = tl; v < n; v += T) {
        double mv[Ls], rv[Ls];
        ld<Ls>(M, nn, (size_t)i * n + v, mv);
        ld<Ls>(r, nD, (size_t)k * n + v, rv);
        MD<Ls>::fma_lazy(acc, mv, rv);
        if (k > 0) {
          double nv[Ls], xv[Ls];
          ld<Ls>(N, nn, (size_t)i * n + v, nv);
          md::neg<Ls>(nv, nv);
          ld<Ls>(dx, nD, (size_t)(k - 1) * n + v, xv);
          MD<Ls>::fma_lazy(acc, nv, xv);
        }
      }
      team_sum_lazy<Ls>(acc, T);
      MD<Ls>::renorm(acc, s2);
      if (tl == 0) st<Ls>(dx, nD, (size_t)k * n + i, s2);
    }
    __syncthreads();
    // r_m -= A_{m-k} dx_k for m >= k + 2 (the term m = k + 1 is N dx_k)
    const int ntask = (D - k - 2) * n;
    for (int task = team; task < ntask; task += nteams) {
      const int mm = k + 2 + task / n, i = task % n;
      double acc[Ls], s2[Ls];
      md::zero<Ls>(acc);
      for (int v = tl; v < n; v += T) {
        double av[Ls], xv[Ls];
        ld<Ls>(At, nnD, (size_t)(mm - k) * nn + (size_t)i * n + v, av);
        ld<Ls>(dx, nD, (size_t)k * n + v, xv);
        MD<Ls>::fma_lazy(acc, av, xv);
      }
      team_sum_lazy<Ls>(acc, T);
      MD<Ls>::renorm(acc, s2);
      if (tl == 0) {
        double rv[Ls], t2[Ls];
        ld<Ls>(r, nD, (size_t)mm * n + i, rv);
        MD<Ls>::sub(rv, s2, t2);
        st<Ls>(r, nD, (size_t)mm * n + i, t2);
      }
    }
    __syncthreads();
  }
  // 9. x := x + dx, norms and status
  double nb = 0.0, nx = 0.0;
  bool finite = true;
  for (int q = tid; q < (int)nD; q += NT) {
    const int i = q / D, s = q - i * D;
    double xv[L], d[Ls], dw[L], t[L];
    ld<L>(x, B.x_ls, (size_t)q, xv);
#pragma unroll
    for (int l = 0; l < Ls; ++l) d[l] = dx[(size_t)l * nD + (size_t)s * n + i];
    md::widen<Ls>(d, dw);
    MD<L>::add(xv, dw, t);
    st<L>(x, B.x_ls, (size_t)q, t);
    const double bq = b[q];
    finite = finite && isfinite(bq) && isfinite(d[0]);
    nb = fmax(nb, fabs(bq));
    nx = fmax(nx, fabs(d[0]));
  }
  nb = block_max(nb, shr);
  nx = block_max(nx, shr);
  const double fin = block_max(finite ? 0.0 : 1.0, shr);
  if (tid == 0) {
    B.norms[2 * (size_t)p] = nb;
    B.norms[2 * (size_t)p + 1] = nx;
    B.status[p] = sh_sing ? MD_ESINGULAR : (fin > 0.0 ? MD_ENONFINITE : MD_OK);
  }
  __syncthreads();
}

template <int L, int Ls>
__global__ void __launch_bounds__(BATCH_NT) batch_step_kernel(BatchArgs B) {
  extern __shared__ double lds[];
  __shared__ double shr[8 * 8 + 16];
  __shared__ int sh_idx, sh_sing;
  double *slot = reinterpret_cast<double *>(B.slots + (size_t)blockIdx.x * B.slot_bytes);
  while (true) {
    if (threadIdx.x == 0) sh_idx = atomicAdd(B.queue, 1);
    __syncthreads();
    const int idx = sh_idx;
    __syncthreads();
    if (idx >= B.P) return;
    const int p = B.order[idx];
    const PathMeta pm = B.meta[p];
    path_step<L, Ls>(B, pm, p, slot, lds, shr, sh_sing);
  }
}

__global__ void batch_reset_kernel(int *queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

size_t batch_eval_lds_bytes(int L, int maxD) {
  size_t best = 0;
  for (int D = 1; D <= maxD; ++D) {
    const size_t wpb = BATCH_NT / worker_lanes(D);
    best = std::max(best, wpb * 3 * L * (D + 1) * sizeof(double));
  }
  return best;
}

}  // namespace mdk

// ------------------------------------------------------------------ host API

struct md_batch {
  int L, P, G;
  int maxn, maxD, maxm, maxnnz;
  std::vector<mdk::PathMeta> meta;
  std::vector<int32_t> order;             // all paths, most expensive first
  std::vector<double> cost;
  int32_t tile[mdk::BATCH_BUCKETS];
  long long x_total, cff_total;
  size_t slot_bytes;
  mdk::PathMeta *d_meta = nullptr;
  int32_t *d_order = nullptr, *d_tables = nullptr, *d_tile = nullptr;
  const int32_t *d_poly_ptr = nullptr, *d_mon_ptr = nullptr, *d_var = nullptr, *d_exp = nullptr;
  const int32_t *d_asm_ptr = nullptr, *d_asm_ent = nullptr;
  // one captured step (graph) for a fixed set of arguments
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *key[8] = {nullptr};
  int key_prec = 0;
  bool seen = false;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t slot_doubles(int L, int Ls, int n, int D, int m, int nnz) {
  auto r = [](size_t c) { return (c + 31) & ~(size_t)31; };
  const size_t nn = (size_t)n * n, nD = (size_t)n * D;
  return r((size_t)L * m * D) + r((size_t)L * nnz * D) + r((size_t)L * nD) + r((size_t)Ls * nn * D) +
         3 * r((size_t)Ls * nn) + 2 * r((size_t)Ls * n) + r((size_t)Ls * nn) + 2 * r((size_t)Ls * nD);
}

// workspace: [queue (256 B)][G slots]
size_t batch_ws_bytes(const md_batch *b) { return 256 + (size_t)b->G * b->slot_bytes; }

hipError_t launch_step(const md_batch *b, int Ls, const int32_t *order, int P, const double *cff, const double *cst,
                       double *x, int32_t *status, double *norms, void *ws, hipStream_t st) {
  mdk::BatchArgs A;
  A.P = P;
  A.meta = b->d_meta;
  A.order = order;
  A.poly_ptr = b->d_poly_ptr;
  A.mon_ptr = b->d_mon_ptr;
  A.var = b->d_var;
  A.exp = b->d_exp;
  A.asm_ptr = b->d_asm_ptr;
  A.asm_ent = b->d_asm_ent;
  A.tile = b->d_tile;
  A.cff = cff;
  A.cst = cst;
  A.x = x;
  A.x_ls = (size_t)b->x_total;
  A.cff_ls = (size_t)b->cff_total;
  A.status = status;
  A.norms = norms;
  A.queue = static_cast<int *>(ws);
  A.slots = static_cast<char *>(ws) + 256;
  A.slot_bytes = b->slot_bytes;
  const size_t lds = mdk::batch_eval_lds_bytes(b->L, b->maxD);
  const int G = std::min(b->G, P);
  if (G <= 0) return hipSuccess;
  hipLaunchKernelGGL(mdk::batch_reset_kernel, dim3(1), dim3(64), 0, st, A.queue);
  if (b->L == 2) {
    hipLaunchKernelGGL((mdk::batch_step_kernel<2, 2>), dim3(G), dim3(mdk::BATCH_NT), lds, st, A);
  } else if (Ls == 4) {
    hipLaunchKernelGGL((mdk::batch_step_kernel<4, 4>), dim3(G), dim3(mdk::BATCH_NT), lds, st, A);
  } else {
    hipLaunchKernelGGL((mdk::batch_step_kernel<4, 2>), dim3(G), dim3(mdk::BATCH_NT), lds, st, A);
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

int md_batch_create(int prec, int npaths, const int32_t *n, const int32_t *d, const int32_t *m,
                    const int32_t *poly_ptr, const int32_t *mon_ptr, const int32_t *var, const int32_t *exp,
                    md_batch **out) {
  if (!out) return mdk::api_fail(MD_EINVAL, "NULL argument");
  *out = nullptr;
  if (prec != MD_DD && prec != MD_QD) return mdk::api_fail(MD_EINVAL, "batches run in double or quad double");
  if (npaths < 1 || !n || !d || !m || !poly_ptr || !mon_ptr) return mdk::api_fail(MD_EINVAL, "bad batch description");
  md_batch *b = new md_batch();
  b->L = prec;
  b->P = npaths;
  b->maxn = b->maxD = b->maxm = b->maxnnz = 0;
  std::vector<int32_t> tab_poly, tab_mon, tab_var, tab_exp, tab_asm, tab_asment;
  long long xo = 0, co = 0;
  size_t poly_o = 0, mon_o = 0, ent_o = 0;
  for (int p = 0; p < npaths; ++p) {
    const int np = n[p], Dp = d[p] + 1, mp = m[p];
    if (np < 1 || np > mdk::BATCH_MAXN || d[p] < 0 || Dp > MD_MAX_COEFFS || mp < 0) {
      delete b;
      return mdk::api_fail(MD_EINVAL, "path size out of range (1 <= n <= 128, 0 <= d < 128)");
    }
    const int32_t *pp = poly_ptr + poly_o, *mpt = mon_ptr + mon_o;
    if (pp[0] != 0 || pp[np] != mp || mpt[0] != 0) {
      delete b;
      return mdk::api_fail(MD_EINVAL, "poly_ptr / mon_ptr of a path must start at 0 and cover its monomials");
    }
    for (int i = 0; i < np; ++i)
      if (pp[i + 1] < pp[i]) {
        delete b;
        return mdk::api_fail(MD_EINVAL, "poly_ptr must be nondecreasing");
      }
    const int nnz = mpt[mp];
    if (nnz < 0 || (nnz > 0 && (!var || !exp))) {
      delete b;
      return mdk::api_fail(MD_EINVAL, "bad monomial supports");
    }
    std::vector<int32_t> cnt((size_t)np * np + 1, 0);
    double cost = 0.0;
    for (int j = 0; j < mp; ++j) {
      if (mpt[j + 1] < mpt[j]) {
        delete b;
        return mdk::api_fail(MD_EINVAL, "mon_ptr must be nondecreasing");
      }
      const int k = mpt[j + 1] - mpt[j];
      cost += (double)std::max(1, 3 * k - 5) * Dp * Dp;
      for (int q = mpt[j]; q < mpt[j + 1]; ++q) {
        const int v = var[ent_o + q], e = exp[ent_o + q];
        if (v < 0 || v >= np || (q > mpt[j] && v <= var[ent_o + q - 1])) {
          delete b;
          return mdk::api_fail(MD_EINVAL, "variables must be in range and strictly increasing per monomial");
        }
        if (e < 1 || e > 2) {
          delete b;
          return mdk::api_fail(MD_EINVAL, "batched paths take exponents 1 and 2");
        }
      }
    }
    // assembly lists of the path: entries contributing to (row i, column v), monomial order
    std::vector<int32_t> rowof(mp, 0);
    for (int i = 0; i < np; ++i)
      for (int j = pp[i]; j < pp[i + 1]; ++j) rowof[j] = i;
    std::vector<std::vector<int32_t>> lists((size_t)np * np);
    for (int j = 0; j < mp; ++j)
      for (int q = mpt[j]; q < mpt[j + 1]; ++q) lists[(size_t)rowof[j] * np + var[ent_o + q]].push_back(q);
    mdk::PathMeta pm;
    pm.n = np;
    pm.D = Dp;
    pm.m = mp;
    pm.nnz = nnz;
    pm.poly_off = (int)tab_poly.size();
    pm.mon_off = (int)tab_mon.size();
    pm.ent_off = (int)tab_var.size();
    pm.asm_off = (int)tab_asm.size();
    pm.asment_off = (int)tab_asment.size();
    pm.x_off = xo;
    pm.cff_off = co;
    pm.bucket = mdk::size_bucket(np, Dp);
    tab_poly.insert(tab_poly.end(), pp, pp + np + 1);
    tab_mon.insert(tab_mon.end(), mpt, mpt + mp + 1);
    tab_var.insert(tab_var.end(), var + ent_o, var + ent_o + nnz);
    tab_exp.insert(tab_exp.end(), exp + ent_o, exp + ent_o + nnz);
    int32_t acc = 0;
    for (size_t ij = 0; ij < (size_t)np * np; ++ij) {
      tab_asm.push_back(acc);
      for (int32_t e : lists[ij]) tab_asment.push_back(e);
      acc += (int32_t)lists[ij].size();
    }
    tab_asm.push_back(acc);
    b->meta.push_back(pm);
    cost += (double)np * np * Dp * Dp / 2 + (double)np * np * np;
    b->cost.push_back(cost);
    b->maxn = std::max(b->maxn, np);
    b->maxD = std::max(b->maxD, Dp);
    b->maxm = std::max(b->maxm, mp);
    b->maxnnz = std::max(b->maxnnz, nnz);
    xo += (long long)np * Dp;
    co += mp;
    poly_o += np + 1;
    mon_o += mp + 1;
    ent_o += nnz;
  }
  b->x_total = xo;
  b->cff_total = co;
  b->order.resize(npaths);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a2, int b2) { return b->cost[a2] > b->cost[b2]; });
  for (int q = 0; q < mdk::BATCH_BUCKETS; ++q) b->tile[q] = 8;
  size_t slot = 0;
  for (const auto &pm : b->meta)
    slot = std::max(slot, slot_doubles(b->L, b->L, pm.n, pm.D, pm.m, pm.nnz) * sizeof(double));
  b->slot_bytes = align256(slot);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    delete b;
    return mdk::api_hip_fail(e, "device query");
  }
  b->G = std::min(npaths, 2 * std::max(cus, 1));
  // device tables: meta, order, tile, then the int tables
  const size_t nt = tab_poly.size() + tab_mon.size() + tab_var.size() + tab_exp.size() + tab_asm.size() +
                    tab_asment.size();
  std::vector<int32_t> all;
  all.reserve(nt + npaths + mdk::BATCH_BUCKETS);
  auto seg = [&](const std::vector<int32_t> &v) {
    size_t o = all.size();
    all.insert(all.end(), v.begin(), v.end());
    return o;
  };
  const size_t o_poly = seg(tab_poly), o_mon = seg(tab_mon), o_var = seg(tab_var), o_exp = seg(tab_exp),
               o_asm = seg(tab_asm), o_ase = seg(tab_asment), o_ord = seg(b->order);
  std::vector<int32_t> tl(b->tile, b->tile + mdk::BATCH_BUCKETS);
  const size_t o_tile = seg(tl);
  if ((e = hipMalloc((void **)&b->d_tables, std::max<size_t>(all.size(), 1) * sizeof(int32_t))) != hipSuccess ||
      (e = hipMemcpy(b->d_tables, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMalloc((void **)&b->d_meta, b->meta.size() * sizeof(mdk::PathMeta))) != hipSuccess ||
      (e = hipMemcpy(b->d_meta, b->meta.data(), b->meta.size() * sizeof(mdk::PathMeta), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) {
    if (b->d_tables) (void)hipFree(b->d_tables);
    if (b->d_meta) (void)hipFree(b->d_meta);
    delete b;
    return mdk::api_hip_fail(e, "batch setup");
  }
  b->d_poly_ptr = b->d_tables + o_poly;
  b->d_mon_ptr = b->d_tables + o_mon;
  b->d_var = b->d_tables + o_var;
  b->d_exp = b->d_tables + o_exp;
  b->d_asm_ptr = b->d_tables + o_asm;
  b->d_asm_ent = b->d_tables + o_ase;
  b->d_order = b->d_tables + o_ord;
  b->d_tile = b->d_tables + o_tile;
  static bool attr = false;
  if (!attr) {  // dynamic LDS of the evaluation workers above 64 KB needs the attribute
    (void)hipFuncSetAttribute((const void *)mdk::batch_step_kernel<2, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              150 * 1024);
    (void)hipFuncSetAttribute((const void *)mdk::batch_step_kernel<4, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              150 * 1024);
    (void)hipFuncSetAttribute((const void *)mdk::batch_step_kernel<4, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              150 * 1024);
    (void)hipGetLastError();
    attr = true;
  }
  *out = b;
  return MD_OK;
}

int md_batch_destroy(md_batch *b) {
  if (!b) return MD_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_tables) (void)hipFree(b->d_tables);
  if (b->d_meta) (void)hipFree(b->d_meta);
  delete b;
  return MD_OK;
}

int md_batch_offsets(const md_batch *b, int64_t *x_off, int64_t *cff_off, int64_t *x_total, int64_t *cff_total) {
  if (!b) return mdk::api_fail(MD_EINVAL, "NULL batch");
  for (int p = 0; p < b->P; ++p) {
    if (x_off) x_off[p] = b->meta[p].x_off;
    if (cff_off) cff_off[p] = b->meta[p].cff_off;
  }
  if (x_total) *x_total = b->x_total;
  if (cff_total) *cff_total = b->cff_total;
  return MD_OK;
}

int md_batch_workspace_size(const md_batch *b, size_t *bytes) {
  if (!b || !bytes) return mdk::api_fail(MD_EINVAL, "NULL argument");
  *bytes = batch_ws_bytes(b);
  return MD_OK;
}

int md_batch_newton_step(md_batch *b, int prec_solve, const double *cff, const double *cst, double *x,
                         int32_t *dev_status, double *dev_norms, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!b || !cff || !cst || !x || !dev_status || !dev_norms) return mdk::api_fail(MD_EINVAL, "NULL argument");
  if (!(prec_solve == b->L || (b->L == MD_QD && prec_solve == MD_DD)))
    return mdk::api_fail(MD_EINVAL, "solve precision: the batch's, or double double under quad double");
  if (!ws || ws_bytes < batch_ws_bytes(b)) return mdk::api_fail(MD_ENOSPACE, "workspace too small");
  // the step is two launches, replayed from a captured graph while the
  // arguments stay the same (captured on the second call with them)
  const void *key[8] = {cff, cst, x, dev_status, dev_norms, ws, nullptr, nullptr};
  bool same = b->key_prec == prec_solve;
  for (int q = 0; q < 8; ++q) same = same && key[q] == b->key[q];
  hipError_t e;
  if (same && b->exec) {
    e = hipGraphLaunch(b->exec, st);
    return e == hipSuccess ? MD_OK : mdk::api_hip_fail(e, "graph launch");
  }
  if (same && b->seen && !mdk::api_timing_enabled()) {
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return mdk::api_hip_fail(e, "capture");
    hipError_t le = launch_step(b, prec_solve, b->d_order, b->P, cff, cst, x, dev_status, dev_norms, ws, b->cap);
    e = hipStreamEndCapture(b->cap, &g);
    if (le != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return mdk::api_hip_fail(le != hipSuccess ? le : e, "capture");
    }
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return mdk::api_hip_fail(e, "graph instantiate");
    }
    e = hipGraphLaunch(b->exec, st);
    return e == hipSuccess ? MD_OK : mdk::api_hip_fail(e, "graph launch");
  }
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  for (int q = 0; q < 8; ++q) b->key[q] = key[q];
  b->key_prec = prec_solve;
  b->seen = true;
  e = launch_step(b, prec_solve, b->d_order, b->P, cff, cst, x, dev_status, dev_norms, ws, st);
  return e == hipSuccess ? MD_OK : mdk::api_hip_fail(e, "batched step");
}

int md_batch_autotune(md_batch *b, int prec_solve, const double *cff, const double *cst, const double *x,
                      double *x_scratch, int32_t *dev_status, double *dev_norms, void *ws, size_t ws_bytes,
                      hipStream_t st, int32_t *chosen) {
  if (!b || !cff || !cst || !x || !x_scratch || !dev_status || !dev_norms) return mdk::api_fail(MD_EINVAL, "NULL argument");
  if (!(prec_solve == b->L || (b->L == MD_QD && prec_solve == MD_DD)))
    return mdk::api_fail(MD_EINVAL, "solve precision: the batch's, or double double under quad double");
  if (!ws || ws_bytes < batch_ws_bytes(b)) return mdk::api_fail(MD_ENOSPACE, "workspace too small");
  static const int cand[3] = {4, 8, 16};
  const size_t xbytes = (size_t)b->L * b->x_total * sizeof(double);
  hipError_t e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int32_t *d_list = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess ||
      (e = hipMalloc((void **)&d_list, (size_t)b->P * sizeof(int32_t))) != hipSuccess)
    return mdk::api_hip_fail(e, "autotune setup");
  for (int bk = 0; bk < mdk::BATCH_BUCKETS; ++bk) {
    std::vector<int32_t> list;
    for (int32_t p : b->order)
      if (b->meta[p].bucket == bk) list.push_back(p);
    if (list.empty()) continue;
    if ((e = hipMemcpy(d_list, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) break;
    float best = 0.0f;
    int best_t = b->tile[bk];
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
      b->tile[bk] = cand[c];
      if ((e = hipMemcpy(const_cast<int32_t *>(b->d_tile), b->tile, sizeof(b->tile), hipMemcpyHostToDevice)) !=
          hipSuccess)
        break;
      float ms = 0.0f;
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
        if ((e = hipMemcpyAsync(x_scratch, x, xbytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) break;
        if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
        if ((e = launch_step(b, prec_solve, d_list, (int)list.size(), cff, cst, x_scratch, dev_status, dev_norms, ws,
                             st)) != hipSuccess)
          break;
        if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) break;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      }
      if (e == hipSuccess && (c == 0 || ms < best)) {
        best = ms;
        best_t = cand[c];
      }
    }
    b->tile[bk] = best_t;
  }
  if (e == hipSuccess)
    e = hipMemcpy(const_cast<int32_t *>(b->d_tile), b->tile, sizeof(b->tile), hipMemcpyHostToDevice);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_list);
  if (e != hipSuccess) return mdk::api_hip_fail(e, "autotune");
  if (chosen)
    for (int q = 0; q < mdk::BATCH_BUCKETS; ++q) chosen[q] = b->tile[q];
  if (b->exec) {  // a captured step holds the old launch; capture again
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->seen = false;
  }
  return MD_OK;
}

int md_batch_set_tiles(md_batch *b, const int32_t *tiles) {
  if (!b || !tiles) return mdk::api_fail(MD_EINVAL, "NULL argument");
  for (int q = 0; q < mdk::BATCH_BUCKETS; ++q)
    if (tiles[q] != 4 && tiles[q] != 8 && tiles[q] != 16) return mdk::api_fail(MD_EINVAL, "tiles are 4, 8 or 16 lanes");
  std::memcpy(b->tile, tiles, sizeof(b->tile));
  hipError_t e = hipMemcpy(const_cast<int32_t *>(b->d_tile), b->tile, sizeof(b->tile), hipMemcpyHostToDevice);
  if (e != hipSuccess) return mdk::api_hip_fail(e, "tiles");
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->seen = false;
  }
  return MD_OK;
}

}  // extern "C"
