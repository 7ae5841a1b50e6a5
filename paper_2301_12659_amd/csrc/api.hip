// The C interface of libmdnewton (declared in include/mdnewton.h): plan
// construction and validation, workspace layout, and the sequence of kernel
// launches for one Newton step (Section 2).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"



struct md_plan {
  int L, n, d, D, m, nnz, maxexp, maxk;
  int32_t *d_poly_ptr = nullptr, *d_mon_ptr = nullptr, *d_var = nullptr, *d_exp = nullptr;
  int32_t *d_order = nullptr, *d_asm_ptr = nullptr, *d_asm_ent = nullptr, *d_row_of = nullptr;
  // second stream of the Newton step: QR of A_0 and M run beside the full
  // evaluation (default priority, non-blocking), with fork and join events
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace {

thread_local std::string g_err;

// Per-kernel-class timing with HIP events (the paper accumulates the time of
// each kernel type, Section 7, Table 4).
bool g_timing = false;
struct EventPair {
  int cls;
  hipEvent_t a, b;
};
std::vector<EventPair> g_pending;
double g_ms[MD_NCLASSES] = {0};
int64_t g_count[MD_NCLASSES] = {0};

struct Timed {
  int cls;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(int c, hipStream_t s) : cls(c), st(s) {
    if (!g_timing) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      a = b = nullptr;
      return;
    }
    (void)hipEventRecord(a, st);
  }
  ~Timed() {
    if (!a) return;
    (void)hipEventRecord(b, st);
    g_pending.push_back({cls, a, b});
  }
};

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(MD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool valid_prec(int p) { return p == MD_D || p == MD_DD || p == MD_QD || p == MD_OD; }

// A solve precision for a plan of L limbs: L itself, or fewer limbs among
// dd and qd (the mixed-precision forms).
bool valid_solve_prec(int ps, int L) { return ps == L || ((ps == MD_DD || ps == MD_QD) && ps < L); }

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Scratch of the QR kernels: flags [n] and the reflector board (x [n][L][n],
// (tau, 1 / (x_0 - beta)) [n][2][L]) of the LDS-resident kernel, or the barrier counter of the
// global-memory kernel used when the columns do not fit in LDS.
size_t qr_scratch_bytes(int L, int n) {
  return align_up((size_t)n * sizeof(int)) + align_up((size_t)n * L * n * sizeof(double)) +
         align_up((size_t)n * 2 * L * sizeof(double)) + 256;
}

// Workspace regions, in doubles, each aligned to 256 bytes.
struct Layout {
  size_t val, der, pw, unit, b, A, qr, tau, qt, bar, invd, M, N, At, r, dxT, dx, sync, vsz, tsz, scale;
  // the second factorization of md_newton_steps (QR, tau, Q^T and M of the
  // next step, computed while the current one finishes), coefficient 0 of
  // the next iterate and the derivative products of its pre-pass
  size_t qr2, tau2, qt2, M2, xn, der0;
  size_t xseq;  // count of xn's workgroups done (md_newton_steps)
  size_t mseq;  // count of M's columns done (md_newton_steps)
  size_t rs;    // rows of R scaled by their diagonal (back substitution of M)
  size_t total;
};

Layout newton_layout(const md_plan *p) {
  const size_t L = p->L, n = p->n, D = p->D;
  Layout w{};
  size_t off = 0;
  auto take = [&](size_t doubles) {
    size_t o = off;
    off += align_up(doubles * sizeof(double));
    return o;
  };
  w.val = take(L * p->m * D);
  w.der = take(L * p->nnz * D);
  w.pw = take(p->maxexp >= 3 ? L * n * D * (p->maxexp - 2) : 1);
  w.unit = take(L * p->m + 1);
  w.b = take(L * n * D);
  w.A = take(L * n * n * D);
  w.qr = take(L * n * n);
  w.tau = take(L * n);
  w.qt = take(L * n * n);
  w.bar = take(qr_scratch_bytes(L, n) / sizeof(double) + 1);
  w.invd = take(L * n);
  w.M = take(L * n * n);
  w.N = take(3 * L * n * n);  // N = M A_1, P = M A_2, Q = M A_3
  w.At = take(L * n * n * D);
  w.r = take(L * n * D);
  w.dxT = take(L * n * D);
  w.dx = take(L * n * D);
  w.sync = take(mdk::stages_sync_ints(p->D) / 2 + 1);
  w.vsz = take((size_t)p->m * D);  // chain maxima of the monomials' forward products
  w.tsz = take(n * D);  // sizes of the terms of b_{i,k} and their maxima over i, for the staggered driver
  w.scale = take(D);
  w.qr2 = take(L * n * n);
  w.tau2 = take(L * n);
  w.qt2 = take(L * n * n);
  w.M2 = take(L * n * n);
  w.xn = take(L * n);
  w.der0 = take(L * p->nnz + 1);
  w.xseq = take(1);
  w.mseq = take(1);
  w.rs = take(L * n * n);
  w.total = off;
  return w;
}

size_t solve_bytes(int L, int n, int D) {
  return align_up((size_t)L * n * sizeof(double)) + align_up((size_t)L * n * n * sizeof(double)) +
         align_up((size_t)3 * L * n * n * sizeof(double)) + align_up((size_t)L * n * n * D * sizeof(double)) +
         2 * align_up((size_t)L * n * D * sizeof(double)) + align_up((size_t)mdk::stages_sync_ints(D) * sizeof(int));
}

double *at(void *ws, size_t byte_off) { return reinterpret_cast<double *>(static_cast<char *>(ws) + byte_off); }


// The hand-over memory of the LDS QR in its scratch, for a launch that
// prepares it ahead of the QR (the A_0 assembly); none for the global QR.
mdk::QrPrep qr_prep(int L, int n, void *scratch) {
  mdk::QrPrep q;
  if (mdk::qr_lds_workgroups(L, n, true) == 0) return q;
  char *p = static_cast<char *>(scratch);
  q.flags = reinterpret_cast<int *>(p);
  p += align_up((size_t)n * sizeof(int));
  p += align_up((size_t)n * L * n * sizeof(double));
  q.tboard = reinterpret_cast<double *>(p);
  q.n = n;
  q.nt = 2 * L * n;
  return q;
}

// prepared: the LDS QR's hand-over memory was prepared by an earlier launch
// on this stream (qr_prep).
hipError_t run_qr(int L, int n, double *a, double *tau, double *qt, int32_t *status, void *scratch, hipStream_t st,
                  bool prepared = false) {
  char *p = static_cast<char *>(scratch);
  int *flags = reinterpret_cast<int *>(p);
  p += align_up((size_t)n * sizeof(int));
  double *vboard = reinterpret_cast<double *>(p);
  p += align_up((size_t)n * L * n * sizeof(double));
  double *tboard = reinterpret_cast<double *>(p);
  p += align_up((size_t)n * 2 * L * sizeof(double));
  unsigned *bar = reinterpret_cast<unsigned *>(p);
  if (mdk::qr_lds_workgroups(L, n, qt != nullptr) > 0)
    return mdk::launch_qr_lds(L, n, a, tau, qt, status, flags, vboard, tboard, st, prepared);
  return mdk::launch_qr(L, n, a, tau, qt, status, bar, st);
}

// Scratch of md_qr_noalloc: the QR's flags, reflector board and scalar slots in a static
// device array (each GPU holds its own copy, at its own address, until the
// process ends).  Host code never passes the array's name to a kernel: it
// stands for a host-side symbol there.  The device address is taken once per
// device with hipGetSymbolAddress, with that device current, and kept.
static __device__ __align__(256) unsigned char scratch[MD_QR_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(MD_EINVAL, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress of the static QR scratch");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MD_OK;
}

int series_solve_impl(int L, int n, int D, const double *qr, const double *tau, const double *A, double *rhs_dx,
                      void *ws, hipStream_t st, int32_t *status) {
  size_t off = 0;
  auto take = [&](size_t doubles) {
    double *p = at(ws, off);
    off += align_up(doubles * sizeof(double));
    return p;
  };
  const size_t nn = (size_t)n * n, nD = (size_t)n * D;
  double *invd = take((size_t)L * n), *M = take((size_t)L * nn), *N = take((size_t)3 * L * nn);
  double *At = take((size_t)L * nn * D), *rT = take((size_t)L * nD), *dxT = take((size_t)L * nD);
  int *sync = reinterpret_cast<int *>(take(mdk::stages_sync_ints(D) / 2 + 1));
  hipError_t e;
  {
    Timed t(MD_CLASS_QHB_BS, st);
    if ((e = mdk::launch_form_m(L, n, qr, tau, invd, M, status, st)) != hipSuccess) return hip_fail(e, "form M");
  }
  {
    Timed t(MD_CLASS_UPDATES, st);
    if ((e = mdk::launch_transpose(L, A, At, nn, D, nn * D, nn * D, st)) != hipSuccess) return hip_fail(e, "A^T");
    if ((e = mdk::launch_transpose(L, rhs_dx, rT, n, D, nD, nD, st)) != hipSuccess) return hip_fail(e, "b^T");
  }
  if (D > 1) {
    Timed t(MD_CLASS_GEMM, st);
    if ((e = mdk::launch_gemm(L, n, M, At + nn, nn * D, N, mdk::stages_products(L, n, D), st)) != hipSuccess)
      return hip_fail(e, "gemm");
  }
  {
    Timed t(MD_CLASS_UPDATES, st);
    if ((e = mdk::launch_stages(L, n, D, M, N, At, rT, dxT, sync, status, st)) != hipSuccess)
      return hip_fail(e, "stages");
    if ((e = mdk::launch_transpose(L, dxT, rhs_dx, D, n, nD, nD, st)) != hipSuccess) return hip_fail(e, "dx");
  }
  return MD_OK;
}

}  // namespace

namespace mdk {
// The library's error message for calls implemented in other files.
int api_fail(int code, const char *msg) { return fail(code, msg); }
int api_hip_fail(hipError_t e, const char *what) { return hip_fail(e, what); }
bool api_timing_enabled() { return g_timing; }
__global__ void copy_kernel(const double *src, double *dst, size_t count) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < count) dst[q] = src[q];
}
hipError_t launch_copy(const double *src, double *dst, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}
}  // namespace mdk

extern "C" {

const char *md_last_error(void) { return g_err.c_str(); }

int md_plan_create(int prec, int n, int d, int m, const int32_t *poly_ptr, const int32_t *mon_ptr,
                   const int32_t *var, const int32_t *exp, md_plan **out) {
  if (!out) return fail(MD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!valid_prec(prec)) return fail(MD_EINVAL, "precision must be 1, 2, 4 or 8 limbs");
  if (n < 1 || n > MD_MAX_DIM) return fail(MD_EINVAL, "n out of range");
  if (d < 0 || d + 1 > MD_MAX_COEFFS) return fail(MD_EINVAL, "degree out of range");
  if (m < 0) return fail(MD_EINVAL, "m < 0");
  if (!poly_ptr || !mon_ptr || (m > 0 && (!var || !exp) && mon_ptr[m] > 0))
    return fail(MD_EINVAL, "NULL index table");
  if (poly_ptr[0] != 0 || poly_ptr[n] != m) return fail(MD_EINVAL, "poly_ptr must run from 0 to m");
  for (int i = 0; i < n; ++i)
    if (poly_ptr[i + 1] < poly_ptr[i]) return fail(MD_EINVAL, "poly_ptr not monotone");
  if (mon_ptr[0] != 0) return fail(MD_EINVAL, "mon_ptr[0] must be 0");
  for (int j = 0; j < m; ++j)
    if (mon_ptr[j + 1] < mon_ptr[j]) return fail(MD_EINVAL, "mon_ptr not monotone");
  const int nnz = mon_ptr[m];
  int maxexp = 1, maxk = 0;
  for (int j = 0; j < m; ++j) {
    maxk = std::max(maxk, (int)(mon_ptr[j + 1] - mon_ptr[j]));
    for (int q = mon_ptr[j]; q < mon_ptr[j + 1]; ++q) {
      if (var[q] < 0 || var[q] >= n) return fail(MD_EINVAL, "variable index out of range");
      if (q > mon_ptr[j] && var[q] <= var[q - 1])
        return fail(MD_EINVAL, "variables must be strictly increasing within a monomial");
      if (exp[q] < 1 || exp[q] > MD_MAX_EXPONENT) return fail(MD_EINVAL, "exponent out of range");
      maxexp = std::max(maxexp, (int)exp[q]);
    }
  }
  md_plan *p = new md_plan();
  p->L = prec;
  p->n = n;
  p->d = d;
  p->D = d + 1;
  p->m = m;
  p->nnz = nnz;
  p->maxexp = maxexp;
  p->maxk = maxk;
  // work order: most expensive monomials first, so that workers of one
  // wavefront get similar work
  std::vector<int32_t> order(m);
  std::iota(order.begin(), order.end(), 0);
  std::vector<int> cost(m);
  for (int j = 0; j < m; ++j) {
    int k = mon_ptr[j + 1] - mon_ptr[j], extra = 0;
    for (int q = mon_ptr[j]; q < mon_ptr[j + 1]; ++q) extra += exp[q] - 1;
    cost[j] = 3 * k + extra;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  // All workgroups of the evaluation are resident at once, one per CU per
  // round of CU-many workgroups, and a CU runs the workgroups it received to
  // the end: reversing every second round pairs the most expensive groups of
  // monomials with the cheapest on each CU (the per-SIMD work otherwise
  // differs by up to 1.5x).
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                 hipSuccess &&
        cus > 0) {
      const int wpb = mdk::evaldiff_workers_per_block(d + 1);
      const int groups = (m + wpb - 1) / wpb;
      std::vector<int32_t> snake;
      snake.reserve(m);
      for (int r0 = 0; r0 < groups; r0 += cus) {
        const int r1 = std::min(groups, r0 + cus);
        const bool rev = ((r0 / cus) & 1) != 0;
        for (int q = 0; q < r1 - r0; ++q) {
          const int gidx = rev ? r1 - 1 - q : r0 + q;
          for (int t = gidx * wpb; t < std::min(m, (gidx + 1) * wpb); ++t) snake.push_back(order[t]);
        }
      }
      order.swap(snake);
    }
    (void)hipGetLastError();
  }
  // assembly lists: entries contributing to (row i, column v), in monomial order
  std::vector<int32_t> row_of(m);
  for (int i = 0; i < n; ++i)
    for (int j = poly_ptr[i]; j < poly_ptr[i + 1]; ++j) row_of[j] = i;
  const size_t nn = (size_t)n * n;
  std::vector<int32_t> asm_ptr(nn + 1, 0), asm_ent(nnz);
  for (int j = 0; j < m; ++j)
    for (int q = mon_ptr[j]; q < mon_ptr[j + 1]; ++q) asm_ptr[(size_t)row_of[j] * n + var[q] + 1]++;
  for (size_t t = 0; t < nn; ++t) asm_ptr[t + 1] += asm_ptr[t];
  {
    std::vector<int32_t> fill(asm_ptr.begin(), asm_ptr.end() - 1);
    for (int j = 0; j < m; ++j)
      for (int q = mon_ptr[j]; q < mon_ptr[j + 1]; ++q) asm_ent[fill[(size_t)row_of[j] * n + var[q]]++] = q;
  }
  auto up = [&](int32_t **dst, const int32_t *src, size_t cnt) -> hipError_t {
    hipError_t e = hipMalloc((void **)dst, std::max<size_t>(cnt, 1) * sizeof(int32_t));
    if (e != hipSuccess) return e;
    if (cnt) e = hipMemcpy(*dst, src, cnt * sizeof(int32_t), hipMemcpyHostToDevice);
    return e;
  };
  hipError_t e;
  if ((e = up(&p->d_poly_ptr, poly_ptr, n + 1)) != hipSuccess || (e = up(&p->d_mon_ptr, mon_ptr, m + 1)) != hipSuccess ||
      (e = up(&p->d_var, var, nnz)) != hipSuccess || (e = up(&p->d_exp, exp, nnz)) != hipSuccess ||
      (e = up(&p->d_order, order.data(), m)) != hipSuccess ||
      (e = up(&p->d_asm_ptr, asm_ptr.data(), nn + 1)) != hipSuccess ||
      (e = up(&p->d_asm_ent, asm_ent.data(), nnz)) != hipSuccess ||
      (e = up(&p->d_row_of, row_of.data(), m)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming)) != hipSuccess) {
    md_plan_destroy(p);
    return hip_fail(e, "plan setup");
  }
  *out = p;
  return MD_OK;
}

int md_plan_destroy(md_plan *p) {
  if (!p) return MD_OK;
  for (int32_t *q : {p->d_poly_ptr, p->d_mon_ptr, p->d_var, p->d_exp, p->d_order, p->d_asm_ptr, p->d_asm_ent,
                     p->d_row_of})
    if (q) (void)hipFree(q);
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->join) (void)hipEventDestroy(p->join);
  if (p->aux) (void)hipStreamDestroy(p->aux);
  delete p;
  return MD_OK;
}

int md_workspace_size(const md_plan *p, size_t *bytes) {
  if (!p || !bytes) return fail(MD_EINVAL, "NULL argument");
  *bytes = newton_layout(p).total;
  return MD_OK;
}

static void eval_args(const md_plan *p, const double *cff, const double *x, void *ws, int Dc, mdk::EvalArgs &a) {
  Layout w = newton_layout(p);
  a.n = p->n;
  a.D = p->D;
  a.Dc = Dc;
  a.m = p->m;
  a.nnz = p->nnz;
  a.mon_ptr = p->d_mon_ptr;
  a.var = p->d_var;
  a.exp = p->d_exp;
  a.order = p->d_order;
  a.cff = cff;
  a.x = x;
  a.pw = at(ws, w.pw);
  a.val = at(ws, w.val);
  a.der = at(ws, w.der);
}

// b and A for the first Dc coefficients (the problem truncated at order Dc);
// tsz (nullable) gets the sizes of the terms of b.  beside_qr: the launch
// runs beside the QR of a Newton step, off the critical path; the evaluation
// then takes one wavefront per monomial, which leaves the QR's wavefronts
// more issue slots on the CUs they share (measured: 0.966 against 0.981 ms
// per medium quad-double step), while alone two wavefronts per monomial are
// faster (353 against 403 us).
static int eval_diff_impl(const md_plan *p, int Dc, const double *cff, const double *cst, const double *x, double *b,
                          double *A, void *ws, hipStream_t st, double *tsz = nullptr, bool beside_qr = false,
                          mdk::TOut rt = mdk::TOut(), mdk::TOut aT = mdk::TOut(), int *clear = nullptr,
                          int clear_count = 0, double *empty = nullptr, size_t empty_count = 0,
                          mdk::CountWait wait = mdk::CountWait()) {
  Layout w = newton_layout(p);
  mdk::EvalArgs a;
  eval_args(p, cff, x, ws, Dc, a);
  a.beside_qr = beside_qr ? 1 : 0;
  if (tsz) a.vsize = at(ws, w.vsz);
  hipError_t e;
  {
    Timed t(MD_CLASS_CONVOLUTIONS, st);
    e = mdk::launch_evaldiff(p->L, a, p->maxexp, at(ws, w.pw), st);
  }
  if (e != hipSuccess) return hip_fail(e, "eval/diff launch");
  {
    Timed t(MD_CLASS_ASSEMBLY, st);
    e = mdk::launch_assemble(p->L, p->n, p->D, Dc, p->m, p->nnz, p->d_poly_ptr, p->d_asm_ptr, p->d_asm_ent, cst,
                             a.val, a.der, b, A, st, tsz, a.vsize, rt, aT, clear, clear_count, empty, empty_count,
                             wait);
  }
  if (e != hipSuccess) return hip_fail(e, "assembly launch");
  return MD_OK;
}

int md_eval_diff(const md_plan *p, const double *cff, const double *cst, const double *x, double *b, double *A,
                 void *ws, size_t ws_bytes, hipStream_t st) {
  if (!p || !cst || !x || !b || !A || (p->m > 0 && !cff)) return fail(MD_EINVAL, "NULL argument");
  if (!ws || ws_bytes < newton_layout(p).total) return fail(MD_ENOSPACE, "workspace too small");
  return eval_diff_impl(p, p->D, cff, cst, x, b, A, ws, st);
}

int md_qr_workspace_size(int prec, int n, size_t *bytes) {
  if (!bytes || !valid_prec(prec) || n < 1 || n > MD_MAX_DIM) return fail(MD_EINVAL, "bad argument");
  *bytes = qr_scratch_bytes(prec, n);
  return MD_OK;
}

int md_qr(int prec, int n, double *a0, double *tau, void *ws, size_t ws_bytes, hipStream_t st, int32_t *dev_status) {
  if (!valid_prec(prec) || n < 1 || n > MD_MAX_DIM) return fail(MD_EINVAL, "bad precision or dimension");
  if (!a0 || !tau) return fail(MD_EINVAL, "NULL argument");
  if (!ws || ws_bytes < qr_scratch_bytes(prec, n)) return fail(MD_ENOSPACE, "workspace too small");
  hipError_t e = run_qr(prec, n, a0, tau, nullptr, dev_status, ws, st);
  return e == hipSuccess ? MD_OK : hip_fail(e, "qr launch");
}

int md_qr_noalloc(int prec, int n, double *a0, double *tau, hipStream_t st, int32_t *dev_status) {
  if (!valid_prec(prec) || n < 1 || n > MD_MAX_DIM) return fail(MD_EINVAL, "bad precision or dimension");
  if (!a0 || !tau) return fail(MD_EINVAL, "NULL argument");
  const size_t need = qr_scratch_bytes(prec, n);
  if (need > (size_t)MD_QR_NOALLOC_MAX_BYTES)
    return fail(MD_ENOSPACE, "md_qr_noalloc: the QR needs " + std::to_string(need) +
                                 " bytes of scratch, more than the static " +
                                 std::to_string((size_t)MD_QR_NOALLOC_MAX_BYTES) + " (use md_qr with a workspace)");
  void *ptr = nullptr;
  const int rc = noalloc_scratch(&ptr);
  if (rc != MD_OK) return rc;
  hipError_t e = run_qr(prec, n, a0, tau, nullptr, dev_status, ptr, st);
  return e == hipSuccess ? MD_OK : hip_fail(e, "qr launch");
}

int md_solve_workspace_size(int prec, int n, int d, size_t *bytes) {
  if (!bytes || !valid_prec(prec) || n < 1 || n > MD_MAX_DIM || d < 0 || d + 1 > MD_MAX_COEFFS)
    return fail(MD_EINVAL, "bad argument");
  *bytes = solve_bytes(prec, n, d + 1);
  return MD_OK;
}

int md_series_solve(int prec, int n, int d, const double *qr, const double *tau, const double *A, double *rhs_dx,
                    void *ws, size_t ws_bytes, hipStream_t st, int32_t *dev_status) {
  if (!valid_prec(prec) || n < 1 || n > MD_MAX_DIM || d < 0 || d + 1 > MD_MAX_COEFFS)
    return fail(MD_EINVAL, "bad precision, dimension or degree");
  if (!qr || !tau || !rhs_dx || (d > 0 && !A)) return fail(MD_EINVAL, "NULL argument");
  if (!ws || ws_bytes < solve_bytes(prec, n, d + 1)) return fail(MD_ENOSPACE, "workspace too small");
  return series_solve_impl(prec, n, d + 1, qr, tau, A, rhs_dx, ws, st, dev_status);
}

// One Newton step with the residual b = -p(x) at the plan's precision L and
// the Jacobian series, the QR of A_0 and the staged solve at Ls <= L limbs.
// Limb-major storage makes the Ls-limb truncation of x, cff and b their
// leading Ls limb planes, so the low-precision kernels read the same
// buffers.  Ls == L is the plain step.
//
// The staggered method (Section 4) runs the step on a window: the problem
// truncated at order hi (coefficients 0..hi-1 evaluated, those from hi on
// left as they are) with the stages lo..hi-1 solved, dx_k = 0 below lo.
// The window's block system is the block Toeplitz solve of hi - lo stages on
// b_lo..b_{hi-1} with A_0..A_{hi-lo-1}, so strided transposes pack it into
// the compact coefficient-major arrays of the stage kernels.  keep_m skips
// the pre-pass, the QR and M and uses the M = A_0^{-1} that the last step
// without keep_m left in the workspace (the factorization of the first
// stage, Section 5.3: a chord step).  With scale (nullable, D doubles) the
// assembly records the size of the terms of every b_{i,k} and scale[k] gets
// max_i |b_{i,k}| / (that size), the residual relative to its own terms.
static int newton_step_impl(const md_plan *p, int Ls, int lo, int hi, bool keep_m, const double *cff,
                            const double *cst, double *x, int32_t *dev_status, double *dev_norms, double *scale,
                            void *ws, hipStream_t st) {
  Layout w = newton_layout(p);
  const int L = p->L, n = p->n, D = p->D, W = hi - lo;
  const bool mixed = Ls != L;
  hipError_t e;
  // the coefficient-0 pre-pass, when it runs, resets the status word itself
  const bool pre0 = !keep_m && p->m > 0 && p->maxk <= mdk::evaldiff0_max_support(Ls);
  if (!pre0 && (e = mdk::launch_status_init(dev_status, st)) != hipSuccess) return hip_fail(e, "status");
  double *b = at(ws, w.b), *A = at(ws, w.A), *qr = at(ws, w.qr), *tau = at(ws, w.tau), *qt = at(ws, w.qt);
  double *invd = at(ws, w.invd), *M = at(ws, w.M), *N = at(ws, w.N), *r = at(ws, w.r), *dx = at(ws, w.dx);
  double *tsz = scale ? at(ws, w.tsz) : nullptr;
  mdk::EvalArgs a;
  if (!keep_m) {
    // 1. pre-pass: coefficient 0 of every derivative product gives A_0 (the
    //    same products as the full evaluation, rounded in another order: the
    //    solve uses this A_0 throughout, for M and for the stages)
    {
      Timed t(MD_CLASS_QR, st);
      eval_args(p, cff, x, ws, 1, a);
      if (pre0) a.reset_status = dev_status;
      e = pre0 ? mdk::launch_evaldiff0(Ls, a, st) : mdk::launch_evaldiff(Ls, a, p->maxexp, at(ws, w.pw), st);
      a.reset_status = nullptr;
      if (e != hipSuccess) return hip_fail(e, "A_0 pre-pass");
      // (its launch also prepares the QR's hand-over memory)
      if ((e = mdk::launch_assemble_A0(Ls, n, D, p->nnz, p->d_asm_ptr, p->d_asm_ent, a.der, qr, st,
                                       qr_prep(Ls, n, at(ws, w.bar)))) != hipSuccess)
        return hip_fail(e, "A_0 assembly");
    }
    // 2. fork: QR of A_0 with Q^T, then M = R^{-1} Q^T, on the second stream
    if ((e = hipEventRecord(p->fork, st)) != hipSuccess) return hip_fail(e, "fork");
    if ((e = hipStreamWaitEvent(p->aux, p->fork, 0)) != hipSuccess) return hip_fail(e, "fork wait");
    {
      Timed t(MD_CLASS_QR, p->aux);
      if ((e = run_qr(Ls, n, qr, tau, qt, dev_status, at(ws, w.bar), p->aux, true)) != hipSuccess)
        return hip_fail(e, "qr");
    }
    {
      Timed t(MD_CLASS_QHB_BS, p->aux);
      if ((e = mdk::launch_m_from_qt(Ls, n, qr, qt, invd, M, dev_status, p->aux, at(ws, w.rs))) != hipSuccess)
        return hip_fail(e, "M");
    }
    if ((e = hipEventRecord(p->join, p->aux)) != hipSuccess) return hip_fail(e, "join");
  }
  // 3. the evaluation and differentiation of the first hi coefficients on the
  //    caller's stream; mixed: the values at L limbs for b, the derivatives
  //    at Ls limbs for A.  The assembly also writes the coefficient-major
  //    copies A_0..A_{W-1} [Ls][W][n][n] and b_lo..b_{hi-1} [Ls][W][n] that
  //    the staged solve reads, clears the solve's counters and empties its dx
  //    slots.
  const size_t nn = (size_t)n * n;
  double *At = at(ws, w.At), *dxT = at(ws, w.dxT);
  int *sync = reinterpret_cast<int *>(at(ws, w.sync));
  const mdk::TOut rt{r, lo, W, Ls}, atT{At, 0, W, Ls};
  const int nsync = mdk::stages_sync_ints(W);
  const size_t ndx = (size_t)Ls * n * W;
  if (!mixed) {
    int rc = eval_diff_impl(p, hi, cff, cst, x, b, A, ws, st, tsz, !keep_m, rt, atT, sync, nsync, dxT, ndx);
    if (rc != MD_OK) return rc;
  } else {
    eval_args(p, cff, x, ws, hi, a);
    a.beside_qr = keep_m ? 0 : 1;
    a.values_only = 1;
    if (tsz) a.vsize = at(ws, w.vsz);
    {
      Timed t(MD_CLASS_CONVOLUTIONS, st);
      if ((e = mdk::launch_evaldiff(L, a, p->maxexp, at(ws, w.pw), st)) != hipSuccess)
        return hip_fail(e, "residual evaluation");
    }
    {
      Timed t(MD_CLASS_ASSEMBLY, st);
      if ((e = mdk::launch_assemble_b(L, n, D, hi, p->m, p->d_poly_ptr, cst, a.val, b, st, tsz, a.vsize, rt, sync,
                                      nsync, dxT, ndx)) != hipSuccess)
        return hip_fail(e, "residual assembly");
    }
    a.values_only = 0;
    a.vsize = nullptr;
    {
      Timed t(MD_CLASS_CONVOLUTIONS, st);
      if ((e = mdk::launch_evaldiff(Ls, a, p->maxexp, at(ws, w.pw), st)) != hipSuccess)
        return hip_fail(e, "Jacobian evaluation");
    }
    {
      Timed t(MD_CLASS_ASSEMBLY, st);
      if ((e = mdk::launch_assemble_A(Ls, n, D, hi, p->nnz, p->d_asm_ptr, p->d_asm_ent, a.der, A, st, atT)) !=
          hipSuccess)
        return hip_fail(e, "Jacobian assembly");
    }
  }
  // 4. join, N = M A_1 (and P = M A_2, Q = M A_3), the staged solve of the window
  if (!keep_m && (e = hipStreamWaitEvent(st, p->join, 0)) != hipSuccess) return hip_fail(e, "join wait");
  if (W > 1) {
    Timed t(MD_CLASS_GEMM, st);
    if ((e = mdk::launch_gemm(Ls, n, M, At + nn, nn * W, N, mdk::stages_products(Ls, n, W), st)) != hipSuccess)
      return hip_fail(e, "gemm");
  }
  {
    Timed t(MD_CLASS_UPDATES, st);
    if ((e = mdk::launch_stages(Ls, n, W, M, N, At, r, dxT, sync, dev_status, st, true)) != hipSuccess)
      return hip_fail(e, "stages");
  }
  {  // dx to series-major, x += dx, norms: one launch
    Timed t(MD_CLASS_X_UPDATE, st);
    e = mdk::launch_finish(L, Ls, n, D, lo, hi, dxT, dx, x, b, dev_norms, dev_status, st, tsz, scale);
    if (e != hipSuccess) return hip_fail(e, "update");
  }
  return MD_OK;
}

int md_newton_step(const md_plan *p, const double *cff, const double *cst, double *x, int32_t *dev_status,
                   double *dev_norms, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!p || !cst || !x || (p->m > 0 && !cff)) return fail(MD_EINVAL, "NULL argument");
  if (!ws || ws_bytes < newton_layout(p).total) return fail(MD_ENOSPACE, "workspace too small");
  return newton_step_impl(p, p->L, 0, p->D, false, cff, cst, x, dev_status, dev_norms, nullptr, ws, st);
}

// Whether md_newton_steps can overlap the factorization of the next step
// with the current one: plain steps whose staged solve is the persistent
// kernel (its first stage is what the next-x_0 blocks reproduce) and whose A_0
// comes from the coefficient-0 pre-pass.
static bool steps_pipelined(const md_plan *p) {
  return p->m > 0 && p->D > 1 && mdk::stages_persistent(p->L, p->n, p->D) &&
         p->maxk <= mdk::evaldiff0_max_support(p->L);
}

// count plain Newton steps.  A_0 of step s+1 depends on coefficient 0 of its
// iterate only, x_0 + dx_0, and dx_0 = M r_0 is known once step s has M and
// b: the launch of the products N, P, Q forms it too (bit for bit as the
// staged solve and the update will) right after the join, and the pre-pass,
// QR and M of step s+1 run on
// the second stream while step s finishes its staged solve and step s+1
// evaluates.  Factorizations alternate between two sets of buffers, the last
// step using the first set (the one md_newton_step and chord steps use).
static int newton_steps_impl(const md_plan *p, int count, const double *cff, const double *cst, double *x,
                             int32_t *dev_status, double *dev_norms, void *ws, hipStream_t st) {
  if (!steps_pipelined(p)) {
    for (int s = 0; s < count; ++s) {
      const int rc = newton_step_impl(p, p->L, 0, p->D, false, cff, cst, x, dev_status, dev_norms, nullptr, ws, st);
      if (rc != MD_OK) return rc;
    }
    return MD_OK;
  }
  Layout w = newton_layout(p);
  const int L = p->L, n = p->n, D = p->D;
  const size_t nn = (size_t)n * n;
  hipError_t e;
  int *xseq = reinterpret_cast<int *>(at(ws, w.xseq)), *mseq = reinterpret_cast<int *>(at(ws, w.mseq));
  // M counted on the device only where the small back substitution forms it
  const bool mcount = n <= 64;
  if ((e = mdk::launch_status_init(dev_status, st, xseq, mseq)) != hipSuccess) return hip_fail(e, "status");
  double *b = at(ws, w.b), *A = at(ws, w.A), *r = at(ws, w.r), *dx = at(ws, w.dx), *N = at(ws, w.N);
  double *At = at(ws, w.At), *dxT = at(ws, w.dxT), *invd = at(ws, w.invd), *xn = at(ws, w.xn);
  double *qrs[2] = {at(ws, w.qr), at(ws, w.qr2)}, *taus[2] = {at(ws, w.tau), at(ws, w.tau2)};
  double *qts[2] = {at(ws, w.qt), at(ws, w.qt2)}, *Ms[2] = {at(ws, w.M), at(ws, w.M2)};
  int *sync = reinterpret_cast<int *>(at(ws, w.sync));
  // factorization of the iterate whose coefficient 0 is in xn ([L][n]) into
  // buffer set k, on the second stream after the fork event; its pre-pass
  // has derivative products of its own (der0), since the evaluation of the
  // current step runs beside it.  The first iterate's xn is a copy made on
  // the caller's stream before a fork event; the next ones' are formed by
  // the launch of the products N, P, Q, whose xn workgroups count themselves
  // done in xseq (xseq_target: the count to wait for, 0: the fork event), so
  // that no event sits between that launch and the staged solve.  The join
  // event is recorded after the last factorization only (and after every
  // one where the caller's stream waits for it instead of M's count): an
  // event record on the second stream delays its next launch.
  auto factor = [&](int k, int xseq_target, bool last) -> int {
    if (xseq_target == 0) {
      if ((e = hipEventRecord(p->fork, st)) != hipSuccess) return hip_fail(e, "fork");
      if ((e = hipStreamWaitEvent(p->aux, p->fork, 0)) != hipSuccess) return hip_fail(e, "fork wait");
    }
    {
      mdk::EvalArgs a;
      eval_args(p, cff, xn, ws, 1, a);
      a.D = 1;  // one coefficient per series: xn and der0 [L][nnz]
      a.der = at(ws, w.der0);
      if (xseq_target > 0) {
        a.wait_ctr = xseq;
        a.wait_target = xseq_target;
        a.wait_status = dev_status;
      }
      // the pre-pass is left out of the class timing: it may wait for xn
      if ((e = mdk::launch_evaldiff0(L, a, p->aux)) != hipSuccess) return hip_fail(e, "A_0 pre-pass");
      Timed t(MD_CLASS_QR, p->aux);
      // (the A_0 assembly also prepares the QR's hand-over memory)
      if ((e = mdk::launch_assemble_A0(L, n, 1, p->nnz, p->d_asm_ptr, p->d_asm_ent, a.der, qrs[k], p->aux,
                                       qr_prep(L, n, at(ws, w.bar)))) != hipSuccess)
        return hip_fail(e, "A_0 assembly");
      if ((e = run_qr(L, n, qrs[k], taus[k], qts[k], dev_status, at(ws, w.bar), p->aux, true)) != hipSuccess)
        return hip_fail(e, "qr");
    }
    {
      Timed t(MD_CLASS_QHB_BS, p->aux);
      if ((e = mdk::launch_m_from_qt(L, n, qrs[k], qts[k], invd, Ms[k], dev_status, p->aux, at(ws, w.rs),
                                     mcount ? mseq : nullptr)) != hipSuccess)
        return hip_fail(e, "M");
    }
    if ((last || !mcount) && (e = hipEventRecord(p->join, p->aux)) != hipSuccess) return hip_fail(e, "join");
    return MD_OK;
  };
  // coefficient 0 of the first iterate into xn
  if ((e = mdk::launch_transpose_ld(L, x, D, xn, n, n, 1, (size_t)n * D, n, st)) != hipSuccess)
    return hip_fail(e, "x_0");
  int rc = factor((count - 1) % 2, 0, count == 1);
  if (rc != MD_OK) return rc;
  for (int s = 0; s < count; ++s) {
    const int k = (count - 1 - s) % 2;
    // the evaluation is on the critical path here (the factorization of the
    // next step has slack): the two-wavefront kernel (0.69 against 0.75 ms
    // per step); the assembly also writes the coefficient-major A and b,
    // clears the staged solve's counters and empties its dx slots, and ends
    // only once M of this step is formed: a wait for its columns' count on
    // the device (the factorizations so far: s + 1), else the join event
    rc = eval_diff_impl(p, D, cff, cst, x, b, A, ws, st, nullptr, false, mdk::TOut{r, 0, D, L},
                        mdk::TOut{At, 0, D, L}, sync, mdk::stages_sync_ints(D), dxT, (size_t)L * n * D,
                        mcount ? mdk::CountWait{mseq, n * (s + 1), dev_status} : mdk::CountWait());
    if (rc != MD_OK) return rc;
    if (!mcount && (e = hipStreamWaitEvent(st, p->join, 0)) != hipSuccess) return hip_fail(e, "join wait");
    {
      // N, P, Q and, before the last step, coefficient 0 of the next iterate
      // (from M and r_0; x is updated later in this stream)
      Timed t(MD_CLASS_GEMM, st);
      e = (s + 1 < count)
              ? mdk::launch_gemm_next_x0(L, n, D, Ms[k], At + nn, nn * D, N, mdk::stages_products(L, n, D), r, x, xn,
                                         xseq, st)
              : mdk::launch_gemm(L, n, Ms[k], At + nn, nn * D, N, mdk::stages_products(L, n, D), st);
      if (e != hipSuccess) return hip_fail(e, "gemm");
    }
    // the next factorization on the second stream, beside the rest of this
    // step and the next evaluation
    if (s + 1 < count && (rc = factor(1 - k, ((n + 3) / 4) * (s + 1), s + 2 == count)) != MD_OK) return rc;
    {
      Timed t(MD_CLASS_UPDATES, st);
      if ((e = mdk::launch_stages(L, n, D, Ms[k], N, At, r, dxT, sync, dev_status, st, true)) != hipSuccess)
        return hip_fail(e, "stages");
    }
    {
      Timed t(MD_CLASS_X_UPDATE, st);
      if ((e = mdk::launch_finish(L, L, n, D, 0, D, dxT, dx, x, b, dev_norms, dev_status, st)) != hipSuccess)
        return hip_fail(e, "update");
    }
  }
  // the caller's stream after every launch of the second stream
  if (mcount && (e = hipStreamWaitEvent(st, p->join, 0)) != hipSuccess) return hip_fail(e, "join wait");
  return MD_OK;
}

int md_newton_steps(const md_plan *p, int count, const double *cff, const double *cst, double *x, int32_t *dev_status,
                    double *dev_norms, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!p || !cst || !x || (p->m > 0 && !cff)) return fail(MD_EINVAL, "NULL argument");
  if (count < 0) return fail(MD_EINVAL, "negative step count");
  if (!ws || ws_bytes < newton_layout(p).total) return fail(MD_ENOSPACE, "workspace too small");
  if (count == 0) return MD_OK;
  return newton_steps_impl(p, count, cff, cst, x, dev_status, dev_norms, ws, st);
}

int md_newton_step_mixed(const md_plan *p, int prec_solve, const double *cff, const double *cst, double *x,
                         int32_t *dev_status, double *dev_norms, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!p || !cst || !x || (p->m > 0 && !cff)) return fail(MD_EINVAL, "NULL argument");
  if (!valid_solve_prec(prec_solve, p->L))
    return fail(MD_EINVAL, "solve precision must be the plan's, or dd or qd below it");
  if (!ws || ws_bytes < newton_layout(p).total) return fail(MD_ENOSPACE, "workspace too small");
  return newton_step_impl(p, prec_solve, 0, p->D, false, cff, cst, x, dev_status, dev_norms, nullptr, ws, st);
}

int md_newton_step_window(const md_plan *p, int prec_solve, int lo, int hi, int keep_factorization,
                          const double *cff, const double *cst, double *x, int32_t *dev_status, double *dev_norms,
                          void *ws, size_t ws_bytes, hipStream_t st) {
  if (!p || !cst || !x || (p->m > 0 && !cff)) return fail(MD_EINVAL, "NULL argument");
  if (!valid_solve_prec(prec_solve, p->L))
    return fail(MD_EINVAL, "solve precision must be the plan's, or dd or qd below it");
  if (lo < 0 || hi > p->D || lo >= hi) return fail(MD_EINVAL, "window must satisfy 0 <= lo < hi <= D");
  if (!ws || ws_bytes < newton_layout(p).total) return fail(MD_ENOSPACE, "workspace too small");
  return newton_step_impl(p, prec_solve, lo, hi, keep_factorization != 0, cff, cst, x, dev_status, dev_norms,
                          nullptr, ws, st);
}

int md_stagger_next_order(int d, int D) { return std::min(D, d + 1 + d / 2); }

int md_newton_staggered(const md_plan *p, int prec_solve, int refactor_every_step, int max_steps, double tol,
                        const double *cff, const double *cst, double *x, int32_t *windows, double *rel,
                        md_stagger_report *report, int32_t *dev_status, double *dev_norms, void *ws,
                        size_t ws_bytes, hipStream_t st) {
  if (!p || !cst || !x || !dev_status || !dev_norms || !report || (p->m > 0 && !cff))
    return fail(MD_EINVAL, "NULL argument");
  if (!valid_solve_prec(prec_solve, p->L))
    return fail(MD_EINVAL, "solve precision must be the plan's, or dd or qd below it");
  if (max_steps < 1 || !(tol >= 0.0)) return fail(MD_EINVAL, "max_steps must be positive and tol non-negative");
  if (!ws || ws_bytes < newton_layout(p).total) return fail(MD_ENOSPACE, "workspace too small");
  const Layout w = newton_layout(p);
  const int D = p->D;
  double *scale = at(ws, w.scale);
  // norms, relative residuals and status come back through pinned, mapped host
  // memory written by one small kernel: one wait per step, no copies
  struct Pinned {
    double *h = nullptr;
    ~Pinned() {
      if (h) (void)hipHostFree(h);
    }
  } pin;
  hipError_t e;
  double *hdev = nullptr;
  if ((e = hipHostMalloc((void **)&pin.h, (3 * (size_t)D + 1) * sizeof(double), hipHostMallocCoherent)) !=
          hipSuccess ||
      (e = hipHostGetDevicePointer((void **)&hdev, pin.h, 0)) != hipSuccess)
    return hip_fail(e, "pinned report buffer");
  const double *h = pin.h;
  // relative residual of each coefficient at the previous step (infinity:
  // not yet evaluated), to recognise a residual that no longer decreases
  std::vector<double> prev((size_t)D, INFINITY);
  *report = md_stagger_report{0, 0, 0, 1, 0};
  int lo = 0, hi = 1;
  for (int step = 0; step < max_steps; ++step) {
    const bool keep = !refactor_every_step && step > 0;
    int rc = newton_step_impl(p, prec_solve, lo, hi, keep, cff, cst, x, dev_status, dev_norms, scale, ws, st);
    if (rc != MD_OK) return rc;
    report->steps = step + 1;
    report->lo = lo;
    report->hi = hi;
    if (!keep) report->factorizations++;
    if (windows) {
      windows[2 * step] = lo;
      windows[2 * step + 1] = hi;
    }
    if ((e = mdk::launch_report(D, dev_norms, scale, dev_status, hdev, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "reading the norms");
    const int32_t status = (int32_t)h[3 * (size_t)D];
    if (status != MD_OK) return fail(status, "a step of the staggered method failed (status " +
                                                 std::to_string(status) + ")");
    if (rel)
      for (int q = 0; q < D; ++q) rel[q] = h[2 * (size_t)D + q];
    // leading coefficients that are done: residual within tol of its terms,
    // or a residual that did not halve since the last step (a Newton or chord
    // step reduces it far more: it is at the level of the rounding errors).
    // A chord step contracts an error e to about sigma e, sigma the distance
    // of the kept factorization; with sigma above 1/2 a residual far above
    // the rounding level would not halve either, so a stalled residual
    // counts only once it is below 2^(-40 L), under the square root of the
    // unit roundoff but far above the rounding level of these residuals
    // (2^(-53 L) times the chain lengths).  Coefficients below lo are done
    // and stay frozen, so lo never decreases.
    const double stall_ceiling = std::ldexp(1.0, -40 * p->L);
    int k = lo;
    while (k < hi) {
      const double rk = h[2 * (size_t)D + k];
      if (!(rk <= tol || (rk > 0.5 * prev[k] && rk <= stall_ceiling))) break;
      ++k;
    }
    for (int q = 0; q < hi; ++q) prev[q] = h[2 * (size_t)D + q];
    if (hi == D && k == D) {
      report->converged = 1;
      break;
    }
    lo = k;
    hi = md_stagger_next_order(hi, D);
  }
  return MD_OK;
}

int md_linear_residual(int prec, int n, int d, const double *A, const double *b, const double *dx, int nrows,
                       const int32_t *rows, double *r, double *norm1, int32_t *dev_status, hipStream_t st) {
  if (!valid_prec(prec) || n < 1 || n > MD_MAX_DIM || d < 0 || d + 1 > MD_MAX_COEFFS)
    return fail(MD_EINVAL, "bad precision, dimension or degree");
  if (!A || !b || !dx || !r) return fail(MD_EINVAL, "NULL argument");
  if (nrows < 1 || (!rows && nrows != n)) return fail(MD_EINVAL, "nrows must be positive (n when rows is NULL)");
  hipError_t e = mdk::launch_residual(prec, n, d + 1, nrows, rows, A, b, dx, r, norm1, dev_status, st);
  return e == hipSuccess ? MD_OK : hip_fail(e, "residual launch");
}

int md_step_arrays(const md_plan *p, void *ws, size_t ws_bytes, double **b, double **A, double **dx) {
  if (!p || !ws || !b || !A || !dx) return fail(MD_EINVAL, "NULL argument");
  const Layout w = newton_layout(p);
  if (ws_bytes < w.total) return fail(MD_ENOSPACE, "workspace too small");
  *b = at(ws, w.b);
  *A = at(ws, w.A);
  *dx = at(ws, w.dx);
  return MD_OK;
}

// Workspace of the complex step: complex monomial values and derivative
// series, b and A, the real form of the block system (2n) with its QR and the
// real staged-solve workspace, dx, and the norms of the imaginary parts.
struct CLayout {
  size_t val, der, b, A, At, bt, a0, tau, qrs, solve, dx, nt, total;
};

static CLayout complex_layout(const md_plan *p) {
  const size_t L = p->L, n = p->n, D = p->D, N = 2 * n;
  CLayout w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t d8 = sizeof(double);
  w.val = take(2 * L * p->m * D * d8 + d8);
  w.der = take(2 * L * p->nnz * D * d8 + d8);
  w.b = take(2 * L * n * D * d8);
  w.A = take(2 * L * n * n * D * d8);
  w.At = take(L * N * N * D * d8);
  w.bt = take(L * N * D * d8);
  w.a0 = take(L * N * N * d8);
  w.tau = take(L * N * d8);
  w.qrs = take(qr_scratch_bytes((int)L, (int)N));
  w.solve = take(solve_bytes((int)L, (int)N, (int)D));
  w.dx = take(2 * L * n * D * d8);
  w.nt = take(2 * D * d8);
  w.total = off;
  return w;
}

static int complex_eval_impl(const md_plan *p, const double *cff, const double *cst, const double *x, double *b,
                             double *A, void *ws, hipStream_t st) {
  const CLayout w = complex_layout(p);
  const size_t L = p->L, n = p->n, D = p->D;
  mdk::EvalArgs a;
  a.n = p->n;
  a.D = p->D;
  a.Dc = p->D;
  a.m = p->m;
  a.nnz = p->nnz;
  a.mon_ptr = p->d_mon_ptr;
  a.var = p->d_var;
  a.exp = p->d_exp;
  a.order = p->d_order;
  a.cff = cff;
  a.x = x;
  a.pw = x;  // not read: exponents are at most 2
  a.val = at(ws, w.val);
  a.der = at(ws, w.der);
  hipError_t e;
  {
    Timed t(MD_CLASS_CONVOLUTIONS, st);
    if ((e = mdk::launch_evaldiff_complex(p->L, a, st)) != hipSuccess) return hip_fail(e, "complex evaluation");
  }
  {
    Timed t(MD_CLASS_ASSEMBLY, st);
    const size_t nD = n * D, nnD = n * n * D, mD = (size_t)p->m * D, zD = (size_t)p->nnz * D;
    for (int part = 0; part < 2; ++part)
      if ((e = mdk::launch_assemble(p->L, p->n, p->D, p->D, p->m, p->nnz, p->d_poly_ptr, p->d_asm_ptr, p->d_asm_ent,
                                    cst + part * L * nD, a.val + part * L * mD, a.der + part * L * zD,
                                    b + part * L * nD, A + part * L * nnD, st)) != hipSuccess)
        return hip_fail(e, "complex assembly");
  }
  return MD_OK;
}

int md_complex_workspace_size(const md_plan *p, size_t *bytes) {
  if (!p || !bytes) return fail(MD_EINVAL, "NULL argument");
  *bytes = complex_layout(p).total;
  return MD_OK;
}

int md_eval_diff_complex(const md_plan *p, const double *cff, const double *cst, const double *x, double *b,
                         double *A, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!p || !cst || !x || !b || !A || (p->m > 0 && !cff)) return fail(MD_EINVAL, "NULL argument");
  if (p->maxexp > 2) return fail(MD_EINVAL, "complex data: exponents must be 1 or 2");
  if (p->L == MD_D) return fail(MD_EINVAL, "complex data: double double, quad double or octo double");
  if (!ws || ws_bytes < complex_layout(p).total) return fail(MD_ENOSPACE, "workspace too small");
  return complex_eval_impl(p, cff, cst, x, b, A, ws, st);
}

int md_newton_step_complex(const md_plan *p, const double *cff, const double *cst, double *x, int32_t *dev_status,
                           double *dev_norms, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!p || !cst || !x || (p->m > 0 && !cff)) return fail(MD_EINVAL, "NULL argument");
  if (p->maxexp > 2) return fail(MD_EINVAL, "complex data: exponents must be 1 or 2");
  if (p->L == MD_D) return fail(MD_EINVAL, "complex data: double double, quad double or octo double");
  if (2 * p->n > MD_MAX_DIM) return fail(MD_EINVAL, "complex data: 2n must be at most MD_MAX_DIM");
  const CLayout w = complex_layout(p);
  if (!ws || ws_bytes < w.total) return fail(MD_ENOSPACE, "workspace too small");
  const int L = p->L, n = p->n, D = p->D, N = 2 * n;
  const size_t nD = (size_t)n * D;
  hipError_t e;
  if ((e = mdk::launch_status_init(dev_status, st)) != hipSuccess) return hip_fail(e, "status");
  double *b = at(ws, w.b), *A = at(ws, w.A), *At = at(ws, w.At), *bt = at(ws, w.bt), *a0 = at(ws, w.a0);
  double *tau = at(ws, w.tau), *dx = at(ws, w.dx);
  int rc = complex_eval_impl(p, cff, cst, x, b, A, ws, st);
  if (rc != MD_OK) return rc;
  {
    Timed t(MD_CLASS_UPDATES, st);
    if ((e = mdk::launch_complex_embed(L, n, D, A, b, At, bt, st)) != hipSuccess) return hip_fail(e, "real form");
    if ((e = mdk::launch_extract(L, N, D, 0, At, a0, st)) != hipSuccess) return hip_fail(e, "A_0");
  }
  {
    Timed t(MD_CLASS_QR, st);
    if ((e = run_qr(L, N, a0, tau, nullptr, dev_status, at(ws, w.qrs), st)) != hipSuccess) return hip_fail(e, "qr");
  }
  if ((rc = series_solve_impl(L, N, D, a0, tau, At, bt, at(ws, w.solve), st, dev_status)) != MD_OK) return rc;
  {
    Timed t(MD_CLASS_X_UPDATE, st);
    if ((e = mdk::launch_complex_unpack(L, n, D, bt, dx, st)) != hipSuccess) return hip_fail(e, "dx");
    double *nt = dev_norms ? at(ws, w.nt) : nullptr;
    if ((e = mdk::launch_update(L, n, D, 0, D, b, dx, x, dev_norms, dev_status, st)) != hipSuccess ||
        (e = mdk::launch_update(L, n, D, 0, D, b + (size_t)L * nD, dx + (size_t)L * nD, x + (size_t)L * nD, nt,
                                dev_status, st)) != hipSuccess)
      return hip_fail(e, "update");
    if (dev_norms && (e = mdk::launch_max(2 * D, nt, dev_norms, st)) != hipSuccess) return hip_fail(e, "norms");
  }
  return MD_OK;
}

int md_adjoint_workspace_size(int prec, int n, int d, size_t *bytes) {
  if (!bytes || !valid_prec(prec) || n < 1 || n > MD_MAX_DIM || d < 0 || d + 1 > MD_MAX_COEFFS)
    return fail(MD_EINVAL, "bad argument");
  const size_t L = prec, nn = (size_t)n * n, nD = (size_t)n * (d + 1);
  *bytes = align_up(L * n * 8) + 2 * align_up(L * nn * 8) + align_up(3 * L * nn * 8) +
           2 * align_up(L * nn * (d + 1) * 8) + 2 * align_up(L * nD * 8) +
           align_up((size_t)mdk::stages_sync_ints(d + 1) * sizeof(int));
  return MD_OK;
}

int md_adjoint_solve(int prec, int n, int d, const double *qr, const double *tau, const double *A, double *g_lambda,
                     void *ws, size_t ws_bytes, hipStream_t st, int32_t *dev_status) {
  size_t need = 0;
  if (md_adjoint_workspace_size(prec, n, d, &need) != MD_OK) return MD_EINVAL;
  if (!qr || !tau || !g_lambda || (d > 0 && !A)) return fail(MD_EINVAL, "NULL argument");
  if (!ws || ws_bytes < need) return fail(MD_ENOSPACE, "workspace too small");
  const int L = prec, D = d + 1;
  const size_t nn = (size_t)n * n, nD = (size_t)n * D;
  size_t off = 0;
  auto take = [&](size_t doubles) {
    double *p = at(ws, off);
    off += align_up(doubles * sizeof(double));
    return p;
  };
  double *invd = take((size_t)L * n), *M = take((size_t)L * nn), *Mt = take((size_t)L * nn),
         *Nt = take((size_t)3 * L * nn);
  double *At = take((size_t)L * nn * D), *AtT = take((size_t)L * nn * D), *rho = take((size_t)L * nD),
         *lamT = take((size_t)L * nD);
  int *sync = reinterpret_cast<int *>(take(mdk::stages_sync_ints(D) / 2 + 1));
  hipError_t e;
  if ((e = mdk::launch_form_m(L, n, qr, tau, invd, M, dev_status, st)) != hipSuccess) return hip_fail(e, "form M");
  if ((e = mdk::launch_transpose(L, M, Mt, n, n, nn, nn, st)) != hipSuccess) return hip_fail(e, "M^T");
  if ((e = mdk::launch_transpose(L, A, At, nn, D, nn * D, nn * D, st)) != hipSuccess) return hip_fail(e, "A^T");
  if ((e = mdk::launch_transpose(L * D, At, AtT, n, n, nn, nn, st)) != hipSuccess) return hip_fail(e, "A_k^T");
  if ((e = mdk::launch_gemm(L, n, Mt, AtT + nn, nn * D, Nt, mdk::stages_products(L, n, D), st)) != hipSuccess)
    return hip_fail(e, "gemm");
  if ((e = mdk::launch_series_to_rev(L, n, D, g_lambda, rho, st)) != hipSuccess) return hip_fail(e, "reverse");
  if ((e = mdk::launch_stages(L, n, D, Mt, Nt, AtT, rho, lamT, sync, dev_status, st)) != hipSuccess)
    return hip_fail(e, "stages");
  if ((e = mdk::launch_rev_to_series(L, n, D, lamT, g_lambda, st)) != hipSuccess) return hip_fail(e, "reverse");
  return MD_OK;
}

int md_coef_grad(const md_plan *p, const double *x, const double *lambda, double *grad_cff, void *ws, size_t ws_bytes,
                 hipStream_t st) {
  if (!p || !x || !lambda || (p->m > 0 && !grad_cff)) return fail(MD_EINVAL, "NULL argument");
  Layout w = newton_layout(p);
  if (!ws || ws_bytes < w.total) return fail(MD_ENOSPACE, "workspace too small");
  if (p->m == 0) return MD_OK;
  hipError_t e;
  double *unit = at(ws, w.unit);
  if ((e = mdk::launch_unit_md(p->L, p->m, unit, st)) != hipSuccess) return hip_fail(e, "unit");
  mdk::EvalArgs a;
  eval_args(p, unit, x, ws, p->D, a);
  if ((e = mdk::launch_evaldiff(p->L, a, p->maxexp, at(ws, w.pw), st)) != hipSuccess) return hip_fail(e, "values");
  if ((e = mdk::launch_coef_grad(p->L, p->n, p->D, p->m, p->d_row_of, lambda, a.val, grad_cff, st)) != hipSuccess)
    return hip_fail(e, "coef grad");
  return MD_OK;
}

int md_timing_enable(int on) {
  g_timing = on != 0;
  return MD_OK;
}

int md_timing_read(double *ms, int64_t *launches) {
  if (!ms || !launches) return fail(MD_EINVAL, "NULL argument");
  for (const EventPair &p : g_pending) {
    float t = 0.0f;
    hipError_t e = hipEventSynchronize(p.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, p.a, p.b);
    if (e == hipSuccess) {
      g_ms[p.cls] += t;
      g_count[p.cls] += 1;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
  for (int c = 0; c < MD_NCLASSES; ++c) {
    ms[c] = g_ms[c];
    launches[c] = g_count[c];
    g_ms[c] = 0.0;
    g_count[c] = 0;
  }
  return MD_OK;
}

int md_arith(int prec, int op, int64_t count, const double *a, const double *b, double *c, hipStream_t st) {
  if (!valid_prec(prec) || op < 0 || op > 6 || count < 0) return fail(MD_EINVAL, "bad precision, op or count");
  if (count == 0 && op != 6) return MD_OK;
  if (!a || !c || (op != 4 && !b)) return fail(MD_EINVAL, "NULL argument");
  if (count > ((int64_t)1 << 31) * 256) return fail(MD_EINVAL, "count too large");
  hipError_t e = (op == 6) ? mdk::launch_dot(prec, count, a, b, c, st) : mdk::launch_arith(prec, op, count, a, b, c, st);
  return e == hipSuccess ? MD_OK : hip_fail(e, "arith launch");
}

}  // extern "C"
