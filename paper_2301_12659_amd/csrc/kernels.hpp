// Host-side launchers of the device kernels (one translation unit per area).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "evalargs.hpp"

namespace mdk {

// Hand-over slots between the workgroups of a running kernel that the
// readers poll themselves: emptied by an earlier launch on the stream
// (SLOT_EMPTY, a signalling-NaN bit pattern that no computed value has),
// written once by their owner with agent-scope stores, read with
// agent-scope loads until no limb holds SLOT_EMPTY.
constexpr long long SLOT_EMPTY = 0x7ff4deadbeef5a5all;
__device__ __forceinline__ bool slot_empty(double x) { return __double_as_longlong(x) == SLOT_EMPTY; }

// Preparation of the LDS QR's hand-over memory, done by a launch ahead of
// the QR on its stream: the column flags cleared and the slots of tau and
// 1/(x_0 - beta) ([n][2 L] doubles) emptied.
struct QrPrep {
  int *flags = nullptr;      // [n]
  double *tboard = nullptr;  // [n][2 L]
  int n = 0, nt = 0;         // n, n 2 L
};
__device__ __forceinline__ void qr_prep_item(const QrPrep &q, size_t t) {
  if (q.flags && t < (size_t)q.n) q.flags[t] = 0;
  if (q.tboard && t < (size_t)q.nt) q.tboard[t] = __longlong_as_double(SLOT_EMPTY);
}

// evaldiff.hip
hipError_t launch_evaldiff(int L, const EvalArgs &a, int maxexp, double *pw, hipStream_t st);
// Coefficient 0 of the derivative products only (der[.][.][0]), one thread
// per monomial; for plans whose supports have at most
// evaldiff0_max_support(L) variables (none for octo doubles).
hipError_t launch_evaldiff0(int L, const EvalArgs &a, hipStream_t st);
int evaldiff0_max_support(int L);
// A coefficient-major copy written by an assembly kernel beside its
// series-major output: p[l][s - lo][q] for lo <= s < lo + W and limbs l < L
// (a window of the coefficients, its leading limbs), q the row (b) or the
// entry i n + j (A, lo = 0).  p == nullptr: none.
struct TOut {
  double *p = nullptr;
  int lo = 0, W = 0, L = 0;
};
// A count to wait for (wait_count): the launch that takes it ends only once
// *ctr >= target.  ctr == nullptr: none.
struct CountWait {
  const int *ctr = nullptr;
  int target = 0;
  int32_t *status = nullptr;
};
// The assembly kernels fill the first Dc coefficients of series stored with
// D; tsz (nullable, [n][D]) gets |c_{i,0,s}| + sum_m vsize_{m,s} (the
// evaluation's chain maxima; |value_{m,s}| when vsize is null), the size of
// the terms of b_{i,s}; rt and at the coefficient-major copies of b and A;
// clear (nullable) clear_count ints set to zero and empty (nullable)
// empty_count slots emptied (SLOT_EMPTY) by the b launch; launch_assemble
// also ends only after wait (so that the launches after it on st follow the
// work on another stream that counts itself done).
hipError_t launch_assemble(int L, int n, int D, int Dc, int m, int nnz, const int32_t *poly_ptr,
                           const int32_t *asm_ptr, const int32_t *asm_ent, const double *cst, const double *val,
                           const double *der, double *b, double *A, hipStream_t st, double *tsz = nullptr,
                           const double *vsize = nullptr, TOut rt = TOut(), TOut at = TOut(), int *clear = nullptr,
                           int clear_count = 0, double *empty = nullptr, size_t empty_count = 0,
                           CountWait wait = CountWait());
size_t evaldiff_lds_bytes(int L, int D);
int evaldiff_workers_per_block(int D);  // monomials per 256-thread workgroup
hipError_t launch_assemble_b(int L, int n, int D, int Dc, int m, const int32_t *poly_ptr, const double *cst,
                             const double *val, double *b, hipStream_t st, double *tsz = nullptr,
                             const double *vsize = nullptr, TOut rt = TOut(), int *clear = nullptr,
                             int clear_count = 0, double *empty = nullptr, size_t empty_count = 0);
hipError_t launch_assemble_A(int L, int n, int D, int Dc, int nnz, const int32_t *asm_ptr, const int32_t *asm_ent,
                             const double *der, double *A, hipStream_t st, TOut at = TOut());
hipError_t launch_assemble_A0(int L, int n, int D, int nnz, const int32_t *asm_ptr, const int32_t *asm_ent,
                              const double *der, double *a0, hipStream_t st, QrPrep prep);

// linalg.hip
// and *counter = *counter2 = 0
hipError_t launch_status_init(int32_t *status, hipStream_t st, int *counter = nullptr, int *counter2 = nullptr);
hipError_t launch_qr(int L, int n, double *a, double *tau, double *qt, int32_t *status, unsigned *bar,
                     hipStream_t st);
int qr_lds_workgroups(int L, int n, bool with_qt);
// prepared: the hand-over memory (flags, tboard) was prepared by an earlier
// launch on st (QrPrep).
hipError_t launch_qr_lds(int L, int n, double *a, double *tau, double *qt, int32_t *status, int *flags,
                         double *vboard, double *tboard, hipStream_t st, bool prepared = false);
// rs (nullable): L n n doubles of scratch for the rows of R scaled by their
// diagonal (n <= 64: a back substitution whose steps have no division)
// done (nullable, with rs): each column's workgroup adds one to it after
// agent-scope stores and a wait for them
hipError_t launch_m_from_qt(int L, int n, const double *qr, const double *qt, double *invd, double *M,
                            int32_t *status, hipStream_t st, double *rs = nullptr, int *done = nullptr);
hipError_t launch_form_m(int L, int n, const double *qr, const double *tau, double *invd, double *M, int32_t *status,
                         hipStream_t st);
hipError_t launch_extract(int L, int n, int D, int k, const double *A, double *out, hipStream_t st);
hipError_t launch_transpose(int L, const double *in, double *out, size_t rows, int cols, size_t in_ls,
                            size_t out_ls, hipStream_t st);
// The same with row strides: out[l][c][r] at out + l out_ls + c out_ld + r from
// in + l in_ls + r in_ld + c (a window of the coefficients of series).
hipError_t launch_transpose_ld(int L, const double *in, size_t in_ld, double *out, size_t out_ld, size_t rows,
                               int cols, size_t in_ls, size_t out_ls, hipStream_t st);
// out + c L n^2 = M (B + c n^2) for c < count (B with limb stride b_ls).
hipError_t launch_gemm(int L, int n, const double *M, const double *B, size_t b_ls, double *out, int count,
                       hipStream_t st);
// Staged solve of the block Toeplitz system on coefficient-major arrays.
// NP holds N = M A_1 and, when stages_products() is 2, P = M A_2 after it
// (L n^2 doubles each); sync is scratch of stages_sync_ints(D) ints.  One
// persistent launch when stages_persistent(), else one launch per stage.
bool stages_persistent(int L, int n, int D);
int stages_sync_ints(int D);
int stages_products(int L, int n, int D);
hipError_t launch_stages_sync(int L, int n, int D, int *sync, double *dxT, hipStream_t st);
hipError_t launch_stages(int L, int n, int D, const double *M, const double *NP, const double *At, double *rT,
                         double *dxT, int *sync, int32_t *status, hipStream_t st, bool sync_ready = false);
// launch_gemm (count products) and, in the same launch, xn [L][n] = x_0 +
// M r_0: coefficient 0 of the iterate after a step whose staged solve is the
// persistent one, bit for bit as that solve and launch_finish form it (rT:
// the step's coefficient-major right-hand side).
hipError_t launch_gemm_next_x0(int L, int n, int D, const double *M, const double *B, size_t b_ls, double *N,
                               int count, const double *rT, const double *x, double *xn, int *done, hipStream_t st);
// x_k += dx_k for lo <= k < hi; norms[2][D]: max |b_k| for k < hi and
// max |dx_k| for lo <= k < hi, zero elsewhere; with tsz ([n][D] term sizes
// from the assembly) rel[k] = max_i |b_{i,k}| / tsz[i][k] for k < hi, zero
// above (passed as the scale argument).
hipError_t launch_update(int L, int n, int D, int lo, int hi, const double *b, const double *dx, double *x,
                         double *norms, int32_t *status, hipStream_t st, const double *tsz = nullptr,
                         double *scale = nullptr);
hipError_t launch_finish(int L, int Ldx, int n, int D, int lo, int hi, const double *dxT, double *dx, double *x,
                         const double *b, double *norms, int32_t *status, hipStream_t st, const double *tsz = nullptr,
                         double *rel = nullptr);
// out[0 .. 3D]: norms[2][D], scale[D] and the status word (as a double),
// written by one small kernel (out may be mapped host memory).
hipError_t launch_report(int D, const double *norms, const double *scale, const int32_t *status, double *out,
                         hipStream_t st);
hipError_t launch_arith(int L, int op, int64_t count, const double *a, const double *b, double *c, hipStream_t st);
hipError_t launch_copy(const double *src, double *dst, size_t count, hipStream_t st);
hipError_t launch_series_to_rev(int L, int n, int D, const double *in, double *out, hipStream_t st);
hipError_t launch_rev_to_series(int L, int n, int D, const double *in, double *out, hipStream_t st);
hipError_t launch_coef_grad(int L, int n, int D, int m, const int32_t *row_of, const double *lambda, const double *val,
                            double *grad, hipStream_t st);
hipError_t launch_unit_md(int L, int m, double *c, hipStream_t st);
hipError_t launch_dot(int L, int64_t count, const double *a, const double *b, double *c, hipStream_t st);

// complex.hip: complex arrays [2][L][...] (real plane, imaginary plane).
hipError_t launch_evaldiff_complex(int L, const EvalArgs &a, hipStream_t st);
// At [L][2n][2n][D] = [[Re A, -Im A], [Im A, Re A]], bt [L][2n][D] = [Re b; Im b].
hipError_t launch_complex_embed(int L, int n, int D, const double *A, const double *b, double *At, double *bt,
                                hipStream_t st);
// dx [2][L][n][D] from dxt [L][2n][D].
hipError_t launch_complex_unpack(int L, int n, int D, const double *dxt, double *dx, hipStream_t st);
hipError_t launch_max(int count, const double *b, double *a, hipStream_t st);

// residual.hip: r [L][nrows][D] = b - T dx on rows (NULL: all), norm1 [D] (nullable).
hipError_t launch_residual(int L, int n, int D, int nrows, const int32_t *rows, const double *A, const double *b,
                           const double *dx, double *r, double *norm1, int32_t *status, hipStream_t st);

// api.hip: record the message returned by md_last_error and return the code.
int api_fail(int code, const char *msg);
int api_hip_fail(hipError_t e, const char *what);
bool api_timing_enabled();

}  // namespace mdk
