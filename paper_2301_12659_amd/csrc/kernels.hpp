// Host-side launchers of the device kernels (one translation unit per area).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mdk {

struct EvalArgs {
  int n, D, m, nnz;
  const int32_t *mon_ptr, *var, *exp, *order;
  const double *cff, *x, *pw;  // pw: powers x^p for p = 2..maxexp-1, [p-2][L][n][D]
  double *val, *der;           // val [L][m][D], der [L][nnz][D]
};

// evaldiff.hip
hipError_t launch_evaldiff(int L, const EvalArgs &a, int maxexp, double *pw, hipStream_t st);
hipError_t launch_assemble(int L, int n, int D, int m, int nnz, const int32_t *poly_ptr, const int32_t *asm_ptr,
                           const int32_t *asm_ent, const double *cst, const double *val, const double *der,
                           double *b, double *A, hipStream_t st);
size_t evaldiff_lds_bytes(int L, int D);

// linalg.hip
hipError_t launch_status_init(int32_t *status, hipStream_t st);
hipError_t launch_qr(int L, int n, double *a, double *tau, int32_t *status, hipStream_t st);
hipError_t launch_form_m(int L, int n, const double *qr, const double *tau, double *invd, double *M, int32_t *status,
                         hipStream_t st);
hipError_t launch_extract(int L, int n, int D, int k, const double *A, double *out, hipStream_t st);
hipError_t launch_gemm_series(int L, int n, int D, int kb, const double *M, const double *A, double *N,
                              hipStream_t st);
hipError_t launch_stages(int L, int n, int D, const double *M, const double *N, const double *A, double *r,
                         double *dx, hipStream_t st);
hipError_t launch_update(int L, int n, int D, const double *b, const double *dx, double *x, double *norms,
                         int32_t *status, hipStream_t st);
hipError_t launch_arith(int L, int op, int64_t count, const double *a, const double *b, double *c, hipStream_t st);
hipError_t launch_copy(const double *src, double *dst, size_t count, hipStream_t st);

}  // namespace mdk
