// Arguments of the evaluation and differentiation kernels (Section 5.1).
#pragma once
#include <cstddef>
#include <cstdint>

namespace mdk {

struct EvalArgs {
  int n, D, Dc, m, nnz;  // D: coefficients stored per series, Dc <= D: coefficients computed
  const int32_t *mon_ptr, *var, *exp, *order;
  const double *cff, *x, *pw;  // pw: powers x^p for p = 2..maxexp-1, [p-2][L][n][D]
  double *val, *der;           // val [L][m][D], der [L][nnz][D]
  int values_only = 0;         // 1: monomial values only (no backward or cross products, der untouched)
  size_t x_ls = 0, cff_ls = 0; // limb strides of x and cff when not n D and m (packed batches)
  double *vsize = nullptr;     // [m][D], nullable: max_j |f_j| over each monomial's forward chain (leading limbs)
  int beside_qr = 0;           // 1: runs beside the QR (one wavefront per monomial, more issue slots for the QR)
  int32_t *reset_status = nullptr;  // coefficient-0 kernel: its first thread sets this status word to MD_OK
  // coefficient-0 kernel: x is written by a launch on another stream, which
  // adds one to *wait_ctr per workgroup once its stores are performed; wait
  // until it reaches wait_target (bounded: MD_EHIP into wait_status), then
  // read x at the device's point of coherence
  const int *wait_ctr = nullptr;
  int wait_target = 0;
  int32_t *wait_status = nullptr;
};

}  // namespace mdk
