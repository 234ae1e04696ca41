// Vector kernels of the CG solver (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "wilson.h"

namespace wd {

constexpr int kMaxRhs = 16;         // right-hand sides per solve
constexpr int kMaxPartials = 1024;  // per-workgroup partial sums per right-hand side

// The right-hand sides a launch works on: one grid row (blockIdx.y) each.
struct RhsSet {
  int n;
  int idx[kMaxRhs];
};

// Per right-hand side scalars in device memory (doubles).
enum : int {
  kRr = 0,      // <r, r> of the current residual
  kPap = 1,     // <p, A p>
  kAlpha = 2,
  kBeta = 3,
  kRrMax = 4,   // largest <r, r> since the last true residual
  kRrTrue = 5,  // <r, r> of the last true residual
  kB2 = 6,      // <b, b>
  kFlag = 7,    // nonzero: a non-finite or non-positive quantity appeared
  kRrPrev = 8,  // <r, r> before the current x, r update (beta's denominator)
  kAlphaPrev = 9,  // alpha of an x update left for the next iteration (blas_update_xp_lo)
  kScalars = 10  // even: the scalars are cleared as 16-byte elements
};

// What a reduction's result updates (finalize modes).
enum : int { kFinPap = 0, kFinTrueRr = 2, kFinNorm = 3 };

// n: 16-byte elements per right-hand side of the vectors in precision prec;
// nhi: FP64 elements per right-hand side; V: lattice sites. The number of
// partial sums of a reduction depends only on the lattice and precision.
hipError_t blas_norm2(const void* v, int prec, long n, long V, const RhsSet& set, double* partials,
                      double* scal, int mode, hipStream_t st);
// Partial sums of |v|^2 only (*nparts per right-hand side), for a following
// kernel that reduces them itself.
hipError_t blas_norm2_partials(const void* v, int prec, long n, long V, const RhsSet& set,
                               double* partials, int* nparts, hipStream_t st);
// x += alpha p, r -= alpha Ap with alpha = <r,r> / <p,Ap> reduced from the
// npap partials in pap (written by blas_norm2_partials on Q p, a buffer other
// than partials); x is the FP64 solution for FP64 vectors, else the FP32
// accumulator x_lo (nlo32 16-byte FP32 elements per right-hand side). Leaves
// the *nrr partial sums of the new <r,r> per right-hand side in partials.
hipError_t blas_update_xr(void* x, void* r, const void* p, const void* ap, int prec, long n, long nlo32,
                          long V, const RhsSet& set, const double* pap, int npap, double* partials,
                          int* nrr, double* scal, hipStream_t st);
// FP64 vectors, an iteration's vector work in two launches that read p once:
// blas_update_r does r -= alpha Ap (alpha reduced from the npap partials in
// pap, as blas_update_xr) and leaves the *nrr partial sums of the new <r,r> in
// partials; blas_update_xp then does x += alpha p and p = r + beta p (beta
// reduced from those partials, as blas_update_p). Same bits as blas_update_xr
// followed by blas_update_p.
hipError_t blas_update_r(void* r, const void* ap, long n, long V, const RhsSet& set, const double* pap,
                         int npap, double* partials, int* nrr, double* scal, hipStream_t st);
hipError_t blas_update_xp(void* x, void* p, const void* r, long n, const RhsSet& set, const double* rr,
                          int nrr, double* scal, hipStream_t st);
// Mixed precision (FP32 or FP16-storage vectors), after the dslash launch that
// applied r -= alpha Ap in its epilogue: x_lo += alpha p (alpha as that launch
// recorded it; x_lo the FP32 accumulator, nlo32 16-byte elements per
// right-hand side), then p = r + beta p with beta reduced from the nrr <r,r>
// partial sums in rr; p is read once. kind:
//   kXpNow:   x_lo += alpha p_cur; p_out = r + beta p_cur (p_out may be p_cur)
//   kXpDefer: p_out = r + beta p_cur into another buffer, x_lo left alone and
//             alpha kept (kAlphaPrev) for the next call
//   kXpPair:  x_lo += alpha_prev p_prev, then += alpha p_cur (the two updates
//             of kXpNow calls in turn, bit for bit); p_out = r + beta p_cur
//             (p_out may be p_prev)
enum : int { kXpNow = 0, kXpDefer = 1, kXpPair = 2 };
hipError_t blas_update_xp_lo(void* x, void* p_out, const void* p_cur, const void* p_prev, const void* r,
                             int kind, int prec, long n, long nlo32, long V, const RhsSet& set,
                             const double* rr, int nrr, double* scal, hipStream_t st);
// x_hi += x_lo, then x_lo = 0
hipError_t blas_flush_x(void* hi, void* lo, long nlo32, long nhi, const RhsSet& set, hipStream_t st);
// p = r + beta p with beta = <r,r>_new / <r,r>_old, <r,r>_new reduced from the
// nrr partial sums blas_update_xr left in rr; also records the new <r,r>.
hipError_t blas_update_p(void* p, const void* r, int prec, long n, long V, const RhsSet& set,
                         const double* rr, int nrr, double* scal, hipStream_t st);
hipError_t blas_residual(void* r, const void* b, long n, long V, const RhsSet& set, double* partials,
                         double* scal, hipStream_t st);
// Mixed precision true residual: lo (FP32 or FP16) = b - ax (ax holds A x,
// FP64) rounded, with <r, r> of the FP64 values recorded as blas_residual
// does; the FP64 residual itself is not stored.
hipError_t blas_residual_demote(void* lo, const void* b, const void* ax, int prec, long n, long nhi, long V,
                                const RhsSet& set, double* partials, double* scal, hipStream_t st);
// lo (FP32 or FP16) = hi (FP64)
hipError_t blas_demote(void* lo, const void* hi, int prec, long n, long nhi, long V, const RhsSet& set,
                       hipStream_t st);
hipError_t blas_copy(void* dst, const void* src, int prec, long n, const RhsSet& set, hipStream_t st);
hipError_t blas_zero(void* dst, int prec, long n, const RhsSet& set, hipStream_t st);

}  // namespace wd
