// Even-odd (red-black) pieces of the Wilson-Dirac solver (internal).
//
// With every extent even, each hop of the operator joins sites of opposite
// parity, so in the (even, odd) block order D = [[A, -H_eo/2], [-H_oe/2, A]]
// with A = 4 + m. The odd-site Schur complement is
//   S = A - H_oe H_eo / (4 A),
// and S x_o = b_o + H_oe b_e / (2 A) with x_e = (b_e + H_eo x_o / 2) / A
// solves D x = b. Fields of one parity are packed fields of V/2 sites
// (pack.hip); an even-odd gauge handle holds the even sites' links, then the
// odd sites'.
#pragma once

#include <hip/hip_runtime.h>

#include "blas.h"
#include "wd_internal.h"

namespace wd {

// Packed FP64 full-lattice fields (field set.idx[i] of `full`) to or from
// their even and odd half fields (the same field index in `even`, `odd`).
hipError_t launch_split_eo(const void* full, void* even, void* odd, const EoGeo& g, const RhsSet& set,
                           bool merge, hipStream_t s);

// out_k = d[i] w_k + c[i] (H_{p,1-p} in)_k for the fields k = set.idx[i]: the
// hopping sum H (both hops of every direction, no 1/2) from the input half
// fields of parity 1-p to the outputs of parity p, plus a multiple of a half
// field w of parity p (w may be null when every d[i] is 0), times gamma5 when
// g5. Fields are packed half fields of g's precision; g an even-odd handle.
hipError_t launch_eo_hop(const wd_gauge* g, int parity, const void* in, const void* w, void* out,
                         const RhsSet& set, const double* d, const double* c, int g5, hipStream_t s);

// out = gamma5 S in on the odd half fields of set (masses[i] for set.idx[i]),
// through the even half fields tmp: tmp = -H_eo in / 2, then
// out = gamma5 [(4+m) in + H_oe tmp / (2(4+m))].
hipError_t launch_schur_q(const wd_gauge* g, const double* masses, const RhsSet& set, const void* in,
                          void* tmp, void* out, hipStream_t s);

// dst = gamma5 src for FP64 packed fields of V sites (n 16-byte elements each).
hipError_t blas_gamma5(void* dst, const void* src, long n, const RhsSet& set, hipStream_t st);

}  // namespace wd
