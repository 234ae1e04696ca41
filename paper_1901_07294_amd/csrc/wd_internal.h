// Internal declarations of the Wilson-Dirac library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "wilson.h"

// The handle behind wd_gauge*: geometry plus the caller-owned packed links.
struct wd_gauge {
  uint64_t magic;
  int32_t dims[4];   // X, Y, Z, T
  int64_t V;         // number of sites
  int32_t prec;      // wd_prec of the packed links and of the spinors used with them
  int32_t c12;       // links stored as two rows (12 reals)
  int32_t eo;        // links split by site parity (wd_gauge_import_eo): even sites' links, then odd
  int device;        // HIP device the packed links live on
  void* links;       // packed links (caller-owned)
  size_t link_bytes;
};

namespace wd {

constexpr uint64_t kGaugeMagic = 0x57444741554745ull;  // "WDGAUGE"
constexpr int kBlock = 256;                           // threads per workgroup, 4 wave64s
constexpr int kNumXcd = 8;                            // MI355X: 8 XCDs, 32 CUs each
constexpr int kMaxMultiRhs = 16;                      // right-hand sides per fused launch

// The right-hand sides of a launch (kernel argument): field index in the
// buffers and diagonal term 4 + m of each.
template <typename R>
struct Diag {
  R d[kMaxMultiRhs];
  int idx[kMaxMultiRhs];
};

// Set the thread's last-error text; returns code for `return set_error(...)`.
int set_error(int code, const char* fmt, ...);
void clear_error();

// Geometry passed to kernels by value.
struct Geo {
  int X, Y, Z, T;
  int XY, XYZ;
  int V;
};

inline Geo make_geo(const int32_t d[4]) {
  Geo g;
  g.X = d[0]; g.Y = d[1]; g.Z = d[2]; g.T = d[3];
  g.XY = g.X * g.Y;
  g.XYZ = g.XY * g.Z;
  g.V = g.XYZ * g.T;
  return g;
}

// Geometry of a lattice split by site parity (even extents): each parity is a
// field of Vh = V/2 half sites h = xh + Xh (y + Y (z + Z t)), x = 2 xh +
// ((y + z + t + parity) & 1).
struct EoGeo {
  int X, Y, Z, T, Xh;
  long Vh;
};

inline EoGeo make_eo_geo(const int32_t d[4]) {
  EoGeo g;
  g.X = d[0]; g.Y = d[1]; g.Z = d[2]; g.T = d[3];
  g.Xh = g.X / 2;
  g.Vh = static_cast<long>(g.X) * g.Y * g.Z * g.T / 2;
  return g;
}

// Argument checks shared by the entry points (they set the last error).
int check_dims(const int32_t dims[4], long* V);
int check_prec(int prec);
int check_device_range(const void* p, size_t bytes, const char* what);
bool overlaps(const void* a, size_t na, const void* b, size_t nb);
int check_gauge(const wd_gauge* g);
int check_layout(const wd_gauge* g, int eo, const char* what);
int check_even_dims(const int32_t dims[4]);
int launch_status(hipError_t e, const char* what);

// Bytes per site of packed fields.
size_t spinor_site_bytes(int prec);
size_t gauge_site_bytes(int prec, int c12);

// Kernel launchers (enqueue only; return the launch status).
hipError_t launch_pack_gauge(const void* canon, void* dst, const Geo& geo, int prec, int c12,
                             hipStream_t s);
hipError_t launch_pack_spinor(const void* canon, void* dst, const Geo& geo, int prec, int nrhs,
                              hipStream_t s);
hipError_t launch_unpack_spinor(const void* src, void* canon, const Geo& geo, int prec, int nrhs,
                                hipStream_t s);
hipError_t launch_dslash(const wd_gauge* g, double mass, const void* in, void* out, int flags,
                         hipStream_t s);

// Even-odd layout (pack.hip): bytes of one parity's packed links; packing
// canonical links into both; spinors of one parity between canonical (the
// other parity's sites zeroed on export) and packed half fields.
size_t eo_gauge_half_bytes(long Vh, int prec, int c12);
hipError_t launch_pack_gauge_eo(const void* canon, void* dst, const EoGeo& g, int prec, int c12,
                                hipStream_t s);
hipError_t launch_spinor_eo(const void* src, void* dst, const EoGeo& g, int prec, int parity, int nrhs,
                            bool import, hipStream_t s);
// nrhs (1..kMaxMultiRhs) packed fields of `in` / `out`: field fields[i] (or i
// if fields is null) with mass masses[i].
hipError_t launch_dslash_multi(const wd_gauge* g, const double* masses, int nrhs, const int* fields,
                               const void* in, void* out, int flags, hipStream_t s);

// Launch choices of the t-marching kernel that leave every site's arithmetic,
// and so every result bit, unchanged: t steps per workgroup, lane groups per
// workgroup, the run length of tiles per XCD (0: hardware order) and
// right-hand sides per lane (1 or 2).
struct MarchTuning {
  int32_t tb, gw, group, rb;
};
// The default choice for a lattice, precision and nrhs; false when the
// t-marching kernel does not apply (the one-site-per-lane kernel runs).
bool march_default(const int32_t dims[4], int prec, int nrhs, MarchTuning* t);
// Alternatives to the default (the default included), all valid.
void march_candidates(const int32_t dims[4], int prec, int nrhs, MarchTuning* out, int* n, int cap);
// Whether t may be used for a launch (bounds, lanes and LDS).
bool march_tuning_valid(const int32_t dims[4], int prec, int nrhs, const MarchTuning& t);
// launch_dslash_multi with an explicit choice (validated by the caller).
hipError_t launch_dslash_tuned(const wd_gauge* g, const double* masses, int nrhs, const void* in,
                               void* out, int flags, const MarchTuning& t, hipStream_t s);
// The autotuner's choice registered for (dims, prec, c12, nrhs), if any.
bool tuned_lookup(const int32_t dims[4], int prec, int c12, int nrhs, MarchTuning* t);

// Work of a CG iteration fused into its two applications of Q, as a mode of
// the t-marching kernel. kCgNorm (first application, t = Q p): t is stored
// and each tile slice (a tile's x rows at one z and t, so the grouping is
// fixed by the lattice, not the launch) leaves its |t|^2 = <p, A p> partial
// sum in rr. kCgUpdate (second application, A p = Q t): A p is used at once
// for r -= alpha A p (alpha = <r,r> / <p,Ap> reduced from pap) instead of
// being stored, and each tile slice leaves its <r,r>; x += alpha p is left
// to the p update, which reads p anyway.
enum : int { kCgNone = 0, kCgNorm = 1, kCgUpdate = 2 };
struct CgFuse {
  int mode;           // kCgNorm or kCgUpdate
  void* r;            // residual, inner precision
  const double* pap;  // <p, A p> partial sums, npap per field slot
  int npap;
  double* rr;         // out: |t|^2 or <r, r> per tile slice, nslices per field slot
  int nslices;
  double* scal;       // per field slot scalars (kScalars doubles)
};
// Tile slices of the fused work on a lattice in a precision, or 0 where it
// does not apply (the one-site-per-lane kernel, or tiles that are not whole
// waves). kCgUpdate exists for FP32 arithmetic (FP32 and FP16 storage) only.
int cg_fuse_slices(const int32_t dims[4], int prec);
// Q = gamma5 D(masses[i]) on field fields[i] of `in` (into `out` for
// kCgNorm), fused with the work of f.mode for the same field slots
// (cg_fuse_slices must be > 0).
hipError_t launch_dslash_cg(const wd_gauge* g, const double* masses, int nrhs, const int* fields,
                            const void* in, void* out, const CgFuse& f, hipStream_t s);

}  // namespace wd
