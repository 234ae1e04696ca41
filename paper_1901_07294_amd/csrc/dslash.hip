// The Wilson-Dirac operator on gfx950: one lane per lattice site.
//
//   out(x) = (4+m) psi(x) - 1/2 sum_mu [ (1-g_mu) U_mu(x) psi(x+mu)
//                                       + (1+g_mu) U_mu(x-mu)^dag psi(x-mu) ]
//
// (the hopping term of eq. (1), Sec. II-A, with the opposite sign of gamma_mu
// and the (4+m) normalisation), optionally multiplied by gamma5 = diag(1,1,-1,-1).
//
// The stencil is bound by HBM bandwidth (1320 flop against >= 960 compulsory
// bytes per site in FP64), so there is no matrix-core work here: every lane
// streams its site's links and spinor planes, coalesced across the wave.
#include <atomic>

#include "stencil.h"
#include "wd_internal.h"

// Compile-time tuning knobs (the defaults are the measured best on MI355X).
#ifndef WD_DSLASH_BLOCK
#define WD_DSLASH_BLOCK 256   // threads per workgroup
#endif
#ifndef WD_XCD_GROUP
#define WD_XCD_GROUP -1       // tiles per XCD run; -1 picks automatically
#endif
#ifndef WD_DSLASH_KERNEL
#define WD_DSLASH_KERNEL 0    // 0: t-marching where the lattice allows it, 1: one site per lane
#endif
#ifndef WD_MARCH_THREADS
#define WD_MARCH_THREADS 256  // target sites per t-marching tile
#endif
#ifndef WD_MARCH_WG_PER_CU
#define WD_MARCH_WG_PER_CU 2  // t-marching workgroups per CU aimed for (LDS permitting)
#endif
#ifndef WD_MARCH_XCD_GROUP
#define WD_MARCH_XCD_GROUP 32 // preferred XCD run length of t-marching tiles
#endif

namespace wd {
namespace {

constexpr int kDslashBlock = WD_DSLASH_BLOCK;
constexpr int kMarchMaxThreads = 256;
constexpr int kMarchTargetThreads = WD_MARCH_THREADS;
constexpr int kMarchWgPerCu = WD_MARCH_WG_PER_CU;
constexpr int kNumCu = 256;
constexpr int kMarchXcdGroup = WD_MARCH_XCD_GROUP;
constexpr size_t kLdsBytes = 160 * 1024;  // LDS per CU on gfx950

// Workgroup -> tile of kBlock consecutive sites. Consecutive workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2; with
// group > 0 the mapping gives every XCD runs of `group` consecutive tiles, so
// that neighbours in y and z, which sit a few tiles away, share an L2.
__device__ __forceinline__ int tile_of_block(int group) {
  const int b = blockIdx.x;
  const int nb = gridDim.x;
  if (group <= 0 || nb % (kNumXcd * group) != 0) return b;
  const int xcd = b % kNumXcd;
  const int l = b / kNumXcd;
  return ((l / group) * kNumXcd + xcd) * group + (l % group);
}

template <typename R, bool C12>
__global__ __launch_bounds__(kDslashBlock) void dslash_kernel(const typename Packed<R>::S* __restrict__ in,
                                                        typename Packed<R>::S* __restrict__ out,
                                                        const typename Packed<R>::L* __restrict__ links,
                                                        Geo geo, R diag, int gamma5, int group) {
  const int s = tile_of_block(group) * kDslashBlock + static_cast<int>(threadIdx.x);
  if (s >= geo.V) return;
  const long V = geo.V;

  const int x = s % geo.X;
  const int y = (s / geo.X) % geo.Y;
  const int z = (s / geo.XY) % geo.Z;
  const int t = s / geo.XYZ;
  // periodic neighbours (extent 1 wraps onto the site itself)
  const int xp = x + 1 == geo.X ? s - (geo.X - 1) : s + 1;
  const int xm = x == 0 ? s + (geo.X - 1) : s - 1;
  const int yp = y + 1 == geo.Y ? s - (geo.Y - 1) * geo.X : s + geo.X;
  const int ym = y == 0 ? s + (geo.Y - 1) * geo.X : s - geo.X;
  const int zp = z + 1 == geo.Z ? s - (geo.Z - 1) * geo.XY : s + geo.XY;
  const int zm = z == 0 ? s + (geo.Z - 1) * geo.XY : s - geo.XY;
  const int tp = t + 1 == geo.T ? s - (geo.T - 1) * geo.XYZ : s + geo.XYZ;
  const int tm = t == 0 ? s + (geo.T - 1) * geo.XYZ : s - geo.XYZ;

  cx<R> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};

  hop<0, -1, C12, R>(in, links, V, xp, s, acc);
  hop<0, +1, C12, R>(in, links, V, xm, xm, acc);
  hop<1, -1, C12, R>(in, links, V, yp, s, acc);
  hop<1, +1, C12, R>(in, links, V, ym, ym, acc);
  hop<2, -1, C12, R>(in, links, V, zp, s, acc);
  hop<2, +1, C12, R>(in, links, V, zm, zm, acc);
  hop<3, -1, C12, R>(in, links, V, tp, s, acc);
  hop<3, +1, C12, R>(in, links, V, tm, tm, acc);

  cx<R> psi[12];
  load_spinor(in, V, s, psi);
  cx<R> o[12];
  epilogue(psi, acc, diag, gamma5, o);
  store_spinor(out, V, s, o);
}

// ---------------------------------------------------------------------------
// t-marching kernel.
//
// A workgroup owns a tile of X x NY sites (whole x rows) at one z and walks
// t0 .. t1-1. The tile's spinors at the current t sit in LDS (double
// buffered), so the x and in-tile y neighbours are read from LDS; the t
// neighbours come from the march itself: psi(t+1) is the workgroup's own
// next slice, and the backward t hop of step t+1, U_t(t)^dag P+ psi(t), is
// built from data of step t and carried in the accumulator. The z hops and
// the y hops that leave the tile need other workgroups' sites; they are done
// one step early, while the workgroups that own those sites load the same
// slice, so their lines are still in L2.
// ---------------------------------------------------------------------------

struct MarchParams {
  int ny;      // rows per tile (divides Y)
  int tb;      // t steps per workgroup
  int ytiles;  // Y / ny
  int group;   // XCD run length (tiles), 0 = hardware order
};

// Hops of time t that involve sites outside the tile: z forward and
// backward, and the y hops of the tile's edge rows.
template <bool C12, typename R>
__device__ __forceinline__ void outer_hops(const typename Packed<R>::S* __restrict__ in,
                                           const typename Packed<R>::L* __restrict__ links, long V,
                                           int st, int dzp, int dzm, bool y_fwd_out, int dyp,
                                           bool y_bwd_out, int dym, cx<R> (&acc)[12]) {
  hop<2, -1, C12, R>(in, links, V, st + dzp, st, acc);
  hop<2, +1, C12, R>(in, links, V, st + dzm, st + dzm, acc);
  if (y_fwd_out) hop<1, -1, C12, R>(in, links, V, st + dyp, st, acc);
  if (y_bwd_out) hop<1, +1, C12, R>(in, links, V, st + dym, st + dym, acc);
}

template <typename R, bool C12>
__global__ __launch_bounds__(kMarchMaxThreads) void dslash_march_kernel(
    const typename Packed<R>::S* __restrict__ in, typename Packed<R>::S* __restrict__ out,
    const typename Packed<R>::L* __restrict__ links, Geo geo, R diag, int gamma5, MarchParams p) {
  using SV = typename Packed<R>::S;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = geo.X * p.ny;  // sites per tile == threads per workgroup
  SV* buf0 = reinterpret_cast<SV*>(smem);
  SV* buf1 = buf0 + (sizeof(R) == 8 ? 12 : 6) * n;
  const long V = geo.V;

  const int tid = static_cast<int>(threadIdx.x);
  const int xl = tid % geo.X;
  const int yl = tid / geo.X;
  const int b = tile_of_block(p.group);
  const int yt = b % p.ytiles;
  const int z = (b / p.ytiles) % geo.Z;
  const int tblk = b / (p.ytiles * geo.Z);
  const int y = yt * p.ny + yl;
  const int t0 = tblk * p.tb;
  const int t1 = min(t0 + p.tb, geo.T);

  const int s0 = xl + geo.X * (y + geo.Y * z);  // the site at t = 0
  // LDS slots of the in-tile x and y neighbours
  const int lxp = yl * geo.X + (xl + 1 == geo.X ? 0 : xl + 1);
  const int lxm = yl * geo.X + (xl == 0 ? geo.X - 1 : xl - 1);
  const bool whole_y = p.ny == geo.Y;
  const bool y_fwd_out = !whole_y && yl + 1 == p.ny;
  const bool y_bwd_out = !whole_y && yl == 0;
  const int lyp = (yl + 1 == p.ny ? 0 : yl + 1) * geo.X + xl;
  const int lym = (yl == 0 ? p.ny - 1 : yl - 1) * geo.X + xl;
  // site offsets of the periodic neighbours
  const int dxm = xl == 0 ? geo.X - 1 : -1;
  const int dyp = y + 1 == geo.Y ? -(geo.Y - 1) * geo.X : geo.X;
  const int dym = y == 0 ? (geo.Y - 1) * geo.X : -geo.X;
  const int dzp = z + 1 == geo.Z ? -(geo.Z - 1) * geo.XY : geo.XY;
  const int dzm = z == 0 ? (geo.Z - 1) * geo.XY : -geo.XY;

  cx<R> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};

  // prologue: the carried hops of t0 and the first slice in LDS
  {
    const int tm = t0 == 0 ? geo.T - 1 : t0 - 1;
    hop<3, +1, C12, R>(in, links, V, s0 + tm * geo.XYZ, s0 + tm * geo.XYZ, acc);
    const int st = s0 + t0 * geo.XYZ;
    outer_hops<C12, R>(in, links, V, st, dzp, dzm, y_fwd_out, dyp, y_bwd_out, dym, acc);
    cx<R> psi[12];
    load_spinor(in, V, st, psi);
    lds_store_spinor(buf0, n, tid, psi);
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    SV* cur = ((t - t0) & 1) ? buf1 : buf0;
    SV* nxt = ((t - t0) & 1) ? buf0 : buf1;
    const int st = s0 + t * geo.XYZ;
    const int sn = t + 1 == geo.T ? s0 : st + geo.XYZ;  // the site at t+1
    const bool more = t + 1 < t1;

    // Slice t+1: this workgroup's own spinors (forward t hop, next LDS
    // slice) and, in the same window, the z and off-tile y hops of t+1,
    // whose spinors other workgroups are loading as their own slice now.
    cx<R> ut[9];
    load_link<C12>(links, V, 3, st, ut);
    cx<R> nacc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) nacc[c] = {R(0), R(0)};
    {
      cx<R> psi[12];
      load_spinor(in, V, sn, psi);
      if (more) {
        lds_store_spinor(nxt, n, tid, psi);
        outer_hops<C12, R>(in, links, V, sn, dzp, dzm, y_fwd_out, dyp, y_bwd_out, dym, nacc);
      }
      cx<R> h[6], g[6];
      project<3, -1>(psi, h);
      su3_mul<false>(ut, h, g);
      reconstruct_add<3, -1>(g, acc);
    }
    // x hops and in-tile y hops from LDS
    {
      cx<R> psi[12];
      lds_load_spinor(cur, n, lxp, psi);
      hop_psi<0, -1, C12, R>(psi, links, V, st, acc);
      lds_load_spinor(cur, n, lxm, psi);
      hop_psi<0, +1, C12, R>(psi, links, V, st + dxm, acc);
      if (!y_fwd_out) {
        lds_load_spinor(cur, n, lyp, psi);
        hop_psi<1, -1, C12, R>(psi, links, V, st, acc);
      }
      if (!y_bwd_out) {
        lds_load_spinor(cur, n, lym, psi);
        hop_psi<1, +1, C12, R>(psi, links, V, st + dym, acc);
      }
    }
    // epilogue of t; the backward t hop of t+1 joins the next accumulator
    {
      cx<R> psi[12];
      lds_load_spinor(cur, n, tid, psi);
      cx<R> o[12];
      epilogue(psi, acc, diag, gamma5, o);
      store_spinor(out, V, st, o);
      if (more) {
        cx<R> h[6], g[6];
        project<3, +1>(psi, h);
        su3_mul<true>(ut, h, g);
        reconstruct_add<3, +1>(g, nacc);
      }
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = nacc[c];
    __syncthreads();
  }
}

int xcd_group(int nblocks, int preferred) {
  if (WD_XCD_GROUP >= 0) return WD_XCD_GROUP;
  for (int g = preferred; g > 1; g /= 2)
    if (nblocks % (kNumXcd * g) == 0) return g;
  return 0;
}

// Geometry of the t-marching kernel for a lattice, or ny = 0 if it does not
// apply (x rows longer than a workgroup, or too few sites per tile).
size_t march_lds_bytes(int threads, size_t real_bytes) {
  return 2 * 24 * real_bytes * static_cast<size_t>(threads);  // two spinor slices
}



MarchParams march_params(const Geo& geo, size_t real_bytes) {
  MarchParams p{0, 0, 0, 0};
  if (geo.X > kMarchMaxThreads) return p;
  int ny = 0;
  for (int d = 1; d <= geo.Y; ++d)
    if (geo.Y % d == 0 && geo.X * d <= kMarchTargetThreads &&
        march_lds_bytes(geo.X * d, real_bytes) <= kLdsBytes)
      ny = d;
  if (ny == 0 || geo.X * ny < 64) return p;
  p.ny = ny;
  p.ytiles = geo.Y / ny;
  const int planes = p.ytiles * geo.Z;
  // as many workgroups as fit on the chip at once (LDS decides how many per
  // CU), t steps split evenly among the workgroups of one tile column
  const int per_cu = static_cast<int>(kLdsBytes / march_lds_bytes(geo.X * ny, real_bytes));
  const int target = kNumCu * (per_cu < kMarchWgPerCu ? per_cu : kMarchWgPerCu);
  int nt = (target + planes - 1) / planes;
  nt = nt < 1 ? 1 : (nt > geo.T ? geo.T : nt);
  p.tb = (geo.T + nt - 1) / nt;
  const int nb = planes * ((geo.T + p.tb - 1) / p.tb);
  p.group = xcd_group(nb, kMarchXcdGroup);
  return p;
}

template <typename R, bool C12>
hipError_t launch_march(const void* in, void* out, const void* links, const Geo& geo, R diag,
                        int g5, const MarchParams& p, hipStream_t st) {
  using SV = typename Packed<R>::S;
  using LV = typename Packed<R>::L;
  const int threads = geo.X * p.ny;
  const size_t lds = march_lds_bytes(threads, sizeof(R));
  // raise the kernel's dynamic LDS limit once to the whole LDS of a CU
  static std::atomic<int> attr_set{0};
  if (!attr_set.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&dslash_march_kernel<R, C12>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(kLdsBytes));
    if (e != hipSuccess) return e;
    attr_set.store(1, std::memory_order_release);
  }
  const unsigned nb = static_cast<unsigned>(p.ytiles * geo.Z * ((geo.T + p.tb - 1) / p.tb));
  dslash_march_kernel<R, C12><<<nb, threads, lds, st>>>(
      static_cast<const SV*>(in), static_cast<SV*>(out), static_cast<const LV*>(links), geo, diag,
      g5, p);
  return hipGetLastError();
}

template <typename R, bool C12>
hipError_t launch_site(const void* in, void* out, const void* links, const Geo& geo, R diag, int g5,
                       hipStream_t st) {
  using SV = typename Packed<R>::S;
  using LV = typename Packed<R>::L;
  const unsigned nb = static_cast<unsigned>((geo.V + kDslashBlock - 1) / kDslashBlock);
  const int group = xcd_group(static_cast<int>(nb), 8);
  dslash_kernel<R, C12><<<nb, kDslashBlock, 0, st>>>(static_cast<const SV*>(in),
                                                       static_cast<SV*>(out),
                                                       static_cast<const LV*>(links), geo, diag,
                                                       g5, group);
  return hipGetLastError();
}

template <typename R, bool C12>
hipError_t launch_typed(const void* in, void* out, const void* links, const Geo& geo, double mass,
                        int g5, hipStream_t st) {
  const R diag = static_cast<R>(4.0 + mass);
  const MarchParams p = march_params(geo, sizeof(R));
  if (WD_DSLASH_KERNEL == 0 && p.ny > 0)
    return launch_march<R, C12>(in, out, links, geo, diag, g5, p, st);
  return launch_site<R, C12>(in, out, links, geo, diag, g5, st);
}

}  // namespace

hipError_t launch_dslash(const wd_gauge* g, double mass, const void* in, void* out, int flags,
                         hipStream_t st) {
  const Geo geo = make_geo(g->dims);
  const int g5 = (flags & WD_FLAG_GAMMA5) ? 1 : 0;
  if (g->prec == WD_FP64)
    return g->c12 ? launch_typed<double, true>(in, out, g->links, geo, mass, g5, st)
                  : launch_typed<double, false>(in, out, g->links, geo, mass, g5, st);
  return g->c12 ? launch_typed<float, true>(in, out, g->links, geo, mass, g5, st)
                : launch_typed<float, false>(in, out, g->links, geo, mass, g5, st);
}

}  // namespace wd
