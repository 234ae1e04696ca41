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

#include "blas.h"
#include "cg_site.h"
#include "stencil.h"
#include "wd_internal.h"

// Compile-time tuning knobs (the defaults are the measured best on MI355X).
#ifndef WD_DSLASH_BLOCK
#define WD_DSLASH_BLOCK 256   // threads per workgroup
#endif
#ifndef WD_MARCH_GW
#define WD_MARCH_GW 0         // right-hand sides per t-marching workgroup; 0 picks automatically
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
#define WD_MARCH_WG_PER_CU 4  // t-marching workgroups per CU aimed for (LDS permitting)
#endif
#ifndef WD_UT_NT
#define WD_UT_NT 1            // non-temporal loads of the t links in the t-marching kernel
#endif
#ifndef WD_MARCH_BUF
#define WD_MARCH_BUF 1        // FP64/FP32 fields below 4 GiB through buffer resources
#endif
#ifndef WD_X_SHFL
#define WD_X_SHFL 1           // backward x links from the neighbour lane (x rows within a wave)
#endif

namespace wd {
namespace {

constexpr int kDslashBlock = WD_DSLASH_BLOCK;
constexpr int kMarchMaxThreads = 256;       // lanes of a one-right-hand-side tile
constexpr int kMarchMultiThreads = 768;     // lanes of a several-right-hand-side workgroup
constexpr int kMarchTargetThreads = WD_MARCH_THREADS;
constexpr int kMarchWgPerCu = WD_MARCH_WG_PER_CU;
constexpr bool kUtNt = WD_UT_NT != 0;
constexpr bool kMarchBuf = WD_MARCH_BUF != 0;
constexpr bool kXShfl = WD_X_SHFL != 0;
constexpr int kNumCu = 256;
// Waves of the t-marching kernel a CU holds at once, from the compiled
// kernels' register use: 256 VGPRs in FP64 (one wave per SIMD), 146-168 with
// FP32 arithmetic (three per SIMD).
constexpr int kWavesPerCuFp64 = 4;
constexpr int kWavesPerCuFp32 = 12;
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

// T: storage type of spinors and links (double, float or _Float16).
template <typename T, bool C12>
__global__ __launch_bounds__(kDslashBlock) void dslash_kernel(
    const typename Packed<T>::S* __restrict__ in_all, typename Packed<T>::S* __restrict__ out_all,
    const typename Packed<T>::L* __restrict__ links, Geo geo, Diag<typename Packed<T>::R> diags,
    long stride, int gamma5, int group) {
  using R = typename Packed<T>::R;
  const int s = tile_of_block(group) * kDslashBlock + static_cast<int>(threadIdx.x);
  if (s >= geo.V) return;
  const long V = geo.V;
  const int rhs = blockIdx.y;
  const typename Packed<T>::S* in = in_all + diags.idx[rhs] * stride;
  typename Packed<T>::S* out = out_all + diags.idx[rhs] * stride;
  const R diag = diags.d[rhs];

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

  hop<0, -1, C12>(in, links, V, xp, s, acc);
  hop<0, +1, C12>(in, links, V, xm, xm, acc);
  hop<1, -1, C12>(in, links, V, yp, s, acc);
  hop<1, +1, C12>(in, links, V, ym, ym, acc);
  hop<2, -1, C12>(in, links, V, zp, s, acc);
  hop<2, +1, C12>(in, links, V, zm, zm, acc);
  hop<3, -1, C12>(in, links, V, tp, s, acc);
  hop<3, +1, C12>(in, links, V, tm, tm, acc);

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
  int group;   // XCD run length (workgroups), 0 = hardware order
  int nrhs;    // right-hand sides of the launch
  int gw;      // lane groups per workgroup
  int rb;      // right-hand sides per lane (gw * rb divides nrhs)
  unsigned link_bytes;    // bytes of the packed links and of one packed spinor field (used
  unsigned spinor_bytes;  // when they are read through buffer resources, below 4 GiB)
};

// How the march kernel reaches a field: a plain pointer (any size) or, with
// BUF, a buffer resource (fields below 4 GiB; no address arithmetic per load).
template <bool BUF, typename E>
__device__ __forceinline__ auto field_in(const E* p, unsigned bytes) {
  if constexpr (BUF) return buf_field(p, bytes);
  else return p;
}
template <bool BUF, typename E>
__device__ __forceinline__ auto field_out(E* p, unsigned bytes) {
  if constexpr (BUF) return buf_field(p, bytes);
  else return p;
}

// One hop for the RB right-hand sides of a lane: the link (direction MU at
// site ls) is loaded once and applied to each one's neighbour spinor at site
// nb. Each right-hand side sees exactly the operations of a one-field hop.
template <int MU, int S, bool C12, int RB, typename SA, typename LA, typename R>
__device__ __forceinline__ void hop_rb(const SA (&in)[RB], const LA& links, long V, int nb, int ls,
                                       cx<R> (&acc)[RB][12]) {
  cx<R> u[9];
  load_link<C12>(links, V, MU, ls, u);
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    cx<R> psi[12];
    load_spinor(in[r], V, nb, psi);
    cx<R> h[6], g[6];
    project<MU, S>(psi, h);
    su3_mul<(S > 0)>(u, h, g);
    reconstruct_add<MU, S>(g, acc[r]);
  }
}

// The same with the neighbour spinors read from the LDS slices (slot li).
template <int MU, int S, bool C12, int RB, typename SL, typename LA, typename R>
__device__ __forceinline__ void lds_hop_rb(SL* const (&slice)[RB], int n, int li, const LA& links, long V,
                                           int ls, cx<R> (&acc)[RB][12]) {
  cx<R> u[9];
  load_link<C12>(links, V, MU, ls, u);
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    cx<R> psi[12];
    lds_load_spinor(slice[r], n, li, psi);
    cx<R> h[6], g[6];
    project<MU, S>(psi, h);
    su3_mul<(S > 0)>(u, h, g);
    reconstruct_add<MU, S>(g, acc[r]);
  }
}

// The same with the link already in registers.
template <int MU, int S, int RB, typename SL, typename R>
__device__ __forceinline__ void lds_hop_u(SL* const (&slice)[RB], int n, int li, const cx<R> (&u)[9],
                                          cx<R> (&acc)[RB][12]) {
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    cx<R> psi[12];
    lds_load_spinor(slice[r], n, li, psi);
    cx<R> h[6], g[6];
    project<MU, S>(psi, h);
    su3_mul<(S > 0)>(u, h, g);
    reconstruct_add<MU, S>(g, acc[r]);
  }
}

// Both x hops from LDS. The backward hop's link U_x(x - 1) is the forward
// hop's link of the lane holding x - 1; with xshfl (every x row lies within
// one wave: X divides 64) it is taken from that lane with a cross-lane
// shuffle (the same values, no memory access), otherwise loaded.
template <bool C12, int RB, typename SL, typename LA, typename R>
__device__ __forceinline__ void lds_x_hops(SL* const (&slice)[RB], int n, int lxp, int lxm, const LA& links,
                                           long V, int st, int dxm, bool xshfl, int src_lane,
                                           cx<R> (&acc)[RB][12]) {
  cx<R> u[9];
  load_link<C12>(links, V, 0, st, u);
  lds_hop_u<0, -1>(slice, n, lxp, u, acc);
  if (xshfl) {
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = {__shfl(u[k].re, src_lane, 64), __shfl(u[k].im, src_lane, 64)};
  } else {
    load_link<C12>(links, V, 0, st + dxm, u);
  }
  lds_hop_u<0, +1>(slice, n, lxm, u, acc);
}

// Hops of time t that involve sites outside the tile: z forward and
// backward, and the y hops of the tile's edge rows.
template <bool C12, int RB, typename SA, typename LA, typename R>
__device__ __forceinline__ void outer_hops(const SA (&in)[RB], const LA& links, long V, int st, int dzp,
                                           int dzm, bool y_fwd_out, int dyp, bool y_bwd_out, int dym,
                                           cx<R> (&acc)[RB][12]) {
  hop_rb<2, -1, C12>(in, links, V, st + dzp, st, acc);
  hop_rb<2, +1, C12>(in, links, V, st + dzm, st + dzm, acc);
  if (y_fwd_out) hop_rb<1, -1, C12>(in, links, V, st + dyp, st, acc);
  if (y_bwd_out) hop_rb<1, +1, C12>(in, links, V, st + dym, st + dym, acc);
}

// Sum over the 64 lanes of a wave in a fixed order (every lane gets it).
__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Doubles of LDS per lane group and right-hand side that the fused CG work
// uses after the spinor slices: per-wave sums of two steps (tiles of at most
// 4 waves) and the per-wave sums of <p, A p>.
constexpr int kCgLds = 2 * 4 + 4;

// MAXT: launch bound. A workgroup holds p.gw groups of n = X * ny lanes of
// one tile; each lane carries RB right-hand sides (links loaded once for
// all), each with its own two LDS slices. The LDS slices hold spinors in the
// arithmetic precision (FP32 for FP16 storage).
// CGM (CG iterations, n a multiple of 64): kCgNorm stores the output and
// leaves each tile slice's squared norm of it in cgf.rr; kCgUpdate does not
// store the output but applies r -= alpha A p of cgf to the field slots (x
// and p follow in a separate kernel).
// The fused modes with FP32 arithmetic and one right-hand side per lane are
// compiled for three waves per SIMD (the plain FP32-arithmetic kernel's
// occupancy), at the cost of a few spilled registers in FP32 storage, which
// measured faster than two waves without spills.
template <int CGM, typename T, int RB>
constexpr int march_waves_per_eu() {
  return RB == 1 && sizeof(typename Packed<T>::R) == 4 && CGM != kCgNone ? 3 : 1;
}

template <typename T, bool C12, int MAXT, int RB, int CGM, bool BUF>
__global__ __launch_bounds__(MAXT)
__attribute__((amdgpu_waves_per_eu(march_waves_per_eu<CGM, T, RB>()))) void dslash_march_kernel(
    const typename Packed<T>::S* __restrict__ in, typename Packed<T>::S* __restrict__ out,
    const typename Packed<T>::L* __restrict__ links, Geo geo, Diag<typename Packed<T>::R> diags,
    long stride, int gamma5, MarchParams p, CgFuse cgf) {
  using R = typename Packed<T>::R;
  using SV = typename Packed<R>::S;
  using GS = typename Packed<T>::S;
  constexpr int kPlanes = sizeof(R) == 8 ? 12 : 6;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = geo.X * p.ny;  // sites per tile == lanes per lane group
  const int slot = static_cast<int>(threadIdx.x) / n;
  // slice (buffer f, right-hand side r) of this lane group
  SV* const base = reinterpret_cast<SV*>(smem) + slot * 2 * RB * kPlanes * n;
  const long V = geo.V;

  const int tid = static_cast<int>(threadIdx.x) - slot * n;
  const int xl = tid % geo.X;
  const int yl = tid / geo.X;
  // The lane groups of a workgroup march in lock step (one barrier per
  // step), so a link line fetched for one of them is an L1/L2 hit for the
  // others. Further workgroups of the same tile are consecutive.
  const int groups = p.nrhs / (p.gw * RB);
  const int bb = tile_of_block(p.group);
  // (with BUF the host launches one lane group per workgroup, so slot is 0 and
  // the fields' bases derive from the block index alone: wave-uniform)
  const int rhs0 = ((bb % groups) * p.gw + (BUF ? 0 : slot)) * RB;
  const int b = bb / groups;
  // the fields: plain pointers, or buffer resources (BUF; the fused CG work
  // writes its outputs through plain pointers)
  constexpr bool kBufOut = BUF && CGM == kCgNone;
  decltype(field_in<BUF>(in, 0u)) inr[RB];
  decltype(field_out<kBufOut>(out, 0u)) outr[RB];
  const auto lk = field_in<BUF>(links, p.link_bytes);
  R diag[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    inr[r] = field_in<BUF>(in + diags.idx[rhs0 + r] * stride, p.spinor_bytes);
    outr[r] = field_out<kBufOut>(out + diags.idx[rhs0 + r] * stride, p.spinor_bytes);
    diag[r] = diags.d[rhs0 + r];
  }
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
  // the lane holding x - 1, for the shuffled backward x link (x rows within a wave)
  // (measured: FP32 storage 196 -> 192 us on 32^3x64; FP64 unchanged; with
  // FP16 storage the 18 shuffles cost more than the 9 small loads they replace)
  const bool xshfl = kXShfl && sizeof(T) == 4 && RB == 1 && CGM == kCgNone && 64 % geo.X == 0;
  const int src_lane = (static_cast<int>(threadIdx.x) & 63) + dxm;
  const int dyp = y + 1 == geo.Y ? -(geo.Y - 1) * geo.X : geo.X;
  const int dym = y == 0 ? (geo.Y - 1) * geo.X : -geo.X;
  const int dzp = z + 1 == geo.Z ? -(geo.Z - 1) * geo.XY : geo.XY;
  const int dzm = z == 0 ? (geo.Z - 1) * geo.XY : -geo.XY;

  cx<R> acc[RB][12];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[r][c] = {R(0), R(0)};

  // fused CG work: per lane group and right-hand side, kCgLds doubles after
  // all spinor slices. For the update, alpha = <r,r> / <p,Ap>: every lane of
  // the tile sums a strided share of the <p,Ap> partial sums and each wave
  // its lanes (an order fixed by the tile size, which the lattice fixes);
  // after the prologue's barrier every lane adds the wave sums in order, so
  // all lanes of all workgroups get the same alpha
  double* cgs = reinterpret_cast<double*>(reinterpret_cast<SV*>(smem) + p.gw * 2 * RB * kPlanes * n) +
                slot * RB * kCgLds;
  double alpha[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) alpha[r] = 0.0;
  if constexpr (CGM == kCgUpdate) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const double* pp = cgf.pap + static_cast<long>(diags.idx[rhs0 + r]) * cgf.npap;
      double t = 0.0;
      int i = tid;
      for (; i + 3 * n < cgf.npap; i += 4 * n) {  // four loads in flight, added in order
        const double a0 = pp[i], a1 = pp[i + n], a2 = pp[i + 2 * n], a3 = pp[i + 3 * n];
        t += a0;
        t += a1;
        t += a2;
        t += a3;
      }
      for (; i < cgf.npap; i += n) t += pp[i];
      t = wave_total(t);
      if ((tid & 63) == 0) cgs[r * kCgLds + 8 + (tid >> 6)] = t;
    }
  }

  // prologue: the carried hops of t0 (in the loop's order: outer hops, then
  // the backward t hop, so every site rounds alike) and the first slice in LDS
  {
    const int tm = t0 == 0 ? geo.T - 1 : t0 - 1;
    const int st = s0 + t0 * geo.XYZ;
    outer_hops<C12>(inr, lk, V, st, dzp, dzm, y_fwd_out, dyp, y_bwd_out, dym, acc);
    hop_rb<3, +1, C12>(inr, lk, V, s0 + tm * geo.XYZ, s0 + tm * geo.XYZ, acc);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      cx<R> psi[12];
      load_spinor(inr[r], V, st, psi);
      lds_store_spinor(base + (2 * r) * kPlanes * n, n, tid, psi);
    }
  }
  __syncthreads();
  if constexpr (CGM == kCgUpdate) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      double t = 0.0;
      for (int w = 0; w < n / 64; ++w) t += cgs[r * kCgLds + 8 + w];
      const long k = diags.idx[rhs0 + r];
      double* sc = cgf.scal + k * kScalars;
      bool flag = false;
      alpha[r] = cg_alpha(t, sc[kRr], &flag);
      if (tid == 0 && b == 0) {  // the field's first tile: one workgroup per field
        sc[kPap] = t;
        sc[kAlpha] = alpha[r];
        sc[kRrPrev] = sc[kRr];
        if (flag) sc[kFlag] = 1.0;
      }
    }
  }

  for (int t = t0; t < t1; ++t) {
    const int f = (t - t0) & 1;  // the buffer holding slice t
    SV* cur[RB];
    SV* nxt[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      cur[r] = base + (2 * r + f) * kPlanes * n;
      nxt[r] = base + (2 * r + (f ^ 1)) * kPlanes * n;
    }
    const int st = s0 + t * geo.XYZ;
    const int sn = t + 1 == geo.T ? s0 : st + geo.XYZ;  // the site at t+1
    const bool more = t + 1 < t1;

    // Slice t+1: this workgroup's own spinors (forward t hop, next LDS
    // slice) and, in the same window, the z and off-tile y hops of t+1,
    // whose spinors other workgroups are loading as their own slice now.
    // U_t(t) serves the forward t hop of t and, from registers, the backward
    // t hop of t+1: no other workgroup reads it
    cx<R> ut[9];
    load_link<C12, kUtNt>(lk, V, 3, st, ut);
    cx<R> nacc[RB][12];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int c = 0; c < 12; ++c) nacc[r][c] = {R(0), R(0)};
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      cx<R> psi[12];
      load_spinor(inr[r], V, sn, psi);
      if (more) {
        lds_store_spinor(nxt[r], n, tid, psi);
        if (r == 0) outer_hops<C12>(inr, lk, V, sn, dzp, dzm, y_fwd_out, dyp, y_bwd_out, dym, nacc);
      }
      cx<R> h[6], g[6];
      project<3, -1>(psi, h);
      su3_mul<false>(ut, h, g);
      reconstruct_add<3, -1>(g, acc[r]);
    }
    // x hops and in-tile y hops from LDS
    lds_x_hops<C12>(cur, n, lxp, lxm, lk, V, st, dxm, xshfl, src_lane, acc);
    if (!y_fwd_out) lds_hop_rb<1, -1, C12>(cur, n, lyp, lk, V, st, acc);
    if (!y_bwd_out) lds_hop_rb<1, +1, C12>(cur, n, lym, lk, V, st + dym, acc);
    // epilogue of t; the backward t hop of t+1 joins the next accumulator
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      cx<R> psi[12];
      lds_load_spinor(cur[r], n, tid, psi);
      cx<R> o[12];
      epilogue(psi, acc[r], diag[r], gamma5, o);
      if constexpr (CGM == kCgUpdate) {
        const long k = diags.idx[rhs0 + r];
        double v = cg_site_update_r(static_cast<GS*>(cgf.r) + k * stride, V, st, o, alpha[r]);
        v = wave_total(v);
        if ((tid & 63) == 0) cgs[r * kCgLds + 4 * ((t - t0) & 1) + (tid >> 6)] = v;
      } else if constexpr (CGM == kCgNorm) {
        double v = store_site_norm(outr[r], V, st, o);
        v = wave_total(v);
        if ((tid & 63) == 0) cgs[r * kCgLds + 4 * ((t - t0) & 1) + (tid >> 6)] = v;
      } else if constexpr (kBufOut && sizeof(R) == 8 && !C12) {
        // FP64 with full links stores with the default cache policy (measured
        // 360.4 -> 358.9 us on 32^3x64; with 12-real links and in FP32 the
        // non-temporal stores are faster)
        store_spinor<0>(outr[r], V, st, o);
      } else {
        store_spinor(outr[r], V, st, o);
      }
      if (more) {
        cx<R> h[6], g[6];
        project<3, +1>(psi, h);
        su3_mul<true>(ut, h, g);
        reconstruct_add<3, +1>(g, nacc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[r][c] = nacc[r][c];
    __syncthreads();
    if constexpr (CGM != kCgNone) {
      // the squared norm of this tile slice (Q p or r): its waves in order (the next write to these
      // words is two steps on, behind the next barrier)
      if (tid == 0) {
        const long ts = (static_cast<long>(t) * geo.Z + z) * p.ytiles + yt;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          double sum = 0.0;
          for (int w = 0; w < n / 64; ++w) sum += cgs[r * kCgLds + 4 * ((t - t0) & 1) + w];
          cgf.rr[static_cast<long>(diags.idx[rhs0 + r]) * cgf.nslices + ts] = sum;
        }
      }
    }
  }
}

// Run length of consecutive workgroups per XCD: the largest power of two up
// to `preferred` that divides the grid evenly.
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



MarchParams march_params(const Geo& geo, size_t real_bytes, int nrhs) {
  MarchParams p{0, 0, 0, 0, nrhs, 1, 1, 0u, 0u};
  if (geo.X > kMarchMaxThreads) return p;
  int ny = 0;
  for (int d = 1; d <= geo.Y; ++d)
    if (geo.Y % d == 0 && geo.X * d <= kMarchTargetThreads &&
        march_lds_bytes(geo.X * d, real_bytes) <= kLdsBytes)
      ny = d;
  if (ny == 0 || geo.X * ny < 64) return p;
  p.ny = ny;
  p.ytiles = geo.Y / ny;
  const int n = geo.X * ny;
  const size_t lds1 = march_lds_bytes(n, real_bytes);
  // right-hand sides per workgroup (FP32 arithmetic only: two FP64 tiles exceed the
  // LDS): a divisor of nrhs that the lanes and LDS of a CU allow, preferring
  // the largest that still fills every CU in one round
  const int columns = p.ytiles * geo.Z;
  if (real_bytes == 4) {
    int best = 1;
    for (int gw = 2; gw <= kMaxMultiRhs && gw <= nrhs; ++gw) {
      if (nrhs % gw != 0 || gw * n > kMarchMultiThreads || gw * lds1 > kLdsBytes) continue;
      if (WD_MARCH_GW > 0 && gw != WD_MARCH_GW) continue;
      const int per_cu = static_cast<int>(kLdsBytes / (gw * lds1));
      const int slots = kNumCu * (per_cu < kMarchWgPerCu ? per_cu : kMarchWgPerCu);
      const int wgs = columns * (nrhs / gw);
      if (WD_MARCH_GW > 0 || (wgs <= slots && wgs * 4 >= slots * 3)) best = gw;
    }
    p.gw = best;
  }
  const int planes = columns * (nrhs / p.gw);
  // as many workgroups as fit on the chip at once (LDS and registers decide
  // how many per CU), without a second round, and at least 4 t steps per
  // workgroup so the prologue of each march stays cheap; t steps split evenly
  const int waves = (p.gw * n + 63) / 64;
  const int by_regs = (real_bytes == 8 ? kWavesPerCuFp64 : kWavesPerCuFp32) / waves;
  int per_cu = static_cast<int>(kLdsBytes / (p.gw * lds1));
  per_cu = per_cu < by_regs ? per_cu : by_regs;
  per_cu = per_cu > 1 ? per_cu : 1;
  const int slots = kNumCu * (per_cu < kMarchWgPerCu ? per_cu : kMarchWgPerCu);
  int nt = slots / planes;
  const int nt_max = geo.T / 4 > 1 ? geo.T / 4 : 1;
  nt = nt < 1 ? 1 : (nt > nt_max ? nt_max : nt);
  p.tb = (geo.T + nt - 1) / nt;
  const int nb = planes * ((geo.T + p.tb - 1) / p.tb);
  // every XCD gets one contiguous eighth of the workgroups: the right-hand
  // sides, y tiles and z planes that share links and halo slices meet in one L2
  p.group = WD_XCD_GROUP >= 0 ? WD_XCD_GROUP : (nb % kNumXcd == 0 ? nb / kNumXcd : 0);
  return p;
}

template <typename T, bool C12, int MAXT, int RB, int CGM, bool BUF>
hipError_t launch_march_t(const void* in, void* out, const void* links, const Geo& geo,
                          const Diag<typename Packed<T>::R>& diag, long stride, int g5,
                          const MarchParams& p, const CgFuse& f, hipStream_t st) {
  using SV = typename Packed<T>::S;
  using LV = typename Packed<T>::L;
  using R = typename Packed<T>::R;
  const int n = geo.X * p.ny;
  size_t lds = static_cast<size_t>(p.gw) * RB * march_lds_bytes(n, sizeof(R));
  if (CGM != kCgNone) lds += static_cast<size_t>(p.gw) * RB * kCgLds * sizeof(double);
  if (lds > kLdsBytes) return hipErrorInvalidValue;
  // raise the kernel's dynamic LDS limit once to the whole LDS of a CU
  static std::atomic<int> attr_set{0};
  if (!attr_set.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&dslash_march_kernel<T, C12, MAXT, RB, CGM, BUF>),
        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
    if (e != hipSuccess) return e;
    attr_set.store(1, std::memory_order_release);
  }
  const unsigned nb = static_cast<unsigned>((p.nrhs / (p.gw * RB)) * p.ytiles * geo.Z *
                                            ((geo.T + p.tb - 1) / p.tb));
  dslash_march_kernel<T, C12, MAXT, RB, CGM, BUF><<<nb, p.gw * n, lds, st>>>(
      static_cast<const SV*>(in), static_cast<SV*>(out), static_cast<const LV*>(links), geo, diag,
      stride, g5, p, f);
  return hipGetLastError();
}

template <typename T, bool C12, int CGM, bool BUF>
hipError_t launch_march_b(const void* in, void* out, const void* links, const Geo& geo,
                          const Diag<typename Packed<T>::R>& diag, long stride, int g5,
                          const MarchParams& p, const CgFuse& f, hipStream_t st) {
  if constexpr (sizeof(typename Packed<T>::R) == 4) {
    if (p.rb == 2)  // two right-hand sides per lane: one lane group per workgroup
      return launch_march_t<T, C12, kMarchMaxThreads, 2, CGM, BUF>(in, out, links, geo, diag, stride, g5,
                                                                  p, f, st);
    if (p.gw > 1)
      return launch_march_t<T, C12, kMarchMultiThreads, 1, CGM, BUF>(in, out, links, geo, diag, stride,
                                                                    g5, p, f, st);
  }
  return launch_march_t<T, C12, kMarchMaxThreads, 1, CGM, BUF>(in, out, links, geo, diag, stride, g5, p,
                                                              f, st);
}

// The operator reads its fields (and the plain operator also writes them)
// through buffer resources when every field is below 4 GiB and a workgroup
// holds one lane group (WD_MARCH_BUF 0 turns it off).
template <typename T, bool C12, int CGM>
hipError_t launch_march(const void* in, void* out, const void* links, const Geo& geo,
                        const Diag<typename Packed<T>::R>& diag, long stride, int g5,
                        const MarchParams& p, const CgFuse& f, hipStream_t st) {
  if (kMarchBuf && p.gw == 1 && p.link_bytes != 0 && p.spinor_bytes != 0)
    return launch_march_b<T, C12, CGM, true>(in, out, links, geo, diag, stride, g5, p, f, st);
  return launch_march_b<T, C12, CGM, false>(in, out, links, geo, diag, stride, g5, p, f, st);
}

template <typename T, bool C12>
hipError_t launch_site(const void* in, void* out, const void* links, const Geo& geo,
                       const Diag<typename Packed<T>::R>& diag, int nrhs, long stride, int g5,
                       hipStream_t st) {
  using SV = typename Packed<T>::S;
  using LV = typename Packed<T>::L;
  const unsigned nb = static_cast<unsigned>((geo.V + kDslashBlock - 1) / kDslashBlock);
  const int group = xcd_group(static_cast<int>(nb), 8);
  dslash_kernel<T, C12><<<dim3(nb, nrhs), kDslashBlock, 0, st>>>(
      static_cast<const SV*>(in), static_cast<SV*>(out), static_cast<const LV*>(links), geo, diag,
      stride, g5, group);
  return hipGetLastError();
}

// Applies a tuning choice to the default parameters.
MarchParams with_tuning(MarchParams p, const MarchTuning& t) {
  p.tb = t.tb;
  p.gw = t.gw;
  p.group = t.group;
  p.rb = t.rb;
  return p;
}

// cg: a CG iteration's fused work (the march kernel only; nullptr for a plain
// apply): cg->mode kCgNorm or kCgUpdate.
template <typename T, bool C12>
hipError_t launch_typed(const wd_gauge* g, const void* in, void* out, const Geo& geo,
                        const double* masses, int nrhs, const int* fields, int g5,
                        const MarchTuning* force, const CgFuse* cg, hipStream_t st) {
  using R = typename Packed<T>::R;
  Diag<R> diag{};
  for (int k = 0; k < nrhs; ++k) {
    diag.d[k] = static_cast<R>(4.0 + masses[k]);
    diag.idx[k] = fields ? fields[k] : k;
  }
  const long stride = spinor_units<T>(geo.V);  // 16-B elements per field
  MarchParams p = march_params(geo, sizeof(R), nrhs);
  // byte sizes for buffer-resource access, or 0 where a field reaches 4 GiB
  const unsigned long sbytes = static_cast<unsigned long>(stride) * 16;
  p.link_bytes = g->link_bytes < (1ul << 32) ? static_cast<unsigned>(g->link_bytes) : 0u;
  p.spinor_bytes = sbytes < (1ul << 32) ? static_cast<unsigned>(sbytes) : 0u;
  if (WD_DSLASH_KERNEL == 0 && p.ny > 0) {
    MarchTuning t;
    if (force != nullptr) p = with_tuning(p, *force);
    else if (tuned_lookup(g->dims, g->prec, g->c12, nrhs, &t)) p = with_tuning(p, t);
    if (cg != nullptr) {
      // whole waves per tile, a partial sum slot for every tile slice, and the
      // inputs the update reads
      if ((geo.X * p.ny) % 64 != 0 || cg->rr == nullptr ||
          static_cast<long>(cg->nslices) < static_cast<long>(geo.T) * geo.Z * p.ytiles)
        return hipErrorInvalidValue;
      if (cg->mode == kCgUpdate && (cg->r == nullptr || cg->pap == nullptr || cg->npap < 1 || cg->scal == nullptr))
        return hipErrorInvalidValue;
      if (cg->mode == kCgNorm)
        return launch_march<T, C12, kCgNorm>(in, out, g->links, geo, diag, stride, g5, p, *cg, st);
      if constexpr (sizeof(R) == 4) {  // the update is fused with FP32 arithmetic only
        if (cg->mode == kCgUpdate)
          return launch_march<T, C12, kCgUpdate>(in, nullptr, g->links, geo, diag, stride, g5, p, *cg,
                                                 st);
      }
      return hipErrorInvalidValue;
    }
    return launch_march<T, C12, kCgNone>(in, out, g->links, geo, diag, stride, g5, p, CgFuse{}, st);
  }
  if (cg != nullptr) return hipErrorInvalidValue;
  return launch_site<T, C12>(in, out, g->links, geo, diag, nrhs, stride, g5, st);
}

template <typename T>
hipError_t launch_prec(const wd_gauge* g, const void* in, void* out, const Geo& geo,
                       const double* masses, int nrhs, const int* fields, int g5,
                       const MarchTuning* force, const CgFuse* cg, hipStream_t st) {
  return g->c12 ? launch_typed<T, true>(g, in, out, geo, masses, nrhs, fields, g5, force, cg, st)
                : launch_typed<T, false>(g, in, out, geo, masses, nrhs, fields, g5, force, cg, st);
}

hipError_t launch_any(const wd_gauge* g, const double* masses, int nrhs, const int* fields,
                      const void* in, void* out, int flags, const MarchTuning* force,
                      const CgFuse* cg, hipStream_t st) {
  if (nrhs < 1) return hipSuccess;
  if (nrhs > kMaxMultiRhs) return hipErrorInvalidValue;
  const Geo geo = make_geo(g->dims);
  const int g5 = (flags & WD_FLAG_GAMMA5) ? 1 : 0;
  switch (g->prec) {
    case WD_FP64: return launch_prec<double>(g, in, out, geo, masses, nrhs, fields, g5, force, cg, st);
    case WD_FP32: return launch_prec<float>(g, in, out, geo, masses, nrhs, fields, g5, force, cg, st);
    case WD_FP16:
      return launch_prec<_Float16>(g, in, out, geo, masses, nrhs, fields, g5, force, cg, st);
    default: return hipErrorInvalidValue;
  }
}

size_t real_bytes_of(int prec) { return prec == WD_FP64 ? 8 : 4; }

}  // namespace

hipError_t launch_dslash_multi(const wd_gauge* g, const double* masses, int nrhs, const int* fields,
                               const void* in, void* out, int flags, hipStream_t st) {
  return launch_any(g, masses, nrhs, fields, in, out, flags, nullptr, nullptr, st);
}

// (With FP64 vectors the engine fuses only the norm: the FP64 kernel holds one
// wave per SIMD, and the x, r update in its epilogue cost more than the
// separate update kernel it saves: 24^4 FP64 CG 46.5 -> 47.9 ms per solve.)
int cg_fuse_slices(const int32_t dims[4], int prec) {
  if (WD_DSLASH_KERNEL != 0) return 0;
  const Geo geo = make_geo(dims);
  const MarchParams p = march_params(geo, real_bytes_of(prec), 1);
  if (p.ny == 0 || (geo.X * p.ny) % 64 != 0) return 0;
  const long n = static_cast<long>(geo.T) * geo.Z * p.ytiles;
  return n <= 0x7fffffffL ? static_cast<int>(n) : 0;
}

hipError_t launch_dslash_cg(const wd_gauge* g, const double* masses, int nrhs, const int* fields,
                            const void* in, void* out, const CgFuse& f, hipStream_t st) {
  return launch_any(g, masses, nrhs, fields, in, out, WD_FLAG_GAMMA5, nullptr, &f, st);
}

hipError_t launch_dslash(const wd_gauge* g, double mass, const void* in, void* out, int flags,
                         hipStream_t st) {
  return launch_dslash_multi(g, &mass, 1, nullptr, in, out, flags, st);
}

hipError_t launch_dslash_tuned(const wd_gauge* g, const double* masses, int nrhs, const void* in,
                               void* out, int flags, const MarchTuning& t, hipStream_t st) {
  return launch_any(g, masses, nrhs, nullptr, in, out, flags, &t, nullptr, st);
}

bool march_default(const int32_t dims[4], int prec, int nrhs, MarchTuning* t) {
  if (WD_DSLASH_KERNEL != 0) return false;
  const MarchParams p = march_params(make_geo(dims), real_bytes_of(prec), nrhs);
  if (p.ny == 0) return false;
  *t = MarchTuning{p.tb, p.gw, p.group, p.rb};
  return true;
}

bool march_tuning_valid(const int32_t dims[4], int prec, int nrhs, const MarchTuning& t) {
  const Geo geo = make_geo(dims);
  const size_t real = real_bytes_of(prec);
  const MarchParams p = march_params(geo, real, nrhs);
  if (WD_DSLASH_KERNEL != 0 || p.ny == 0 || nrhs < 1 || nrhs > kMaxMultiRhs) return false;
  if (t.tb < 1 || t.tb > geo.T || t.group < 0) return false;
  if (t.rb != 1 && t.rb != 2) return false;
  if (t.gw < 1 || nrhs % (t.gw * t.rb) != 0) return false;
  const int n = geo.X * p.ny;
  if (t.gw > 1 || t.rb > 1) {  // several right-hand sides per workgroup: FP32 arithmetic only
    if (real != 4 || t.gw * n > kMarchMultiThreads) return false;
  }
  if (t.rb > 1 && t.gw != 1) return false;  // two per lane: one lane group per workgroup
  if (static_cast<size_t>(t.gw) * t.rb * march_lds_bytes(n, real) > kLdsBytes) return false;
  const long nb = static_cast<long>(nrhs / (t.gw * t.rb)) * p.ytiles * geo.Z * ((geo.T + t.tb - 1) / t.tb);
  return nb >= 1 && nb <= 0x7fffffffL;
}

void march_candidates(const int32_t dims[4], int prec, int nrhs, MarchTuning* out, int* n, int cap) {
  *n = 0;
  MarchTuning d;
  if (!march_default(dims, prec, nrhs, &d) || cap < 1) return;
  out[(*n)++] = d;
  const Geo geo = make_geo(dims);
  const MarchParams p = march_params(geo, real_bytes_of(prec), nrhs);
  // t steps per workgroup: the distinct ceil(T / nt) for nt workgroups along t
  int tbs[64];
  int ntb = 0;
  for (int nt = 1; nt <= geo.T && ntb < 64; ++nt) {
    const int tb = (geo.T + nt - 1) / nt;
    if (tb < 2 && nt > 1) break;
    if (ntb == 0 || tbs[ntb - 1] != tb) tbs[ntb++] = tb;
  }
  for (int rb = 1; rb <= 2; ++rb)
    for (int gw = 1; gw <= nrhs; ++gw) {
      if (nrhs % (gw * rb) != 0) continue;
      for (int i = 0; i < ntb; ++i) {
        const long nb =
            static_cast<long>(nrhs / (gw * rb)) * p.ytiles * geo.Z * ((geo.T + tbs[i] - 1) / tbs[i]);
        const int groups[2] = {0, nb % kNumXcd == 0 ? static_cast<int>(nb / kNumXcd) : 0};
        for (int j = 0; j < (groups[1] > 0 ? 2 : 1); ++j) {
          const MarchTuning t{tbs[i], gw, groups[j], rb};
          if (!march_tuning_valid(dims, prec, nrhs, t)) continue;
          if (t.tb == d.tb && t.gw == d.gw && t.group == d.group && t.rb == d.rb) continue;
          if (*n < cap) out[(*n)++] = t;
        }
      }
    }
}

}  // namespace wd
