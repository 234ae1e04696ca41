// Hops between the two parities of an even-odd split lattice, for the Schur
// complement of the odd sites (eo.h), and gamma5 on FP64 fields.
//
// One lane per output half site. The eight neighbours of an output site all
// have the other parity: the x neighbours sit in the same half row at x
// half-index xh or xh +/- 1 (which one depends on the row's parity offset),
// the y, z and t neighbours at the same half index in the neighbouring half
// rows, planes and slices. The forward hop of direction mu uses the output
// site's own link (this parity's links), the backward hop the link of the
// neighbour it comes from (the other parity's links, at the neighbour's index).
// Over both parities every link is read once per application of H_{p,1-p},
// as in the full operator.
#include "eo.h"
#include "stencil.h"

namespace wd {
namespace {

constexpr int kEoBlock = 256;

// Workgroup -> run of kEoBlock half sites: consecutive workgroups go to the 8
// XCDs in turn; when the grid divides evenly, every XCD gets one contiguous
// eighth of the field instead, so that the t and z neighbours a workgroup
// reads were loaded into the same L2 by workgroups of its own XCD.
__device__ __forceinline__ int eo_tile(int contiguous) {
  const int b = blockIdx.x;
  if (!contiguous) return b;
  const int per = gridDim.x / kNumXcd;
  return (b % kNumXcd) * per + b / kNumXcd;
}

template <typename R>
struct EoCoef {
  R d[kMaxRhs];
  R c[kMaxRhs];
  int idx[kMaxRhs];
};

template <typename T, bool C12>
__global__ __launch_bounds__(kEoBlock) void eo_hop_kernel(
    const typename Packed<T>::S* __restrict__ in_all, const typename Packed<T>::S* __restrict__ w_all,
    typename Packed<T>::S* __restrict__ out_all, const typename Packed<T>::L* __restrict__ lp,
    const typename Packed<T>::L* __restrict__ lq, EoGeo g, int p, EoCoef<typename Packed<T>::R> cf,
    long stride, int g5, int contiguous) {
  using R = typename Packed<T>::R;
  const long hl = static_cast<long>(eo_tile(contiguous)) * kEoBlock + threadIdx.x;
  if (hl >= g.Vh) return;
  const int h = static_cast<int>(hl);
  const long Vh = g.Vh;
  const int slot = blockIdx.y;
  const long k = cf.idx[slot];
  const typename Packed<T>::S* in = in_all + k * stride;
  typename Packed<T>::S* out = out_all + k * stride;

  const int xh = h % g.Xh;
  const int r = h / g.Xh;
  const int y = r % g.Y;
  const int z = (r / g.Y) % g.Z;
  const int t = r / (g.Y * g.Z);
  const int o = (y + z + t + p) & 1;  // this row's x offset: x = 2 xh + o
  const int row = h - xh;
  // x + 1 is 2 xh + o + 1: half index xh when o = 0, xh + 1 (wrapping) when o = 1;
  // x - 1 is 2 xh + o - 1: xh - 1 (wrapping) when o = 0, xh when o = 1
  const int xp = row + (o ? (xh + 1 == g.Xh ? 0 : xh + 1) : xh);
  const int xm = row + (o ? xh : (xh == 0 ? g.Xh - 1 : xh - 1));
  const int sy = g.Xh, sz = g.Xh * g.Y, st = sz * g.Z;
  const int yp = y + 1 == g.Y ? h - (g.Y - 1) * sy : h + sy;
  const int ym = y == 0 ? h + (g.Y - 1) * sy : h - sy;
  const int zp = z + 1 == g.Z ? h - (g.Z - 1) * sz : h + sz;
  const int zm = z == 0 ? h + (g.Z - 1) * sz : h - sz;
  const int tp = t + 1 == g.T ? h - (g.T - 1) * st : h + st;
  const int tm = t == 0 ? h + (g.T - 1) * st : h - st;

  cx<R> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};
  hop<0, -1, C12>(in, lp, Vh, xp, h, acc);
  hop<0, +1, C12>(in, lq, Vh, xm, xm, acc);
  hop<1, -1, C12>(in, lp, Vh, yp, h, acc);
  hop<1, +1, C12>(in, lq, Vh, ym, ym, acc);
  hop<2, -1, C12>(in, lp, Vh, zp, h, acc);
  hop<2, +1, C12>(in, lq, Vh, zm, zm, acc);
  hop<3, -1, C12>(in, lp, Vh, tp, h, acc);
  hop<3, +1, C12>(in, lq, Vh, tm, tm, acc);

  const R d = cf.d[slot], c = cf.c[slot];
  cx<R> res[12];
  if (w_all != nullptr) {
    cx<R> wv[12];
    load_spinor(w_all + k * stride, Vh, h, wv);
#pragma unroll
    for (int i = 0; i < 12; ++i) res[i] = {fmar(d, wv[i].re, c * acc[i].re), fmar(d, wv[i].im, c * acc[i].im)};
  } else {
#pragma unroll
    for (int i = 0; i < 12; ++i) res[i] = {c * acc[i].re, c * acc[i].im};
  }
  if (g5) {
#pragma unroll
    for (int i = 6; i < 12; ++i) res[i] = -res[i];
  }
  store_spinor(out, Vh, h, res);
}

// dst = gamma5 src on FP64 packed fields: plane 3 * spin + colour, spins 2
// and 3 negated.
__global__ __launch_bounds__(256) void gamma5_kernel(double2* __restrict__ dst, const double2* __restrict__ src,
                                                     long n, RhsSet set) {
  const long k = set.idx[blockIdx.y];
  for (long e = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * 256) {
    const int plane = static_cast<int>((e / kLayoutBlock) % 12);
    double2 v = src[k * n + e];
    if (plane >= 6) v = make_double2(-v.x, -v.y);
    dst[k * n + e] = v;
  }
}

template <typename T, bool C12>
hipError_t launch_hop_t(const wd_gauge* g, int p, const void* in, const void* w, void* out, const RhsSet& set,
                        const double* d, const double* c, int g5, hipStream_t s) {
  using S = typename Packed<T>::S;
  using L = typename Packed<T>::L;
  using R = typename Packed<T>::R;
  const EoGeo geo = make_eo_geo(g->dims);
  EoCoef<R> cf{};
  for (int i = 0; i < set.n; ++i) {
    cf.d[i] = static_cast<R>(d[i]);
    cf.c[i] = static_cast<R>(c[i]);
    cf.idx[i] = set.idx[i];
  }
  const size_t half = eo_gauge_half_bytes(geo.Vh, g->prec, g->c12);
  const char* links = static_cast<const char*>(g->links);
  const L* lp = reinterpret_cast<const L*>(links + p * half);        // this parity: forward hops
  const L* lq = reinterpret_cast<const L*>(links + (p ^ 1) * half);  // the other: backward hops
  const unsigned nb = static_cast<unsigned>((geo.Vh + kEoBlock - 1) / kEoBlock);
  const int contiguous = nb % kNumXcd == 0 ? 1 : 0;
  eo_hop_kernel<T, C12><<<dim3(nb, set.n), kEoBlock, 0, s>>>(
      static_cast<const S*>(in), static_cast<const S*>(w), static_cast<S*>(out), lp, lq, geo, p, cf,
      spinor_units<T>(geo.Vh), g5, contiguous);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_hop_prec(const wd_gauge* g, int p, const void* in, const void* w, void* out,
                           const RhsSet& set, const double* d, const double* c, int g5, hipStream_t s) {
  return g->c12 ? launch_hop_t<T, true>(g, p, in, w, out, set, d, c, g5, s)
                : launch_hop_t<T, false>(g, p, in, w, out, set, d, c, g5, s);
}

}  // namespace

hipError_t launch_eo_hop(const wd_gauge* g, int parity, const void* in, const void* w, void* out,
                         const RhsSet& set, const double* d, const double* c, int g5, hipStream_t s) {
  if (set.n < 1) return hipSuccess;
  if (set.n > kMaxRhs || !g->eo || (parity != 0 && parity != 1)) return hipErrorInvalidValue;
  switch (g->prec) {
    case WD_FP64: return launch_hop_prec<double>(g, parity, in, w, out, set, d, c, g5, s);
    case WD_FP32: return launch_hop_prec<float>(g, parity, in, w, out, set, d, c, g5, s);
    case WD_FP16: return launch_hop_prec<_Float16>(g, parity, in, w, out, set, d, c, g5, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_schur_q(const wd_gauge* g, const double* masses, const RhsSet& set, const void* in,
                          void* tmp, void* out, hipStream_t s) {
  double d[kMaxRhs], c[kMaxRhs];
  for (int i = 0; i < set.n; ++i) {
    d[i] = 0.0;
    c[i] = -0.5;
  }
  hipError_t e = launch_eo_hop(g, 0, in, nullptr, tmp, set, d, c, 0, s);
  if (e != hipSuccess) return e;
  for (int i = 0; i < set.n; ++i) {
    const double a = 4.0 + masses[i];
    d[i] = a;
    c[i] = 1.0 / (2.0 * a);
  }
  return launch_eo_hop(g, 1, tmp, in, out, set, d, c, 1, s);
}

hipError_t blas_gamma5(void* dst, const void* src, long n, const RhsSet& set, hipStream_t st) {
  if (set.n == 0) return hipSuccess;
  long nb = (n + 1023) / 1024;
  nb = nb < 1 ? 1 : (nb > 4096 ? 4096 : nb);
  gamma5_kernel<<<dim3(static_cast<unsigned>(nb), set.n), 256, 0, st>>>(
      static_cast<double2*>(dst), static_cast<const double2*>(src), n, set);
  return hipGetLastError();
}

}  // namespace wd
