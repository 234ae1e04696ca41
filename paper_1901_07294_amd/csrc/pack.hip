// Conversion between the canonical complex128 layouts of the C ABI and the
// packed structure-of-arrays layouts of fields.h (once per field, outside the
// operator application).
#include "blas.h"
#include "fields.h"
#include "wd_internal.h"

namespace wd {
namespace {

// FP64 link entry -> binary16, rounded once to nearest even.
__device__ __forceinline__ _Float16 to_half(double v) { return static_cast<_Float16>(v); }


// Site s of a packed spinor field d (storage T) from its 12 canonical
// complex128 values.
template <typename T>
__device__ __forceinline__ void pack_site(const double2* __restrict__ src, typename Packed<T>::S* __restrict__ d,
                                          long s, long V) {
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int c = 0; c < 12; ++c) d[pidx(s, c, 12, V)] = src[c];
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const double2 a = src[2 * j];
      const double2 b = src[2 * j + 1];
      d[pidx(s, j, 6, V)] = make_float4(static_cast<float>(a.x), static_cast<float>(a.y),
                                        static_cast<float>(b.x), static_cast<float>(b.y));
    }
  } else {
    cx<float> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = {static_cast<float>(src[c].x), static_cast<float>(src[c].y)};
    store_spinor(d, V, static_cast<int>(s), v);
  }
}

// The 12 canonical complex128 values of site s of a packed spinor field p.
template <typename T>
__device__ __forceinline__ void unpack_site(const typename Packed<T>::S* __restrict__ p,
                                            double2* __restrict__ d, long s, long V) {
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int c = 0; c < 12; ++c) d[c] = p[pidx(s, c, 12, V)];
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const float4 t = p[pidx(s, j, 6, V)];
      d[2 * j] = make_double2(t.x, t.y);
      d[2 * j + 1] = make_double2(t.z, t.w);
    }
  } else {
    cx<float> v[12];
    load_spinor(p, V, static_cast<int>(s), v);  // the values the operator reads
#pragma unroll
    for (int c = 0; c < 12; ++c) d[c] = make_double2(v[c].re, v[c].im);
  }
}

// One thread per (right-hand side, site). The canonical spinor of a site is 12
// consecutive complex128 values (192 B); the packed planes are written
// coalesced. T is the storage type.
template <typename T>
__global__ __launch_bounds__(kBlock) void pack_spinor_kernel(const double2* __restrict__ canon,
                                                             typename Packed<T>::S* __restrict__ dst,
                                                             long V, long total) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= total) return;
  const long k = i / V;
  const long s = i - k * V;
  pack_site<T>(canon + i * 12, dst + k * spinor_units<T>(V), s, V);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void unpack_spinor_kernel(
    const typename Packed<T>::S* __restrict__ src, double2* __restrict__ canon, long V, long total) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= total) return;
  const long k = i / V;
  const long s = i - k * V;
  unpack_site<T>(src + k * spinor_units<T>(V), canon + i * 12, s, V);
}

// Link mu of site s of a packed gauge field dst (storage T) from its 9
// canonical complex128 entries.
template <typename T, bool C12>
__device__ __forceinline__ void pack_link(const double2* __restrict__ src, void* __restrict__ dst, long s,
                                          int mu, long V) {
  if constexpr (sizeof(T) == 8) {
    constexpr int n = C12 ? 6 : 9;
    double2* d = static_cast<double2*>(dst);
#pragma unroll
    for (int k = 0; k < n; ++k) d[pidx(s, mu * n + k, 4 * n, V)] = src[k];
  } else if constexpr (sizeof(T) == 4 && C12) {
    float4* d = static_cast<float4*>(dst);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double2 a = src[2 * j];
      const double2 b = src[2 * j + 1];
      d[pidx(s, mu * 3 + j, 12, V)] = make_float4(static_cast<float>(a.x), static_cast<float>(a.y),
                                                  static_cast<float>(b.x), static_cast<float>(b.y));
    }
  } else if constexpr (sizeof(T) == 4) {
    float2* d = static_cast<float2*>(dst);
#pragma unroll
    for (int k = 0; k < 9; ++k)
      d[pidx(s, mu * 9 + k, 36, V)] = make_float2(static_cast<float>(src[k].x), static_cast<float>(src[k].y));
  } else if constexpr (C12) {
    h4* d = static_cast<h4*>(dst);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double2 a = src[2 * j];
      const double2 b = src[2 * j + 1];
      d[pidx<kHalfBlock>(s, mu * 3 + j, 12, V)] = h4{to_half(a.x), to_half(a.y), to_half(b.x), to_half(b.y)};
    }
  } else {
    h2* d = static_cast<h2*>(dst);
#pragma unroll
    for (int k = 0; k < 9; ++k)
      d[pidx<kHalfBlock>(s, mu * 9 + k, 36, V)] = h2{to_half(src[k].x), to_half(src[k].y)};
  }
}

// One thread per (site, direction). Canonical links of a site are 4 x 9
// consecutive complex128 values.
template <typename T, bool C12>
__global__ __launch_bounds__(kBlock) void pack_gauge_kernel(const double2* __restrict__ canon,
                                                            void* __restrict__ dst, long V) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= 4 * V) return;
  pack_link<T, C12>(canon + i * 9, dst, i >> 2, static_cast<int>(i & 3), V);
}

// ----------------------------------------------------------- even-odd layout
//
// A field split by site parity (x+y+z+t) mod 2 keeps the sites of each parity
// as a packed field of Vh = V/2 sites (the layouts above), in half-site order
// h = xh + (X/2) * (y + Y * (z + Z * t)) with x = 2 xh + ((y + z + t + parity) & 1).

// Canonical site index of half site h of parity q.
__device__ __forceinline__ long eo_site(const EoGeo& g, long h, int q) {
  const long xh = h % g.Xh;
  const long r = h / g.Xh;  // y + Y (z + Z t)
  const int y = static_cast<int>(r % g.Y);
  const int z = static_cast<int>((r / g.Y) % g.Z);
  const int t = static_cast<int>(r / (static_cast<long>(g.Y) * g.Z));
  return 2 * xh + ((y + z + t + q) & 1) + static_cast<long>(g.X) * r;
}

// One thread per (parity, half site, direction): both parities' links, each
// a packed gauge field of Vh sites, even first, `half` bytes apart.
template <typename T, bool C12>
__global__ __launch_bounds__(kBlock) void pack_gauge_eo_kernel(const double2* __restrict__ canon,
                                                               char* __restrict__ dst, EoGeo g,
                                                               size_t half) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= 8L * g.Vh) return;
  const int q = static_cast<int>(i / (4L * g.Vh));
  const long j = i - q * 4L * g.Vh;
  const long h = j >> 2;
  const int mu = static_cast<int>(j & 3);
  pack_link<T, C12>(canon + (eo_site(g, h, q) * 4 + mu) * 9, dst + q * half, h, mu, g.Vh);
}

// Sites of parity q of canonical spinors -> packed half fields, and back (the
// sites of the other parity of the canonical array are set to zero).
template <typename T>
__global__ __launch_bounds__(kBlock) void pack_spinor_eo_kernel(const double2* __restrict__ canon,
                                                                typename Packed<T>::S* __restrict__ dst,
                                                                EoGeo g, int q, long total) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= total) return;
  const long k = i / g.Vh;
  const long h = i - k * g.Vh;
  const long V = 2L * g.Vh;
  pack_site<T>(canon + (k * V + eo_site(g, h, q)) * 12, dst + k * spinor_units<T>(g.Vh), h, g.Vh);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void unpack_spinor_eo_kernel(
    const typename Packed<T>::S* __restrict__ src, double2* __restrict__ canon, EoGeo g, int q, long total) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= total) return;
  const long k = i / g.Vh;
  const long h = i - k * g.Vh;
  const long V = 2L * g.Vh;
  double2* site = canon + (k * V + eo_site(g, h, q)) * 12;
  unpack_site<T>(src + k * spinor_units<T>(g.Vh), site, h, g.Vh);
  double2* other = canon + (k * V + eo_site(g, h, q ^ 1)) * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) other[c] = make_double2(0.0, 0.0);
}

// Packed FP64 full-lattice fields <-> their two packed FP64 half fields (even,
// odd), one thread per (right-hand side, parity, half site). Field k of each
// is at k * (its 16-byte elements per field).
__global__ __launch_bounds__(kBlock) void split_eo_kernel(const double2* __restrict__ full,
                                                          double2* __restrict__ even,
                                                          double2* __restrict__ odd, EoGeo g,
                                                          RhsSet set, bool merge) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= 2L * g.Vh) return;
  const int q = static_cast<int>(i / g.Vh);
  const long h = i - q * g.Vh;
  const long V = 2L * g.Vh;
  const long k = set.idx[blockIdx.y];
  const long s = eo_site(g, h, q);
  const double2* f = full + k * spinor_units<double>(V);
  double2* p = (q == 0 ? even : odd) + k * spinor_units<double>(g.Vh);
  if (merge) {
    double2* fo = const_cast<double2*>(f);
#pragma unroll
    for (int c = 0; c < 12; ++c) fo[pidx(s, c, 12, V)] = p[pidx(h, c, 12, g.Vh)];
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) p[pidx(h, c, 12, g.Vh)] = f[pidx(s, c, 12, V)];
  }
}

unsigned blocks_for(long n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

template <typename T>
void pack_gauge_t(const double2* src, void* dst, long V, int c12, hipStream_t s) {
  const unsigned nb = blocks_for(4 * V);
  if (c12) pack_gauge_kernel<T, true><<<nb, kBlock, 0, s>>>(src, dst, V);
  else pack_gauge_kernel<T, false><<<nb, kBlock, 0, s>>>(src, dst, V);
}

template <typename T>
void pack_spinor_t(const double2* src, void* dst, long V, long total, hipStream_t s) {
  pack_spinor_kernel<T><<<blocks_for(total), kBlock, 0, s>>>(
      src, static_cast<typename Packed<T>::S*>(dst), V, total);
}

template <typename T>
void unpack_spinor_t(const void* src, double2* dst, long V, long total, hipStream_t s) {
  unpack_spinor_kernel<T><<<blocks_for(total), kBlock, 0, s>>>(
      static_cast<const typename Packed<T>::S*>(src), dst, V, total);
}

}  // namespace

hipError_t launch_pack_gauge(const void* canon, void* dst, const Geo& geo, int prec, int c12,
                             hipStream_t s) {
  const auto* src = static_cast<const double2*>(canon);
  switch (prec) {
    case WD_FP64: pack_gauge_t<double>(src, dst, geo.V, c12, s); break;
    case WD_FP32: pack_gauge_t<float>(src, dst, geo.V, c12, s); break;
    case WD_FP16: pack_gauge_t<_Float16>(src, dst, geo.V, c12, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pack_spinor(const void* canon, void* dst, const Geo& geo, int prec, int nrhs,
                              hipStream_t s) {
  const long V = geo.V;
  const long total = V * nrhs;
  if (total == 0) return hipSuccess;
  const auto* src = static_cast<const double2*>(canon);
  switch (prec) {
    case WD_FP64: pack_spinor_t<double>(src, dst, V, total, s); break;
    case WD_FP32: pack_spinor_t<float>(src, dst, V, total, s); break;
    case WD_FP16: pack_spinor_t<_Float16>(src, dst, V, total, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t eo_gauge_half_bytes(long Vh, int prec, int c12) {
  return static_cast<size_t>(packed_sites(Vh)) * gauge_site_bytes(prec, c12);
}

hipError_t launch_pack_gauge_eo(const void* canon, void* dst, const EoGeo& g, int prec, int c12,
                                hipStream_t s) {
  const auto* src = static_cast<const double2*>(canon);
  char* d = static_cast<char*>(dst);
  const size_t half = eo_gauge_half_bytes(g.Vh, prec, c12);
  const unsigned nb = blocks_for(8L * g.Vh);
#define WD_EO_PACK(T)                                                                     \
  if (c12) pack_gauge_eo_kernel<T, true><<<nb, kBlock, 0, s>>>(src, d, g, half);          \
  else pack_gauge_eo_kernel<T, false><<<nb, kBlock, 0, s>>>(src, d, g, half);
  switch (prec) {
    case WD_FP64: WD_EO_PACK(double) break;
    case WD_FP32: WD_EO_PACK(float) break;
    case WD_FP16: WD_EO_PACK(_Float16) break;
    default: return hipErrorInvalidValue;
  }
#undef WD_EO_PACK
  return hipGetLastError();
}

hipError_t launch_spinor_eo(const void* src, void* dst, const EoGeo& g, int prec, int parity, int nrhs,
                            bool import, hipStream_t s) {
  const long total = g.Vh * nrhs;
  if (total == 0) return hipSuccess;
  const unsigned nb = blocks_for(total);
#define WD_EO_SPINOR(T)                                                                              \
  if (import)                                                                                        \
    pack_spinor_eo_kernel<T><<<nb, kBlock, 0, s>>>(static_cast<const double2*>(src),                 \
                                                   static_cast<Packed<T>::S*>(dst), g, parity, total); \
  else                                                                                               \
    unpack_spinor_eo_kernel<T><<<nb, kBlock, 0, s>>>(static_cast<const Packed<T>::S*>(src),          \
                                                     static_cast<double2*>(dst), g, parity, total);
  switch (prec) {
    case WD_FP64: WD_EO_SPINOR(double) break;
    case WD_FP32: WD_EO_SPINOR(float) break;
    case WD_FP16: WD_EO_SPINOR(_Float16) break;
    default: return hipErrorInvalidValue;
  }
#undef WD_EO_SPINOR
  return hipGetLastError();
}

hipError_t launch_split_eo(const void* full, void* even, void* odd, const EoGeo& g, const RhsSet& set,
                           bool merge, hipStream_t s) {
  if (set.n == 0) return hipSuccess;
  split_eo_kernel<<<dim3(blocks_for(2L * g.Vh), set.n), kBlock, 0, s>>>(
      static_cast<const double2*>(full), static_cast<double2*>(even), static_cast<double2*>(odd), g, set,
      merge);
  return hipGetLastError();
}

hipError_t launch_unpack_spinor(const void* src, void* canon, const Geo& geo, int prec, int nrhs,
                                hipStream_t s) {
  const long V = geo.V;
  const long total = V * nrhs;
  if (total == 0) return hipSuccess;
  auto* dst = static_cast<double2*>(canon);
  switch (prec) {
    case WD_FP64: unpack_spinor_t<double>(src, dst, V, total, s); break;
    case WD_FP32: unpack_spinor_t<float>(src, dst, V, total, s); break;
    case WD_FP16: unpack_spinor_t<_Float16>(src, dst, V, total, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wd
