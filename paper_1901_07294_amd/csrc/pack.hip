// Conversion between the canonical complex128 layouts of the C ABI and the
// packed structure-of-arrays layouts of fields.h (once per field, outside the
// operator application).
#include "fields.h"
#include "wd_internal.h"

namespace wd {
namespace {

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
  const double2* src = canon + i * 12;
  typename Packed<T>::S* d = dst + k * spinor_units<T>(V);
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

template <typename T>
__global__ __launch_bounds__(kBlock) void unpack_spinor_kernel(
    const typename Packed<T>::S* __restrict__ src, double2* __restrict__ canon, long V, long total) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= total) return;
  const long k = i / V;
  const long s = i - k * V;
  double2* d = canon + i * 12;
  const typename Packed<T>::S* p = src + k * spinor_units<T>(V);
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

// FP64 link entry -> binary16, rounded once to nearest even.
__device__ __forceinline__ _Float16 to_half(double v) { return static_cast<_Float16>(v); }

// One thread per (site, direction). Canonical links of a site are 4 x 9
// consecutive complex128 values.
template <typename T, bool C12>
__global__ __launch_bounds__(kBlock) void pack_gauge_kernel(const double2* __restrict__ canon,
                                                            void* __restrict__ dst, long V) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= 4 * V) return;
  const long s = i >> 2;
  const int mu = static_cast<int>(i & 3);
  const double2* src = canon + i * 9;
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
