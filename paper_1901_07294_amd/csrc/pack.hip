// Conversion between the canonical complex128 layouts of the C ABI and the
// packed structure-of-arrays layouts of fields.h (once per field, outside the
// operator application).
#include "fields.h"
#include "wd_internal.h"

namespace wd {
namespace {

// One thread per (right-hand side, site). The canonical spinor of a site is 12
// consecutive complex128 values (192 B); the packed planes are written
// coalesced.
template <typename R>
__global__ __launch_bounds__(kBlock) void pack_spinor_kernel(const double2* __restrict__ canon,
                                                             typename Packed<R>::S* __restrict__ dst,
                                                             long V, long total) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= total) return;
  const long k = i / V;
  const long s = i - k * V;
  const long PV = packed_sites(V);
  const double2* src = canon + i * 12;
  if constexpr (sizeof(R) == 8) {
    double2* d = dst + k * 12 * PV;
#pragma unroll
    for (int c = 0; c < 12; ++c) d[pidx(s, c, 12, V)] = src[c];
  } else {
    float4* d = dst + k * 6 * PV;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const double2 a = src[2 * j];
      const double2 b = src[2 * j + 1];
      d[pidx(s, j, 6, V)] = make_float4(static_cast<float>(a.x), static_cast<float>(a.y),
                                 static_cast<float>(b.x), static_cast<float>(b.y));
    }
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void unpack_spinor_kernel(
    const typename Packed<R>::S* __restrict__ src, double2* __restrict__ canon, long V, long total) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= total) return;
  const long k = i / V;
  const long s = i - k * V;
  const long PV = packed_sites(V);
  double2* d = canon + i * 12;
  if constexpr (sizeof(R) == 8) {
    const double2* p = src + k * 12 * PV;
#pragma unroll
    for (int c = 0; c < 12; ++c) d[c] = p[pidx(s, c, 12, V)];
  } else {
    const float4* p = src + k * 6 * PV;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const float4 t = p[pidx(s, j, 6, V)];
      d[2 * j] = make_double2(t.x, t.y);
      d[2 * j + 1] = make_double2(t.z, t.w);
    }
  }
}

// One thread per (site, direction). Canonical links of a site are 4 x 9
// consecutive complex128 values.
template <typename R, bool C12>
__global__ __launch_bounds__(kBlock) void pack_gauge_kernel(const double2* __restrict__ canon,
                                                            void* __restrict__ dst, long V) {
  const long i = static_cast<long>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= 4 * V) return;
  const long s = i >> 2;
  const int mu = static_cast<int>(i & 3);
  const double2* src = canon + i * 9;
  if constexpr (sizeof(R) == 8) {
    constexpr int n = C12 ? 6 : 9;
    double2* d = static_cast<double2*>(dst);
#pragma unroll
    for (int k = 0; k < n; ++k) d[pidx(s, mu * n + k, 4 * n, V)] = src[k];
  } else if constexpr (C12) {
    float4* d = static_cast<float4*>(dst);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double2 a = src[2 * j];
      const double2 b = src[2 * j + 1];
      d[pidx(s, mu * 3 + j, 12, V)] = make_float4(static_cast<float>(a.x), static_cast<float>(a.y),
                                            static_cast<float>(b.x), static_cast<float>(b.y));
    }
  } else {
    float2* d = static_cast<float2*>(dst);
#pragma unroll
    for (int k = 0; k < 9; ++k)
      d[pidx(s, mu * 9 + k, 36, V)] = make_float2(static_cast<float>(src[k].x), static_cast<float>(src[k].y));
  }
}

unsigned blocks_for(long n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_pack_gauge(const void* canon, void* dst, const Geo& geo, int prec, int c12,
                             hipStream_t s) {
  const long V = geo.V;
  const auto* src = static_cast<const double2*>(canon);
  const unsigned nb = blocks_for(4 * V);
  if (prec == WD_FP64) {
    if (c12) pack_gauge_kernel<double, true><<<nb, kBlock, 0, s>>>(src, dst, V);
    else pack_gauge_kernel<double, false><<<nb, kBlock, 0, s>>>(src, dst, V);
  } else {
    if (c12) pack_gauge_kernel<float, true><<<nb, kBlock, 0, s>>>(src, dst, V);
    else pack_gauge_kernel<float, false><<<nb, kBlock, 0, s>>>(src, dst, V);
  }
  return hipGetLastError();
}

hipError_t launch_pack_spinor(const void* canon, void* dst, const Geo& geo, int prec, int nrhs,
                              hipStream_t s) {
  const long V = geo.V;
  const long total = V * nrhs;
  if (total == 0) return hipSuccess;
  const auto* src = static_cast<const double2*>(canon);
  if (prec == WD_FP64)
    pack_spinor_kernel<double><<<blocks_for(total), kBlock, 0, s>>>(src, static_cast<double2*>(dst), V, total);
  else
    pack_spinor_kernel<float><<<blocks_for(total), kBlock, 0, s>>>(src, static_cast<float4*>(dst), V, total);
  return hipGetLastError();
}

hipError_t launch_unpack_spinor(const void* src, void* canon, const Geo& geo, int prec, int nrhs,
                                hipStream_t s) {
  const long V = geo.V;
  const long total = V * nrhs;
  if (total == 0) return hipSuccess;
  auto* dst = static_cast<double2*>(canon);
  if (prec == WD_FP64)
    unpack_spinor_kernel<double><<<blocks_for(total), kBlock, 0, s>>>(static_cast<const double2*>(src), dst, V, total);
  else
    unpack_spinor_kernel<float><<<blocks_for(total), kBlock, 0, s>>>(static_cast<const float4*>(src), dst, V, total);
  return hipGetLastError();
}

}  // namespace wd
