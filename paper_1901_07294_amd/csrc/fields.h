// Packed device layouts of spinor and gauge fields, and their loads/stores.
//
// Every packed field is an array of structures of arrays: sites are grouped in
// blocks of 64 consecutive sites (one wave), and inside a block each "plane"
// (one 8- or 16-byte piece of every site's data) is a contiguous run of 64
// elements. A wave's load of one plane is one contiguous 512 B - 1 KiB run,
// and all planes of a block follow each other, so a wave streams its sites'
// data as one contiguous region (Sec. II-B: the data layout decides how well
// the stencil vectorises; one lane per site plays the role of Grid's one
// vector lane per virtual node, without intra-vector permutes).
//
//  spinor, per right-hand side (stride packed_sites(V) * 24 reals):
//    FP64: 12 planes of double2   plane c = 3*spin + colour
//    FP32:  6 planes of float4    plane j holds components 2j, 2j+1
//  gauge, all four directions in one block:
//    FP64 full: 36 planes of double2   plane 9*mu + 3*row + col
//    FP64 c12 : 24 planes of double2   plane 6*mu + 3*row + col, rows 0-1
//    FP32 full: 36 planes of float2
//    FP32 c12 : 12 planes of float4    plane 3*mu + j holds entries 2j, 2j+1 of rows 0-1
#pragma once

#include <hip/hip_runtime.h>

#include "cplx.h"

// Sites per AoSoA block of a packed field (0: plain planes of V sites).
#ifndef WD_LAYOUT_BLOCK
#define WD_LAYOUT_BLOCK 64
#endif

namespace wd {

constexpr int kLayoutBlock = WD_LAYOUT_BLOCK;

// Sites a packed field of V sites is padded to.
__host__ __device__ constexpr long packed_sites(long V) {
  return kLayoutBlock > 0 ? (V + kLayoutBlock - 1) / kLayoutBlock * kLayoutBlock : V;
}

// Element index of plane c (of P planes per site) of site s in a packed field.
__device__ __forceinline__ long pidx(long s, int c, int P, long V) {
  if constexpr (kLayoutBlock > 0)
    return ((s / kLayoutBlock) * P + c) * kLayoutBlock + (s % kLayoutBlock);
  else
    return c * V + s;
}

// Vector types of packed spinors (S) and links (L) per arithmetic precision.
template <typename R>
struct Packed;
template <>
struct Packed<double> {
  using S = double2;
  using L = double2;
};
template <>
struct Packed<float> {
  using S = float4;
  using L = float2;
};

// Native vector types for the non-temporal (streaming) stores of results.
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ spinors

__device__ __forceinline__ void load_spinor(const double2* __restrict__ p, long V, int s,
                                            cx<double> (&v)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double2 t = p[pidx(s, c, 12, V)];
    v[c] = {t.x, t.y};
  }
}

__device__ __forceinline__ void load_spinor(const float4* __restrict__ p, long V, int s,
                                            cx<float> (&v)[12]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const float4 t = p[pidx(s, j, 6, V)];
    v[2 * j] = {t.x, t.y};
    v[2 * j + 1] = {t.z, t.w};
  }
}

__device__ __forceinline__ void store_spinor(double2* __restrict__ p, long V, int s,
                                             const cx<double> (&v)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const nd2 t = {v[c].re, v[c].im};
    __builtin_nontemporal_store(t, reinterpret_cast<nd2*>(p + pidx(s, c, 12, V)));
  }
}

__device__ __forceinline__ void store_spinor(float4* __restrict__ p, long V, int s,
                                             const cx<float> (&v)[12]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const nf4 t = {v[2 * j].re, v[2 * j].im, v[2 * j + 1].re, v[2 * j + 1].im};
    __builtin_nontemporal_store(t, reinterpret_cast<nf4*>(p + pidx(s, j, 6, V)));
  }
}

// Spinors staged in LDS use the same plane layout over the n sites of a tile.
__device__ __forceinline__ void lds_store_spinor(double2* p, int n, int i, const cx<double> (&v)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c * n + i] = make_double2(v[c].re, v[c].im);
}

__device__ __forceinline__ void lds_store_spinor(float4* p, int n, int i, const cx<float> (&v)[12]) {
#pragma unroll
  for (int j = 0; j < 6; ++j)
    p[j * n + i] = make_float4(v[2 * j].re, v[2 * j].im, v[2 * j + 1].re, v[2 * j + 1].im);
}

__device__ __forceinline__ void lds_load_spinor(const double2* p, int n, int i, cx<double> (&v)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double2 t = p[c * n + i];
    v[c] = {t.x, t.y};
  }
}

__device__ __forceinline__ void lds_load_spinor(const float4* p, int n, int i, cx<float> (&v)[12]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const float4 t = p[j * n + i];
    v[2 * j] = {t.x, t.y};
    v[2 * j + 1] = {t.z, t.w};
  }
}

// -------------------------------------------------------------------- links

// Third row of an SU(3) matrix from its first two: r2 = conj(r0 x r1).
template <typename R>
__device__ __forceinline__ void rebuild_row2(cx<R> (&u)[9]) {
  u[6] = conj(mul(u[1], u[5]) - mul(u[2], u[4]));
  u[7] = conj(mul(u[2], u[3]) - mul(u[0], u[5]));
  u[8] = conj(mul(u[0], u[4]) - mul(u[1], u[3]));
}

template <bool C12>
__device__ __forceinline__ void load_link(const double2* __restrict__ p, long V, int mu, int s,
                                          cx<double> (&u)[9]) {
  constexpr int n = C12 ? 6 : 9;
#pragma unroll
  for (int k = 0; k < n; ++k) {
    const double2 t = p[pidx(s, mu * n + k, 4 * n, V)];
    u[k] = {t.x, t.y};
  }
  if constexpr (C12) rebuild_row2(u);
}

template <bool C12>
__device__ __forceinline__ void load_link(const float2* __restrict__ p, long V, int mu, int s,
                                          cx<float> (&u)[9]) {
  if constexpr (C12) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float4 t = q[pidx(s, mu * 3 + j, 12, V)];
      u[2 * j] = {t.x, t.y};
      u[2 * j + 1] = {t.z, t.w};
    }
    rebuild_row2(u);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float2 t = p[pidx(s, mu * 9 + k, 36, V)];
      u[k] = {t.x, t.y};
    }
  }
}

}  // namespace wd
