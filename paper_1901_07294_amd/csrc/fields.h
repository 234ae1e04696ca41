// Packed device layouts of spinor and gauge fields, and their loads/stores.
//
// Every packed field is an array of structures of arrays: sites are grouped in
// blocks of B consecutive sites, and inside a block each "plane" (one 4- to
// 16-byte piece of every site's data) is a contiguous run of B elements; the
// planes of a block follow each other (Sec. II-B: the data layout decides how
// well the stencil vectorises; one lane per site plays the role of Grid's one
// vector lane per virtual node, without intra-vector permutes). A wave's load
// of one plane is one contiguous 256 B - 1 KiB run.
//
// B is 2048 sites for FP64 and FP32 fields: a whole x-y plane or two of a
// typical lattice, so the workgroups that march neighbouring tiles stream
// long contiguous runs of each plane (measured on MI355X: the FP64 and FP32
// operators run 5 % faster than with 64-site blocks). FP16 fields,
// whose link planes have 4-byte elements, keep B = 64 sites (one wave), with
// which their planes stay in short contiguous groups. Every field is padded
// to a whole number of 2048-site blocks.
//
//  spinor, per right-hand side (whole blocks, padded):
//    FP64: 12 planes of double2   plane c = 3*spin + colour
//    FP32:  6 planes of float4    plane j holds components 2j, 2j+1
//    FP16:  3 planes of 8 x binary16 (plane j holds components 4j .. 4j+3),
//           then one plane of FP32 per-site scales: 52 B per site
//  gauge, all four directions in one block:
//    FP64 full: 36 planes of double2   plane 9*mu + 3*row + col
//    FP64 c12 : 24 planes of double2   plane 6*mu + 3*row + col, rows 0-1
//    FP32 full: 36 planes of float2
//    FP32 c12 : 12 planes of float4    plane 3*mu + j holds entries 2j, 2j+1 of rows 0-1
//    FP16 full: 36 planes of 2 x binary16
//    FP16 c12 : 12 planes of 4 x binary16 (as FP32 c12)
//
// FP16 is a storage format only (arithmetic is FP32). A spinor site is stored
// as q = v / s with s = max |v| over its 24 reals (v in FP32) and read back as
// float(q) * s; links are stored unscaled (every entry of an SU(3) matrix is at
// most 1 in modulus), each FP64 entry rounded once to binary16. Every rounding
// is to nearest even.
#pragma once

#include <hip/hip_runtime.h>

#include "cplx.h"

namespace wd {

// Sites per block of FP64 and FP32 fields (and the padding unit of every
// field), and per block of FP16 fields.
#ifndef WD_LAYOUT_BLOCK
#define WD_LAYOUT_BLOCK 2048
#endif
constexpr int kLayoutBlock = WD_LAYOUT_BLOCK;
constexpr int kHalfBlock = 64;
static_assert(kLayoutBlock % kHalfBlock == 0, "a layout block holds whole waves of sites");

// Sites a packed field of V sites is padded to.
__host__ __device__ constexpr long packed_sites(long V) {
  return (V + kLayoutBlock - 1) / kLayoutBlock * kLayoutBlock;
}

// Element index of plane c (of P planes per site) of site s in a packed field
// of blocks of B sites.
template <int B = kLayoutBlock>
__device__ __forceinline__ long pidx(long s, int c, int P, long /*V*/) {
  return ((s / B) * P + c) * B + (s % B);
}

// binary16 vectors of the FP16 storage format.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// Per storage type T: arithmetic type R, 16-byte spinor element S, link
// element L, sites per block, and 16-byte spinor elements per block.
template <typename T>
struct Packed;
template <>
struct Packed<double> {
  using R = double;
  using S = double2;
  using L = double2;
  static constexpr int kBlock = kLayoutBlock;
  static constexpr long kBlockUnits = kLayoutBlock * 12;
};
template <>
struct Packed<float> {
  using R = float;
  using S = float4;
  using L = float2;
  static constexpr int kBlock = kLayoutBlock;
  static constexpr long kBlockUnits = kLayoutBlock * 6;
};
template <>
struct Packed<_Float16> {
  using R = float;
  using S = h8;
  using L = h2;
  static constexpr int kBlock = kHalfBlock;
  static constexpr long kBlockUnits = kHalfBlock * 3 + kHalfBlock / 4;  // 3 planes + FP32 scales
};

// 16-byte elements of one packed spinor field of V sites.
template <typename T>
__host__ __device__ constexpr long spinor_units(long V) {
  return packed_sites(V) / Packed<T>::kBlock * Packed<T>::kBlockUnits;
}

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

// FP16 spinor: 16-byte element of plane j of site s, and (in floats) the
// site's scale, which follows the three planes of its block.
__device__ __forceinline__ long half_unit(long s, int j) {
  return (s / kHalfBlock) * Packed<_Float16>::kBlockUnits + j * kHalfBlock + (s % kHalfBlock);
}
__device__ __forceinline__ long half_scale_index(long s) {
  return ((s / kHalfBlock) * Packed<_Float16>::kBlockUnits + 3 * kHalfBlock) * 4 + (s % kHalfBlock);
}

// The product float(q) * scale is rounded on its own (contraction is off),
// so a site reads the same FP32 values whether they come from here or from a
// copy staged in LDS. It is written as a multiply-add with +0 (the same
// value; an exact zero comes out as +0) so that the conversion from binary16
// folds into one mixed-precision multiply-add.
__device__ __forceinline__ void load_spinor(const h8* __restrict__ p, long /*V*/, int s,
                                            cx<float> (&v)[12]) {
  const float sc = reinterpret_cast<const float*>(p)[half_scale_index(s)];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const h8 t = p[half_unit(s, j)];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      v[4 * j + k] = {fmar(static_cast<float>(t[2 * k]), sc, 0.0f),
                      fmar(static_cast<float>(t[2 * k + 1]), sc, 0.0f)};
  }
}

// An FP32 value rounded to binary16. The empty asm pins x in a register as
// an FP32 result, so the compiler cannot merge the multiply that produced it
// and this conversion into one mixed-precision instruction with a single
// rounding (which would make the stored bits depend on the kernel).
__device__ __forceinline__ _Float16 f32_to_half(float x) {
  __asm__ volatile("" : "+v"(x));
  return static_cast<_Float16>(x);
}

// Quantises a site: scale = max |component|, q = v * (1 / scale) rounded to
// FP32 and then to binary16. When the scale is subnormal (below 2^-126) its
// reciprocal would overflow to infinity; such a site is first multiplied by
// 2^64 (exact), which gives the same q as unbounded exponents would, and the
// stored scale stays the site's own largest modulus.
__device__ __forceinline__ float half_quantise(const cx<float> (&v)[12], h8 (&q)[3]) {
  float m = 0.0f;
#pragma unroll
  for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
  if (m > 0.0f && m < 0x1p-126f) {
    const float k = 0x1p64f;
    const float inv = 1.0f / (m * k);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        q[j][2 * c] = f32_to_half((v[4 * j + c].re * k) * inv);
        q[j][2 * c + 1] = f32_to_half((v[4 * j + c].im * k) * inv);
      }
    return m;
  }
  const float inv = m > 0.0f ? 1.0f / m : 0.0f;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      q[j][2 * k] = f32_to_half(v[4 * j + k].re * inv);
      q[j][2 * k + 1] = f32_to_half(v[4 * j + k].im * inv);
    }
  return m;
}

__device__ __forceinline__ void store_spinor(h8* __restrict__ p, long /*V*/, int s,
                                             const cx<float> (&v)[12]) {
  h8 q[3];
  const float m = half_quantise(v, q);
#pragma unroll
  for (int j = 0; j < 3; ++j) __builtin_nontemporal_store(q[j], p + half_unit(s, j));
  __builtin_nontemporal_store(m, reinterpret_cast<float*>(p) + half_scale_index(s));
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

typedef float nf2 __attribute__((ext_vector_type(2)));

// One 4- to 16-byte element read with a non-temporal load: for data that no
// other workgroup reads again, so that its lines displace less of the ones
// that neighbouring workgroups still have to read from L2.
template <typename N, typename E>
__device__ __forceinline__ N nt_load(const E* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const N*>(p));
}

// Third row of an SU(3) matrix from its first two: r2 = conj(r0 x r1).
template <typename R>
__device__ __forceinline__ void rebuild_row2(cx<R> (&u)[9]) {
  u[6] = conj(mul(u[1], u[5]) - mul(u[2], u[4]));
  u[7] = conj(mul(u[2], u[3]) - mul(u[0], u[5]));
  u[8] = conj(mul(u[0], u[4]) - mul(u[1], u[3]));
}

// NT: non-temporal loads (links that no other workgroup reads again).
template <bool C12, bool NT = false>
__device__ __forceinline__ void load_link(const double2* __restrict__ p, long V, int mu, int s,
                                          cx<double> (&u)[9]) {
  constexpr int n = C12 ? 6 : 9;
#pragma unroll
  for (int k = 0; k < n; ++k) {
    const long e = pidx(s, mu * n + k, 4 * n, V);
    if constexpr (NT) {
      const nd2 t = nt_load<nd2>(p + e);
      u[k] = {t.x, t.y};
    } else {
      const double2 t = p[e];
      u[k] = {t.x, t.y};
    }
  }
  if constexpr (C12) rebuild_row2(u);
}

template <bool C12, bool NT = false>
__device__ __forceinline__ void load_link(const float2* __restrict__ p, long V, int mu, int s,
                                          cx<float> (&u)[9]) {
  if constexpr (C12) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const long e = pidx(s, mu * 3 + j, 12, V);
      const nf4 t = NT ? nt_load<nf4>(q + e) : nf4{q[e].x, q[e].y, q[e].z, q[e].w};
      u[2 * j] = {t.x, t.y};
      u[2 * j + 1] = {t.z, t.w};
    }
    rebuild_row2(u);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const long e = pidx(s, mu * 9 + k, 36, V);
      const nf2 t = NT ? nt_load<nf2>(p + e) : nf2{p[e].x, p[e].y};
      u[k] = {t.x, t.y};
    }
  }
}

template <bool C12, bool NT = false>
__device__ __forceinline__ void load_link(const h2* __restrict__ p, long V, int mu, int s,
                                          cx<float> (&u)[9]) {
  if constexpr (C12) {
    const h4* q = reinterpret_cast<const h4*>(p);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const long e = pidx<kHalfBlock>(s, mu * 3 + j, 12, V);
      const h4 t = NT ? nt_load<h4>(q + e) : q[e];
      u[2 * j] = {static_cast<float>(t.x), static_cast<float>(t.y)};
      u[2 * j + 1] = {static_cast<float>(t.z), static_cast<float>(t.w)};
    }
    rebuild_row2(u);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const long e = pidx<kHalfBlock>(s, mu * 9 + k, 36, V);
      const h2 t = NT ? nt_load<h2>(p + e) : p[e];
      u[k] = {static_cast<float>(t.x), static_cast<float>(t.y)};
    }
  }
}

// ------------------------------------------------ buffer-resource access
//
// FP64 and FP32 fields of less than 4 GiB can be read and written through a
// raw buffer resource: the field's base (wave-uniform) sits in scalar
// registers, every lane adds one 32-bit byte offset (its site's element in
// plane 0) and every plane a scalar constant, so that no vector instruction
// computes an address. With a 64-bit address per load the FP64 operator spent
// about as many vector instructions on addresses as on arithmetic. Stores and
// the non-temporal loads carry the non-temporal cache policy explicitly.

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename E>
struct BufField {
  __amdgpu_buffer_rsrc_t r;
};

constexpr int kBufWord3 = 0x00020000;  // descriptor word 3: raw dword access (gfx9 family)
constexpr int kBufNt = 2;              // cache policy: non-temporal
constexpr int kPlane16 = kLayoutBlock * 16;  // bytes between planes of 16-byte elements

template <typename E>
__device__ __forceinline__ BufField<E> buf_field(const E* p, unsigned bytes) {
  return {__builtin_amdgcn_make_buffer_rsrc(const_cast<E*>(p), static_cast<short>(0),
                                            static_cast<int>(bytes), kBufWord3)};
}

// Byte offset of site s's element of plane 0 in a field of P planes of
// ES-byte elements (the caller guarantees the field is below 4 GiB).
template <int P, int ES>
__device__ __forceinline__ unsigned site_off(int s) {
  const unsigned u = static_cast<unsigned>(s);
  return ((u / kLayoutBlock) * (P * kLayoutBlock) + (u % kLayoutBlock)) * ES;
}

template <int POL = 0>
__device__ __forceinline__ nd2 buf_ld2(const BufField<double2>& f, unsigned o, int so) {
  return __builtin_bit_cast(nd2, __builtin_amdgcn_raw_buffer_load_b128(f.r, o, so, POL));
}

__device__ __forceinline__ void load_spinor(const BufField<double2>& f, long /*V*/, int s,
                                            cx<double> (&v)[12]) {
  const unsigned o = site_off<12, 16>(s);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const nd2 t = buf_ld2(f, o, c * kPlane16);
    v[c] = {t.x, t.y};
  }
}

__device__ __forceinline__ void load_spinor(const BufField<float4>& f, long /*V*/, int s,
                                            cx<float> (&v)[12]) {
  const unsigned o = site_off<6, 16>(s);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const nf4 t = __builtin_bit_cast(nf4, __builtin_amdgcn_raw_buffer_load_b128(f.r, o, j * kPlane16, 0));
    v[2 * j] = {t.x, t.y};
    v[2 * j + 1] = {t.z, t.w};
  }
}

// POL: the stores' cache policy (non-temporal by default)
template <int POL = kBufNt>
__device__ __forceinline__ void store_spinor(const BufField<double2>& f, long /*V*/, int s,
                                             const cx<double> (&v)[12]) {
  const unsigned o = site_off<12, 16>(s);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const nd2 t = {v[c].re, v[c].im};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, t), f.r, o, c * kPlane16, POL);
  }
}

__device__ __forceinline__ void store_spinor(const BufField<float4>& f, long /*V*/, int s,
                                             const cx<float> (&v)[12]) {
  const unsigned o = site_off<6, 16>(s);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const nf4 t = {v[2 * j].re, v[2 * j].im, v[2 * j + 1].re, v[2 * j + 1].im};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, t), f.r, o, j * kPlane16, kBufNt);
  }
}

template <bool C12, bool NT = false>
__device__ __forceinline__ void load_link(const BufField<double2>& f, long /*V*/, int mu, int s,
                                          cx<double> (&u)[9]) {
  constexpr int n = C12 ? 6 : 9;
  const unsigned o = site_off<4 * n, 16>(s);
#pragma unroll
  for (int k = 0; k < n; ++k) {
    const nd2 t = buf_ld2<NT ? kBufNt : 0>(f, o, (mu * n + k) * kPlane16);
    u[k] = {t.x, t.y};
  }
  if constexpr (C12) rebuild_row2(u);
}

template <bool C12, bool NT = false>
__device__ __forceinline__ void load_link(const BufField<float2>& f, long /*V*/, int mu, int s,
                                          cx<float> (&u)[9]) {
  constexpr int pol = NT ? kBufNt : 0;
  if constexpr (C12) {
    const unsigned o = site_off<12, 16>(s);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const nf4 t = __builtin_bit_cast(
          nf4, __builtin_amdgcn_raw_buffer_load_b128(f.r, o, (mu * 3 + j) * kPlane16, pol));
      u[2 * j] = {t.x, t.y};
      u[2 * j + 1] = {t.z, t.w};
    }
    rebuild_row2(u);
  } else {
    const unsigned o = site_off<36, 8>(s);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const nf2 t = __builtin_bit_cast(
          nf2, __builtin_amdgcn_raw_buffer_load_b64(f.r, o, (mu * 9 + k) * kLayoutBlock * 8, pol));
      u[k] = {t.x, t.y};
    }
  }
}

// FP16 storage (64-site blocks): a spinor block is 3 planes of 64 x 16 bytes
// followed by 64 FP32 scales; links are planes of 64 x 4 bytes (full) or
// 64 x 8 bytes (12-real).
__device__ __forceinline__ unsigned half_block_off(int s) {
  return (static_cast<unsigned>(s) / kHalfBlock) * (Packed<_Float16>::kBlockUnits * 16u);
}

__device__ __forceinline__ void load_spinor(const BufField<h8>& f, long /*V*/, int s, cx<float> (&v)[12]) {
  const unsigned b = half_block_off(s);
  const unsigned l = static_cast<unsigned>(s) % kHalfBlock;
  const float sc = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                 f.r, b + 3 * kHalfBlock * 16 + l * 4, 0, 0));
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const h8 t = __builtin_bit_cast(h8, __builtin_amdgcn_raw_buffer_load_b128(f.r, b + l * 16, j * kHalfBlock * 16, 0));
#pragma unroll
    for (int k = 0; k < 4; ++k)
      v[4 * j + k] = {fmar(static_cast<float>(t[2 * k]), sc, 0.0f),
                      fmar(static_cast<float>(t[2 * k + 1]), sc, 0.0f)};
  }
}

__device__ __forceinline__ void store_spinor(const BufField<h8>& f, long /*V*/, int s,
                                             const cx<float> (&v)[12]) {
  h8 q[3];
  const float m = half_quantise(v, q);
  const unsigned b = half_block_off(s);
  const unsigned l = static_cast<unsigned>(s) % kHalfBlock;
#pragma unroll
  for (int j = 0; j < 3; ++j)
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, q[j]), f.r, b + l * 16, j * kHalfBlock * 16,
                                           kBufNt);
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, m), f.r, b + 3 * kHalfBlock * 16 + l * 4, 0,
                                        kBufNt);
}

template <bool C12, bool NT = false>
__device__ __forceinline__ void load_link(const BufField<h2>& f, long /*V*/, int mu, int s, cx<float> (&u)[9]) {
  constexpr int pol = NT ? kBufNt : 0;
  const unsigned blk = static_cast<unsigned>(s) / kHalfBlock;
  const unsigned l = static_cast<unsigned>(s) % kHalfBlock;
  if constexpr (C12) {
    const unsigned o = blk * (12 * kHalfBlock * 8) + l * 8;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const h4 t = __builtin_bit_cast(
          h4, __builtin_amdgcn_raw_buffer_load_b64(f.r, o, (mu * 3 + j) * kHalfBlock * 8, pol));
      u[2 * j] = {static_cast<float>(t.x), static_cast<float>(t.y)};
      u[2 * j + 1] = {static_cast<float>(t.z), static_cast<float>(t.w)};
    }
    rebuild_row2(u);
  } else {
    const unsigned o = blk * (36 * kHalfBlock * 4) + l * 4;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const h2 t = __builtin_bit_cast(
          h2, __builtin_amdgcn_raw_buffer_load_b32(f.r, o, (mu * 9 + k) * kHalfBlock * 4, pol));
      u[k] = {static_cast<float>(t.x), static_cast<float>(t.y)};
    }
  }
}

}  // namespace wd
