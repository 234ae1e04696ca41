// One site's CG residual update r -= alpha (A p), for the dslash launch that
// fuses it into its epilogue (FP32 and FP16 storage), and the whole vector
// update x += alpha p, r -= alpha (A p) of FP16-storage vectors for the
// separate kernel; each returns the site's contribution to <r, r> (of the
// values as stored). Also the store of a site of t = Q p with its squared
// norm, for the dslash launch that fuses <p, A p> = |t|^2 into its epilogue.
#pragma once

#include "fields.h"

namespace wd {

__device__ __forceinline__ double norm2(double2 a) { return fmar(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ double norm2(float4 a) {
  const double x = a.x, y = a.y, z = a.z, w = a.w;
  return fmar(x, x, fmar(y, y, fmar(z, z, w * w)));
}

__device__ __forceinline__ double site_norm2(const cx<float> (&v)[12]) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double re = v[c].re, im = v[c].im;
    s = fmar(re, re, fmar(im, im, s));
  }
  return s;
}

// Quantises and stores a site (cached stores: CG vectors are read again at
// once); returns the squared norm of the values as stored.
__device__ __forceinline__ double store_half_site(h8* __restrict__ p, long s, const cx<float> (&v)[12]) {
  h8 q[3];
  const float m = half_quantise(v, q);
#pragma unroll
  for (int j = 0; j < 3; ++j) p[half_unit(s, j)] = q[j];
  reinterpret_cast<float*>(p)[half_scale_index(s)] = m;
  double n = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double d = static_cast<float>(q[j][k]) * m;
      n = fmar(d, d, n);
    }
  return n;
}

// r -= alpha (A p) at one site; ap holds A p. FP32 vectors.
__device__ __forceinline__ double cg_site_update_r(float4* __restrict__ r, long V, long s,
                                                   const cx<float> (&ap)[12], double alpha) {
  const float a = static_cast<float>(alpha);
  double n = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const long e = pidx(s, j, 6, V);
    float4 re = r[e];
    re.x = fmar(-a, ap[2 * j].re, re.x);
    re.y = fmar(-a, ap[2 * j].im, re.y);
    re.z = fmar(-a, ap[2 * j + 1].re, re.z);
    re.w = fmar(-a, ap[2 * j + 1].im, re.w);
    r[e] = re;
    n += norm2(re);
  }
  return n;
}

// The same for FP16-storage vectors: r is requantised per site.
__device__ __forceinline__ double cg_site_update_r(h8* __restrict__ r, long V, long s,
                                                   const cx<float> (&ap)[12], double alpha) {
  const float a = static_cast<float>(alpha);
  cx<float> rv[12];
  load_spinor(r, V, static_cast<int>(s), rv);
#pragma unroll
  for (int c = 0; c < 12; ++c) rv[c] = {fmar(-a, ap[c].re, rv[c].re), fmar(-a, ap[c].im, rv[c].im)};
  return store_half_site(r, s, rv);
}

// x_lo += alpha p at one site, x_lo the FP32 accumulator (FP32 layout) and p
// in FP16 storage (pv: p at the site, dequantised).
__device__ __forceinline__ void cg_site_update_x(float4* __restrict__ x, long V, long s,
                                                 const cx<float> (&pv)[12], float a) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const long e = pidx(s, j, 6, V);
    float4 xe = x[e];
    xe.x = fmar(a, pv[2 * j].re, xe.x);
    xe.y = fmar(a, pv[2 * j].im, xe.y);
    xe.z = fmar(a, pv[2 * j + 1].re, xe.z);
    xe.w = fmar(a, pv[2 * j + 1].im, xe.w);
    x[e] = xe;
  }
}

// x_lo += a0 p0, then += a1 p1, at one site (two updates of
// cg_site_update_x in turn, with one read and one write of x_lo).
__device__ __forceinline__ void cg_site_update_x2(float4* __restrict__ x, long V, long s,
                                                  const cx<float> (&p0)[12], float a0,
                                                  const cx<float> (&p1)[12], float a1) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const long e = pidx(s, j, 6, V);
    float4 xe = x[e];
    xe.x = fmar(a0, p0[2 * j].re, xe.x);
    xe.y = fmar(a0, p0[2 * j].im, xe.y);
    xe.z = fmar(a0, p0[2 * j + 1].re, xe.z);
    xe.w = fmar(a0, p0[2 * j + 1].im, xe.w);
    xe.x = fmar(a1, p1[2 * j].re, xe.x);
    xe.y = fmar(a1, p1[2 * j].im, xe.y);
    xe.z = fmar(a1, p1[2 * j + 1].re, xe.z);
    xe.w = fmar(a1, p1[2 * j + 1].im, xe.w);
    x[e] = xe;
  }
}

// FP16-storage vectors: x is the FP32 accumulator x_lo (FP32 layout); r is
// requantised per site.
__device__ __forceinline__ double cg_site_update(float4* __restrict__ x, h8* __restrict__ r,
                                                 const h8* __restrict__ p, long V, long s,
                                                 const cx<float> (&ap)[12], double alpha) {
  const float a = static_cast<float>(alpha);
  cx<float> pv[12];
  load_spinor(p, V, static_cast<int>(s), pv);
  cg_site_update_x(x, V, s, pv, a);
  return cg_site_update_r(r, V, s, ap, alpha);
}

// Stores a site of t = Q p (streaming stores, as the plain operator) and
// returns its squared norm (of the values as stored).
__device__ __forceinline__ double store_site_norm(double2* __restrict__ p, long V, int s,
                                                  const cx<double> (&v)[12]) {
  store_spinor(p, V, s, v);
  double n = 0.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) n += fmar(v[c].re, v[c].re, v[c].im * v[c].im);
  return n;
}
__device__ __forceinline__ double store_site_norm(float4* __restrict__ p, long V, int s,
                                                  const cx<float> (&v)[12]) {
  store_spinor(p, V, s, v);
  return site_norm2(v);
}
__device__ __forceinline__ double store_site_norm(h8* __restrict__ p, long /*V*/, int s,
                                                  const cx<float> (&v)[12]) {
  h8 q[3];
  const float m = half_quantise(v, q);
#pragma unroll
  for (int j = 0; j < 3; ++j) __builtin_nontemporal_store(q[j], p + half_unit(s, j));
  __builtin_nontemporal_store(m, reinterpret_cast<float*>(p) + half_scale_index(s));
  double n = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double d = static_cast<float>(q[j][k]) * m;
      n = fmar(d, d, n);
    }
  return n;
}

// alpha = <r, r> / <p, A p> and its failure flag from <p, A p> = t.
__device__ __forceinline__ double cg_alpha(double t, double rr, bool* flag) {
  *flag = !isfinite(t);
  if (!(t > 0.0)) {
    if (rr > 0.0) *flag = true;
    return 0.0;
  }
  return rr / t;
}

}  // namespace wd
