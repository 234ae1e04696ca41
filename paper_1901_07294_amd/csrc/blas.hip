// Vector kernels of the conjugate-gradient solver: fused updates and
// deterministic reductions over packed spinor fields.
//
// A packed FP64 or FP32 field (fields.h) is a flat array of 16-byte
// elements: 12 per site in FP64 (double2), 6 per site in FP32 (float4), in
// blocks of kLayoutBlock sites. Their elementwise kernels walk that flat array; the
// reductions skip the padding sites of the last block. An FP16 field shares
// one scale among the 24 reals of a site, so its kernels work site by site
// (one thread per site, real sites only), in FP32 arithmetic, and store
// results requantised. Every reduction is two-stage with a fixed
// assignment of elements to threads and a fixed combination order, so a sum
// depends only on the lattice, never on how many right-hand sides are in
// flight or on timing: results are bitwise reproducible.
#include "blas.h"
#include "cg_site.h"
#include "fields.h"

namespace wd {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// This thread's share of pp[0..np): pp[threadIdx.x + kThreads * j] added in
// order of j, with four loads in flight.
__device__ __forceinline__ double strided_sum(const double* __restrict__ pp, int np) {
  double s = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * kThreads < np; i += 4 * kThreads) {
    const double a0 = pp[i], a1 = pp[i + kThreads], a2 = pp[i + 2 * kThreads], a3 = pp[i + 3 * kThreads];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; i < np; i += kThreads) s += pp[i];
  return s;
}

// Sum of v over the workgroup, combined in a fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[kThreads / 64];
  v = wave_sum(v);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) part[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += part[i];
  return s;
}

// <p, A p> and alpha = <r, r> / <p, A p> from the partial sums of the
// preceding norm kernel, computed by every workgroup in the same order (so
// all agree bit for bit); workgroup 0 records them in the scalars.
// Non-finite or non-positive curvature raises kFlag.
__device__ __forceinline__ double alpha_from_partials(const double* __restrict__ pp, int np,
                                                      double* sc) {
  __shared__ double s_alpha;
  double t = strided_sum(pp, np);
  t = block_sum(t);
  if (threadIdx.x == 0) {
    bool flag = !isfinite(t);
    double a;
    if (!(t > 0.0)) {
      a = 0.0;
      if (sc[kRr] > 0.0) flag = true;
    } else {
      a = sc[kRr] / t;
    }
    if (blockIdx.x == 0) {
      sc[kPap] = t;
      sc[kAlpha] = a;
      sc[kRrPrev] = sc[kRr];
      if (flag) sc[kFlag] = 1.0;
    }
    s_alpha = a;
  }
  __syncthreads();
  return s_alpha;
}

// The new <r, r> from the partial sums of the preceding x, r update and
// beta = <r,r>_new / <r,r>_old, computed by every workgroup in the same order
// (the order a one-workgroup reduction would take); workgroup 0 records
// <r,r>, its running maximum and beta. Only workgroup 0 writes the scalars,
// and the others read kRrPrev alone, which this kernel does not write.
__device__ __forceinline__ double beta_from_partials(const double* __restrict__ pp, int np,
                                                     double* sc) {
  __shared__ double s_beta;
  double s = strided_sum(pp, np);
  s = block_sum(s);
  if (threadIdx.x == 0) {
    const double old = sc[kRrPrev];
    const double b = old > 0.0 ? s / old : 0.0;
    if (blockIdx.x == 0) {
      if (!isfinite(s)) sc[kFlag] = 1.0;
      sc[kBeta] = b;
      sc[kRr] = s;
      if (s > sc[kRrMax]) sc[kRrMax] = s;
    }
    s_beta = b;
  }
  __syncthreads();
  return s_beta;
}

// Is flat element e of a packed field of P elements per site a real site?
template <int P>
__device__ __forceinline__ bool real_site(long e, long V) {
  return (e / (P * kLayoutBlock)) * kLayoutBlock + (e % kLayoutBlock) < V;
}

template <typename T>
struct Elems;
template <>
struct Elems<double2> {
  static constexpr int P = 12;
};
template <>
struct Elems<float4> {
  static constexpr int P = 6;
};

// ---------------------------------------------------------------- partials

template <typename T>
__global__ __launch_bounds__(kThreads) void norm2_partial_kernel(const T* __restrict__ v, long n,
                                                                 long V, RhsSet set,
                                                                 double* __restrict__ partials) {
  const int slot = blockIdx.y;
  const T* x = v + set.idx[slot] * n;
  double s = 0.0;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads)
    if (real_site<Elems<T>::P>(e, V)) s += norm2(x[e]);
  s = block_sum(s);
  if (threadIdx.x == 0) partials[set.idx[slot] * gridDim.x + blockIdx.x] = s;
}

// x += alpha p ; r -= alpha Ap ; partial |r|^2   (alpha from the scalars).
// FP64 vectors update the FP64 solution x_hi; FP32 vectors update the FP32
// accumulator x_lo (same layout as p), which is added into x_hi at each
// reliable update.
template <typename T>
__global__ __launch_bounds__(kThreads) void update_xr_kernel(T* __restrict__ x, T* __restrict__ r,
                                                             const T* __restrict__ p,
                                                             const T* __restrict__ ap, long n, long V,
                                                             RhsSet set, double* __restrict__ scal,
                                                             const double* __restrict__ pap, int npap,
                                                             double* __restrict__ partials) {
  const int k = set.idx[blockIdx.y];
  const double alpha = alpha_from_partials(pap + k * npap, npap, scal + k * kScalars);
  T* xk = x + k * n;
  T* rk = r + k * n;
  const T* pk = p + k * n;
  const T* apk = ap + k * n;
  double s = 0.0;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads) {
    const T pe = pk[e];
    T re = rk[e];
    const T ae = apk[e];
    T xe = xk[e];
    if constexpr (Elems<T>::P == 12) {
      xe.x = fmar(alpha, pe.x, xe.x);
      xe.y = fmar(alpha, pe.y, xe.y);
      re.x = fmar(-alpha, ae.x, re.x);
      re.y = fmar(-alpha, ae.y, re.y);
    } else {
      const float a = static_cast<float>(alpha);
      xe.x = fmar(a, pe.x, xe.x);
      xe.y = fmar(a, pe.y, xe.y);
      xe.z = fmar(a, pe.z, xe.z);
      xe.w = fmar(a, pe.w, xe.w);
      re.x = fmar(-a, ae.x, re.x);
      re.y = fmar(-a, ae.y, re.y);
      re.z = fmar(-a, ae.z, re.z);
      re.w = fmar(-a, ae.w, re.w);
    }
    xk[e] = xe;
    rk[e] = re;
    if (real_site<Elems<T>::P>(e, V)) s += norm2(re);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = s;
}

// FP64 vectors, first half of the vector work of an iteration: r -= alpha Ap
// and the partial sums of the new |r|^2 (alpha reduced from the <p, A p>
// partials, as in update_xr_kernel). The second half, update_xp_kernel,
// updates x and p together, so p is read once per iteration.
__global__ __launch_bounds__(kThreads) void update_r_kernel(double2* __restrict__ r,
                                                            const double2* __restrict__ ap, long n,
                                                            long V, RhsSet set, double* __restrict__ scal,
                                                            const double* __restrict__ pap, int npap,
                                                            double* __restrict__ partials) {
  const int k = set.idx[blockIdx.y];
  const double alpha = alpha_from_partials(pap + k * npap, npap, scal + k * kScalars);
  double2* rk = r + k * n;
  const double2* apk = ap + k * n;
  double s = 0.0;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads) {
    double2 re = rk[e];
    const double2 ae = apk[e];
    re.x = fmar(-alpha, ae.x, re.x);
    re.y = fmar(-alpha, ae.y, re.y);
    rk[e] = re;
    if (real_site<12>(e, V)) s += norm2(re);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = s;
}

// FP64 vectors: x += alpha p, then p = r + beta p, with alpha as workgroup 0 of
// update_r_kernel recorded it (the value every workgroup there applied) and
// beta reduced from that kernel's |r|^2 partials. Each element gets the
// multiply-adds of update_xr_kernel and update_p_kernel, so the bits match.
__global__ __launch_bounds__(kThreads) void update_xp_kernel(double2* __restrict__ x,
                                                             double2* __restrict__ p,
                                                             const double2* __restrict__ r, long n,
                                                             RhsSet set, const double* __restrict__ rr,
                                                             int nrr, double* __restrict__ scal) {
  const int k = set.idx[blockIdx.y];
  double* sc = scal + k * kScalars;
  const double alpha = sc[kAlpha];  // not written by this kernel
  const double beta = beta_from_partials(rr + k * nrr, nrr, sc);
  double2* xk = x + k * n;
  double2* pk = p + k * n;
  const double2* rk = r + k * n;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads) {
    double2 pe = pk[e];
    const double2 re = rk[e];
    double2 xe = xk[e];
    xe.x = fmar(alpha, pe.x, xe.x);
    xe.y = fmar(alpha, pe.y, xe.y);
    pe.x = fmar(beta, pe.x, re.x);
    pe.y = fmar(beta, pe.y, re.y);
    xk[e] = xe;
    pk[e] = pe;
  }
}

// Mixed precision, FP32 vectors, after the dslash launch that applied
// r -= alpha Ap in its epilogue: x_lo += alpha p, then p = r + beta p, with
// alpha as that launch recorded it (the value all its workgroups applied) and
// beta reduced from its <r,r> per tile slice. The multiply-adds are those of
// update_xr_kernel and update_p_kernel, so the bits match. KIND (blas.h):
// which x update is applied; p_out is written after p_cur and p_prev are
// read, by the same lane, so it may be either of them.
template <int KIND>
__global__ __launch_bounds__(kThreads) void update_xp_lo_kernel(float4* __restrict__ x, float4* p_out,
                                                                const float4* p_cur, const float4* p_prev,
                                                                const float4* __restrict__ r, long n,
                                                                RhsSet set, const double* __restrict__ rr,
                                                                int nrr, double* __restrict__ scal) {
  const int k = set.idx[blockIdx.y];
  double* sc = scal + k * kScalars;
  const float a = static_cast<float>(sc[kAlpha]);  // not written by this kernel
  const float a0 = KIND == kXpPair ? static_cast<float>(sc[kAlphaPrev]) : 0.0f;
  if (KIND == kXpDefer && blockIdx.x == 0 && threadIdx.x == 0) sc[kAlphaPrev] = sc[kAlpha];
  const float b = static_cast<float>(beta_from_partials(rr + k * nrr, nrr, sc));
  float4* xk = x + k * n;
  float4* pok = p_out + k * n;
  const float4* pck = p_cur + k * n;
  const float4* ppk = p_prev + k * n;
  const float4* rk = r + k * n;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads) {
    float4 pe = pck[e];
    const float4 re = rk[e];
    if constexpr (KIND != kXpDefer) {
      float4 xe = xk[e];
      if constexpr (KIND == kXpPair) {
        const float4 q = ppk[e];
        xe.x = fmar(a0, q.x, xe.x);
        xe.y = fmar(a0, q.y, xe.y);
        xe.z = fmar(a0, q.z, xe.z);
        xe.w = fmar(a0, q.w, xe.w);
      }
      xe.x = fmar(a, pe.x, xe.x);
      xe.y = fmar(a, pe.y, xe.y);
      xe.z = fmar(a, pe.z, xe.z);
      xe.w = fmar(a, pe.w, xe.w);
      xk[e] = xe;
    }
    pe.x = fmar(b, pe.x, re.x);
    pe.y = fmar(b, pe.y, re.y);
    pe.z = fmar(b, pe.z, re.z);
    pe.w = fmar(b, pe.w, re.w);
    pok[e] = pe;
  }
}

// x_hi += x_lo (FP32 element j of a block holds FP64 elements 2j and 2j+1 of
// the same sites), then x_lo = 0
__global__ __launch_bounds__(kThreads) void flush_x_kernel(double2* __restrict__ hi,
                                                           float4* __restrict__ lo, long n, long nhi,
                                                           RhsSet set) {
  const int k = set.idx[blockIdx.y];
  double2* hk = hi + k * nhi;
  float4* lk = lo + k * n;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads) {
    const long blk = e / (6 * kLayoutBlock);
    const long j = (e / kLayoutBlock) % 6;
    const long lane = e % kLayoutBlock;
    const long h0 = (blk * 12 + 2 * j) * kLayoutBlock + lane;
    const float4 l = lk[e];
    double2 x0 = hk[h0];
    double2 x1 = hk[h0 + kLayoutBlock];
    x0.x += l.x;
    x0.y += l.y;
    x1.x += l.z;
    x1.y += l.w;
    hk[h0] = x0;
    hk[h0 + kLayoutBlock] = x1;
    lk[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

// p = r + beta p
template <typename T>
__global__ __launch_bounds__(kThreads) void update_p_kernel(T* __restrict__ p, const T* __restrict__ r,
                                                            long n, RhsSet set,
                                                            const double* __restrict__ rr, int nrr,
                                                            double* __restrict__ scal) {
  const int k = set.idx[blockIdx.y];
  const double beta = beta_from_partials(rr + k * nrr, nrr, scal + k * kScalars);
  T* pk = p + k * n;
  const T* rk = r + k * n;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads) {
    T pe = pk[e];
    const T re = rk[e];
    if constexpr (Elems<T>::P == 12) {
      pe.x = fmar(beta, pe.x, re.x);
      pe.y = fmar(beta, pe.y, re.y);
    } else {
      const float b = static_cast<float>(beta);
      pe.x = fmar(b, pe.x, re.x);
      pe.y = fmar(b, pe.y, re.y);
      pe.z = fmar(b, pe.z, re.z);
      pe.w = fmar(b, pe.w, re.w);
    }
    pk[e] = pe;
  }
}

// r = b - r (r holds A x on entry), partial |r|^2
__global__ __launch_bounds__(kThreads) void residual_kernel(double2* __restrict__ r,
                                                            const double2* __restrict__ b, long n,
                                                            long V, RhsSet set,
                                                            double* __restrict__ partials) {
  const int k = set.idx[blockIdx.y];
  double2* rk = r + k * n;
  const double2* bk = b + k * n;
  double s = 0.0;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads) {
    const double2 be = bk[e];
    double2 re = rk[e];
    re.x = be.x - re.x;
    re.y = be.y - re.y;
    rk[e] = re;
    if (real_site<12>(e, V)) s += norm2(re);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = s;
}

// lo = FP32(hi), over FP32 elements
__global__ __launch_bounds__(kThreads) void demote_kernel(float4* __restrict__ lo,
                                                          const double2* __restrict__ hi, long n,
                                                          long nhi, RhsSet set) {
  const int k = set.idx[blockIdx.y];
  float4* lk = lo + k * n;
  const double2* hk = hi + k * nhi;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads) {
    const long blk = e / (6 * kLayoutBlock);
    const long j = (e / kLayoutBlock) % 6;
    const long lane = e % kLayoutBlock;
    const long h0 = (blk * 12 + 2 * j) * kLayoutBlock + lane;
    const double2 a = hk[h0];
    const double2 c = hk[h0 + kLayoutBlock];
    lk[e] = make_float4(static_cast<float>(a.x), static_cast<float>(a.y), static_cast<float>(c.x),
                        static_cast<float>(c.y));
  }
}

// lo = FP32(b - ax) over FP32 elements, with partial |b - ax|^2 of the FP64
// values (the mixed solver's true residual: its FP64 form is not kept)
__global__ __launch_bounds__(kThreads) void residual_demote_kernel(float4* __restrict__ lo,
                                                                   const double2* __restrict__ b,
                                                                   const double2* __restrict__ ax, long n,
                                                                   long nhi, long V, RhsSet set,
                                                                   double* __restrict__ partials) {
  const int k = set.idx[blockIdx.y];
  float4* lk = lo + k * n;
  const double2* bk = b + k * nhi;
  const double2* ak = ax + k * nhi;
  double s = 0.0;
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads) {
    const long blk = e / (6 * kLayoutBlock);
    const long j = (e / kLayoutBlock) % 6;
    const long lane = e % kLayoutBlock;
    const long h0 = (blk * 12 + 2 * j) * kLayoutBlock + lane;
    const double2 b0 = bk[h0], b1 = bk[h0 + kLayoutBlock];
    const double2 a0 = ak[h0], a1 = ak[h0 + kLayoutBlock];
    const double2 r0 = make_double2(b0.x - a0.x, b0.y - a0.y);
    const double2 r1 = make_double2(b1.x - a1.x, b1.y - a1.y);
    lk[e] = make_float4(static_cast<float>(r0.x), static_cast<float>(r0.y), static_cast<float>(r1.x),
                        static_cast<float>(r1.y));
    if (real_site<6>(e, V)) s += norm2(r0) + norm2(r1);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void copy_kernel(T* __restrict__ dst, const T* __restrict__ src,
                                                        long n, RhsSet set) {
  const int k = set.idx[blockIdx.y];
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads)
    dst[k * n + e] = src[k * n + e];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void zero_kernel(T* __restrict__ dst, long n, RhsSet set) {
  const int k = set.idx[blockIdx.y];
  T z;
  memset(&z, 0, sizeof(T));
  for (long e = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; e < n;
       e += static_cast<long>(gridDim.x) * kThreads)
    dst[k * n + e] = z;
}

// ------------------------------------------------------------ FP16 fields

#define WD_SITE_LOOP(i, V) \
  for (long i = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; i < (V); \
       i += static_cast<long>(gridDim.x) * kThreads)

__global__ __launch_bounds__(kThreads) void norm2_half_kernel(const h8* __restrict__ v, long units,
                                                              long V, RhsSet set,
                                                              double* __restrict__ partials) {
  const int k = set.idx[blockIdx.y];
  const h8* x = v + k * units;
  double s = 0.0;
  WD_SITE_LOOP(i, V) {
    cx<float> a[12];
    load_spinor(x, V, static_cast<int>(i), a);
    s += site_norm2(a);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = s;
}

// x_lo += alpha p (FP32 accumulator, FP32 layout) ; r -= alpha Ap (FP32,
// requantised) ; partial |r|^2
__global__ __launch_bounds__(kThreads) void update_xr_half_kernel(
    float4* __restrict__ x, h8* __restrict__ r, const h8* __restrict__ p, const h8* __restrict__ ap,
    long units, long nlo32, long V, RhsSet set, double* __restrict__ scal,
    const double* __restrict__ pap, int npap, double* __restrict__ partials) {
  const int k = set.idx[blockIdx.y];
  const double a = alpha_from_partials(pap + k * npap, npap, scal + k * kScalars);
  float4* xk = x + k * nlo32;
  h8* rk = r + k * units;
  double s = 0.0;
  WD_SITE_LOOP(i, V) {
    cx<float> av[12];
    load_spinor(ap + k * units, V, static_cast<int>(i), av);
    s += cg_site_update(xk, rk, p + k * units, V, i, av, a);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = s;
}

// Mixed precision, FP16-storage vectors, after the dslash launch that applied
// r -= alpha Ap: x_lo += alpha p (x_lo FP32, nlo32 elements per right-hand
// side), then p = r + beta p requantised; alpha, beta, KIND and the buffers
// as update_xp_lo_kernel.
template <int KIND>
__global__ __launch_bounds__(kThreads) void update_xp_half_kernel(float4* __restrict__ x, h8* p_out,
                                                                  const h8* p_cur, const h8* p_prev,
                                                                  const h8* __restrict__ r, long units,
                                                                  long nlo32, long V, RhsSet set,
                                                                  const double* __restrict__ rr, int nrr,
                                                                  double* __restrict__ scal) {
  const int k = set.idx[blockIdx.y];
  double* sc = scal + k * kScalars;
  const float a = static_cast<float>(sc[kAlpha]);  // not written by this kernel
  const float a0 = KIND == kXpPair ? static_cast<float>(sc[kAlphaPrev]) : 0.0f;
  if (KIND == kXpDefer && blockIdx.x == 0 && threadIdx.x == 0) sc[kAlphaPrev] = sc[kAlpha];
  const float b = static_cast<float>(beta_from_partials(rr + k * nrr, nrr, sc));
  float4* xk = x + k * nlo32;
  h8* pok = p_out + k * units;
  const h8* pck = p_cur + k * units;
  const h8* ppk = p_prev + k * units;
  const h8* rk = r + k * units;
  WD_SITE_LOOP(i, V) {
    cx<float> pv[12], rv[12];
    load_spinor(pck, V, static_cast<int>(i), pv);
    if constexpr (KIND == kXpPair) {
      cx<float> qv[12];
      load_spinor(ppk, V, static_cast<int>(i), qv);
      cg_site_update_x2(xk, V, i, qv, a0, pv, a);
    } else if constexpr (KIND == kXpNow) {
      cg_site_update_x(xk, V, i, pv, a);
    }
    load_spinor(rk, V, static_cast<int>(i), rv);
#pragma unroll
    for (int c = 0; c < 12; ++c) pv[c] = {fmar(b, pv[c].re, rv[c].re), fmar(b, pv[c].im, rv[c].im)};
    store_half_site(pok, i, pv);
  }
}

// p = r + beta p
__global__ __launch_bounds__(kThreads) void update_p_half_kernel(h8* __restrict__ p,
                                                                 const h8* __restrict__ r, long units,
                                                                 long V, RhsSet set,
                                                                 const double* __restrict__ rr, int nrr,
                                                                 double* __restrict__ scal) {
  const int k = set.idx[blockIdx.y];
  const float b = static_cast<float>(beta_from_partials(rr + k * nrr, nrr, scal + k * kScalars));
  h8* pk = p + k * units;
  WD_SITE_LOOP(i, V) {
    cx<float> pv[12], rv[12];
    load_spinor(pk, V, static_cast<int>(i), pv);
    load_spinor(r + k * units, V, static_cast<int>(i), rv);
#pragma unroll
    for (int c = 0; c < 12; ++c) pv[c] = {fmar(b, pv[c].re, rv[c].re), fmar(b, pv[c].im, rv[c].im)};
    store_half_site(pk, i, pv);
  }
}

// lo = FP16(hi): components rounded to FP32, then quantised per site
__global__ __launch_bounds__(kThreads) void demote_half_kernel(h8* __restrict__ lo,
                                                               const double2* __restrict__ hi,
                                                               long units, long nhi, long V,
                                                               RhsSet set) {
  const int k = set.idx[blockIdx.y];
  const double2* hk = hi + k * nhi;
  WD_SITE_LOOP(i, V) {
    cx<float> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const double2 t = hk[pidx(i, c, 12, V)];
      v[c] = {static_cast<float>(t.x), static_cast<float>(t.y)};
    }
    store_half_site(lo + k * units, i, v);
  }
}

// lo = FP16(b - ax) (components rounded to FP32, then quantised per site),
// with partial |b - ax|^2 of the FP64 values
__global__ __launch_bounds__(kThreads) void residual_demote_half_kernel(h8* __restrict__ lo,
                                                                        const double2* __restrict__ b,
                                                                        const double2* __restrict__ ax,
                                                                        long units, long nhi, long V,
                                                                        RhsSet set,
                                                                        double* __restrict__ partials) {
  const int k = set.idx[blockIdx.y];
  const double2* bk = b + k * nhi;
  const double2* ak = ax + k * nhi;
  double s = 0.0;
  WD_SITE_LOOP(i, V) {
    cx<float> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const double2 bt = bk[pidx(i, c, 12, V)], at = ak[pidx(i, c, 12, V)];
      const double2 t = make_double2(bt.x - at.x, bt.y - at.y);
      s += norm2(t);
      v[c] = {static_cast<float>(t.x), static_cast<float>(t.y)};
    }
    store_half_site(lo + k * units, i, v);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = s;
}

#undef WD_SITE_LOOP

// One workgroup per right-hand side: sum its partials in a fixed order and
// update the scalars. Non-finite or non-positive curvature raises kFlag.
__global__ __launch_bounds__(kThreads) void finalize_kernel(const double* __restrict__ partials,
                                                            int nparts, RhsSet set, int mode,
                                                            double* __restrict__ scal) {
  const int k = set.idx[blockIdx.x];
  double s = strided_sum(partials + k * nparts, nparts);
  s = block_sum(s);
  if (threadIdx.x != 0) return;
  double* sc = scal + k * kScalars;
  if (!isfinite(s)) sc[kFlag] = 1.0;
  switch (mode) {
    case kFinPap:  // <p, A p> = |Q p|^2 ; alpha = rr / pAp
      sc[kPap] = s;
      if (!(s > 0.0)) {
        sc[kAlpha] = 0.0;
        if (sc[kRr] > 0.0) sc[kFlag] = 1.0;
      } else {
        sc[kAlpha] = sc[kRr] / s;
      }
      break;
    case kFinTrueRr:  // true residual after a reliable update
      sc[kRr] = s;
      sc[kRrMax] = s;
      sc[kRrTrue] = s;
      break;
    case kFinNorm:  // plain norm (|b|^2)
      sc[kB2] = s;
      break;
  }
}

dim3 grid(long n, int nset) {
  long nb = (n + kThreads * 4 - 1) / (kThreads * 4);
  if (nb > kMaxPartials) nb = kMaxPartials;
  if (nb < 1) nb = 1;
  return dim3(static_cast<unsigned>(nb), static_cast<unsigned>(nset));
}

}  // namespace

hipError_t blas_norm2(const void* v, int prec, long n, long V, const RhsSet& set, double* partials,
                      double* scal, int mode, hipStream_t st) {
  int np = 0;
  const hipError_t e = blas_norm2_partials(v, prec, n, V, set, partials, &np, st);
  if (e != hipSuccess) return e;
  finalize_kernel<<<set.n, kThreads, 0, st>>>(partials, np, set, mode, scal);
  return hipGetLastError();
}

hipError_t blas_norm2_partials(const void* v, int prec, long n, long V, const RhsSet& set,
                               double* partials, int* nparts, hipStream_t st) {
  const dim3 g = grid(prec == WD_FP16 ? V : n, set.n);
  *nparts = static_cast<int>(g.x);
  if (prec == WD_FP64)
    norm2_partial_kernel<double2><<<g, kThreads, 0, st>>>(static_cast<const double2*>(v), n, V, set, partials);
  else if (prec == WD_FP32)
    norm2_partial_kernel<float4><<<g, kThreads, 0, st>>>(static_cast<const float4*>(v), n, V, set, partials);
  else
    norm2_half_kernel<<<g, kThreads, 0, st>>>(static_cast<const h8*>(v), n, V, set, partials);
  return hipGetLastError();
}

hipError_t blas_update_xr(void* x, void* r, const void* p, const void* ap, int prec, long n, long nlo32,
                          long V, const RhsSet& set, const double* pap, int npap, double* partials,
                          int* nrr, double* scal, hipStream_t st) {
  const dim3 g = grid(prec == WD_FP16 ? V : n, set.n);
  *nrr = static_cast<int>(g.x);
  if (prec == WD_FP64)
    update_xr_kernel<double2><<<g, kThreads, 0, st>>>(static_cast<double2*>(x), static_cast<double2*>(r),
                                                       static_cast<const double2*>(p),
                                                       static_cast<const double2*>(ap), n, V, set,
                                                       scal, pap, npap, partials);
  else if (prec == WD_FP32)
    update_xr_kernel<float4><<<g, kThreads, 0, st>>>(static_cast<float4*>(x), static_cast<float4*>(r),
                                                      static_cast<const float4*>(p),
                                                      static_cast<const float4*>(ap), n, V, set, scal,
                                                      pap, npap, partials);
  else
    update_xr_half_kernel<<<g, kThreads, 0, st>>>(static_cast<float4*>(x), static_cast<h8*>(r),
                                                  static_cast<const h8*>(p), static_cast<const h8*>(ap),
                                                  n, nlo32, V, set, scal, pap, npap, partials);
  return hipGetLastError();
}

hipError_t blas_update_r(void* r, const void* ap, long n, long V, const RhsSet& set, const double* pap,
                         int npap, double* partials, int* nrr, double* scal, hipStream_t st) {
  const dim3 g = grid(n, set.n);
  *nrr = static_cast<int>(g.x);
  update_r_kernel<<<g, kThreads, 0, st>>>(static_cast<double2*>(r), static_cast<const double2*>(ap), n, V,
                                          set, scal, pap, npap, partials);
  return hipGetLastError();
}

hipError_t blas_update_xp(void* x, void* p, const void* r, long n, const RhsSet& set, const double* rr,
                          int nrr, double* scal, hipStream_t st) {
  update_xp_kernel<<<grid(n, set.n), kThreads, 0, st>>>(static_cast<double2*>(x), static_cast<double2*>(p),
                                                        static_cast<const double2*>(r), n, set, rr, nrr,
                                                        scal);
  return hipGetLastError();
}

hipError_t blas_flush_x(void* hi, void* lo, long nlo32, long nhi, const RhsSet& set, hipStream_t st) {
  flush_x_kernel<<<grid(nlo32, set.n), kThreads, 0, st>>>(static_cast<double2*>(hi),
                                                          static_cast<float4*>(lo), nlo32, nhi, set);
  return hipGetLastError();
}

hipError_t blas_update_p(void* p, const void* r, int prec, long n, long V, const RhsSet& set,
                         const double* rr, int nrr, double* scal, hipStream_t st) {
  if (prec == WD_FP64)
    update_p_kernel<double2><<<grid(n, set.n), kThreads, 0, st>>>(
        static_cast<double2*>(p), static_cast<const double2*>(r), n, set, rr, nrr, scal);
  else if (prec == WD_FP32)
    update_p_kernel<float4><<<grid(n, set.n), kThreads, 0, st>>>(
        static_cast<float4*>(p), static_cast<const float4*>(r), n, set, rr, nrr, scal);
  else
    update_p_half_kernel<<<grid(V, set.n), kThreads, 0, st>>>(static_cast<h8*>(p),
                                                              static_cast<const h8*>(r), n, V, set, rr,
                                                              nrr, scal);
  return hipGetLastError();
}

hipError_t blas_update_xp_lo(void* x, void* p_out, const void* p_cur, const void* p_prev, const void* r,
                             int kind, int prec, long n, long nlo32, long V, const RhsSet& set,
                             const double* rr, int nrr, double* scal, hipStream_t st) {
  if (kind != kXpNow && kind != kXpDefer && kind != kXpPair) return hipErrorInvalidValue;
  if (kind == kXpDefer && p_out == p_cur) return hipErrorInvalidValue;
  if (prec == WD_FP32) {
    auto* xo = static_cast<float4*>(x);
    auto* po = static_cast<float4*>(p_out);
    auto* pc = static_cast<const float4*>(p_cur);
    auto* pp = static_cast<const float4*>(p_prev);
    auto* rv = static_cast<const float4*>(r);
    const dim3 g = grid(n, set.n);
    if (kind == kXpNow) update_xp_lo_kernel<kXpNow><<<g, kThreads, 0, st>>>(xo, po, pc, pp, rv, n, set, rr, nrr, scal);
    else if (kind == kXpDefer)
      update_xp_lo_kernel<kXpDefer><<<g, kThreads, 0, st>>>(xo, po, pc, pp, rv, n, set, rr, nrr, scal);
    else update_xp_lo_kernel<kXpPair><<<g, kThreads, 0, st>>>(xo, po, pc, pp, rv, n, set, rr, nrr, scal);
  } else if (prec == WD_FP16) {
    auto* xo = static_cast<float4*>(x);
    auto* po = static_cast<h8*>(p_out);
    auto* pc = static_cast<const h8*>(p_cur);
    auto* pp = static_cast<const h8*>(p_prev);
    auto* rv = static_cast<const h8*>(r);
    const dim3 g = grid(V, set.n);
    if (kind == kXpNow)
      update_xp_half_kernel<kXpNow><<<g, kThreads, 0, st>>>(xo, po, pc, pp, rv, n, nlo32, V, set, rr, nrr, scal);
    else if (kind == kXpDefer)
      update_xp_half_kernel<kXpDefer><<<g, kThreads, 0, st>>>(xo, po, pc, pp, rv, n, nlo32, V, set, rr, nrr,
                                                               scal);
    else
      update_xp_half_kernel<kXpPair><<<g, kThreads, 0, st>>>(xo, po, pc, pp, rv, n, nlo32, V, set, rr, nrr,
                                                              scal);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t blas_residual(void* r, const void* b, long n, long V, const RhsSet& set, double* partials,
                         double* scal, hipStream_t st) {
  const dim3 g = grid(n, set.n);
  residual_kernel<<<g, kThreads, 0, st>>>(static_cast<double2*>(r), static_cast<const double2*>(b), n,
                                          V, set, partials);
  finalize_kernel<<<set.n, kThreads, 0, st>>>(partials, static_cast<int>(g.x), set, kFinTrueRr, scal);
  return hipGetLastError();
}

hipError_t blas_residual_demote(void* lo, const void* b, const void* ax, int prec, long n, long nhi, long V,
                                const RhsSet& set, double* partials, double* scal, hipStream_t st) {
  dim3 g;
  if (prec == WD_FP32) {
    g = grid(n, set.n);
    residual_demote_kernel<<<g, kThreads, 0, st>>>(static_cast<float4*>(lo), static_cast<const double2*>(b),
                                                   static_cast<const double2*>(ax), n, nhi, V, set, partials);
  } else if (prec == WD_FP16) {
    g = grid(V, set.n);
    residual_demote_half_kernel<<<g, kThreads, 0, st>>>(static_cast<h8*>(lo), static_cast<const double2*>(b),
                                                        static_cast<const double2*>(ax), n, nhi, V, set,
                                                        partials);
  } else {
    return hipErrorInvalidValue;
  }
  finalize_kernel<<<set.n, kThreads, 0, st>>>(partials, static_cast<int>(g.x), set, kFinTrueRr, scal);
  return hipGetLastError();
}

hipError_t blas_demote(void* lo, const void* hi, int prec, long n, long nhi, long V, const RhsSet& set,
                       hipStream_t st) {
  if (prec == WD_FP32)
    demote_kernel<<<grid(n, set.n), kThreads, 0, st>>>(static_cast<float4*>(lo),
                                                       static_cast<const double2*>(hi), n, nhi, set);
  else if (prec == WD_FP16)
    demote_half_kernel<<<grid(V, set.n), kThreads, 0, st>>>(static_cast<h8*>(lo),
                                                            static_cast<const double2*>(hi), n, nhi, V,
                                                            set);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Copies and zero fills move whole 16-byte elements (FP16 fields included).
hipError_t blas_copy(void* dst, const void* src, int prec, long n, const RhsSet& set, hipStream_t st) {
  if (prec == WD_FP64)
    copy_kernel<double2><<<grid(n, set.n), kThreads, 0, st>>>(static_cast<double2*>(dst),
                                                              static_cast<const double2*>(src), n, set);
  else
    copy_kernel<float4><<<grid(n, set.n), kThreads, 0, st>>>(static_cast<float4*>(dst),
                                                             static_cast<const float4*>(src), n, set);
  return hipGetLastError();
}

hipError_t blas_zero(void* dst, int prec, long n, const RhsSet& set, hipStream_t st) {
  if (prec == WD_FP64)
    zero_kernel<double2><<<grid(n, set.n), kThreads, 0, st>>>(static_cast<double2*>(dst), n, set);
  else
    zero_kernel<float4><<<grid(n, set.n), kThreads, 0, st>>>(static_cast<float4*>(dst), n, set);
  return hipGetLastError();
}

}  // namespace wd
