// Complex arithmetic on (re, im) register pairs.
//
// gfx950 has no complex instructions, so complex products are spelled out in
// real FMAs (the alternative to fused complex multiply-add of Sec. V-E;
// the conjugate form conj(a)*b of Sec. III-D is what U^dag h needs).
#pragma once

#include <hip/hip_runtime.h>

// Every translation unit that includes this header compiles the code after
// this point with FMA contraction off: the only fused multiply-adds are the
// explicit ones below, so a result does not depend on how the compiler
// schedules the kernel it is computed in (prologue or loop of a march,
// one or several right-hand sides per workgroup).
#pragma clang fp contract(off)

namespace wd {

template <typename R>
struct cx {
  R re, im;
};

// a * b + c with a single rounding
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }

// a + i*b and a - i*b
template <typename R>
__device__ __forceinline__ cx<R> addi(cx<R> a, cx<R> b) { return {a.re - b.im, a.im + b.re}; }
template <typename R>
__device__ __forceinline__ cx<R> subi(cx<R> a, cx<R> b) { return {a.re + b.im, a.im - b.re}; }

// a*b rounded once. In FP32 it is spelled as a multiply-add with +0, which
// gives the same value (an exact zero product comes out as +0), so that every
// use of a link entry is a multiply-add operand: with binary16 links the
// compiler then folds each conversion to FP32 into a mixed-precision
// multiply-add instead of converting separately.
template <typename R>
__device__ __forceinline__ R prod(R a, R b) {
  if constexpr (sizeof(R) == 4) return fmar(a, b, R(0));
  else return a * b;
}

// a*b and conj(a)*b
template <typename R>
__device__ __forceinline__ cx<R> mul(cx<R> a, cx<R> b) {
  return {fmar(a.re, b.re, -prod(a.im, b.im)), fmar(a.re, b.im, prod(a.im, b.re))};
}
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {fmar(a.re, b.re, prod(a.im, b.im)), fmar(a.re, b.im, -prod(a.im, b.re))};
}
// c + a*b and c + conj(a)*b
template <typename R>
__device__ __forceinline__ cx<R> fma(cx<R> a, cx<R> b, cx<R> c) {
  return {fmar(-a.im, b.im, fmar(a.re, b.re, c.re)), fmar(a.im, b.re, fmar(a.re, b.im, c.im))};
}
template <typename R>
__device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c) {
  return {fmar(a.im, b.im, fmar(a.re, b.re, c.re)), fmar(-a.im, b.re, fmar(a.re, b.im, c.im))};
}
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> scale(R s, cx<R> a) { return {s * a.re, s * a.im}; }

}  // namespace wd
