// Complex arithmetic on (re, im) register pairs.
//
// gfx950 has no complex instructions, so complex products are spelled out in
// real FMAs (the alternative to fused complex multiply-add of Sec. V-E;
// the conjugate form conj(a)*b of Sec. III-D is what U^dag h needs).
#pragma once

#include <hip/hip_runtime.h>

namespace wd {

template <typename R>
struct cx {
  R re, im;
};

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

// a*b and conj(a)*b
template <typename R>
__device__ __forceinline__ cx<R> mul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// c + a*b and c + conj(a)*b
template <typename R>
__device__ __forceinline__ cx<R> fma(cx<R> a, cx<R> b, cx<R> c) {
  return {c.re + a.re * b.re - a.im * b.im, c.im + a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c) {
  return {c.re + a.re * b.re + a.im * b.im, c.im + a.re * b.im - a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> scale(R s, cx<R> a) { return {s * a.re, s * a.im}; }

}  // namespace wd
