// Per-site pieces of the Wilson-Dirac stencil shared by the dslash kernels:
// spin projection, SU(3) multiplication, reconstruction into the accumulator.
//
// Each hop first projects the 4-spinor to a 2-spinor, h = psi_u -/+ A_mu psi_l
// with gamma_mu = [[0, A_mu], [A_mu^dag, 0]] in the DeGrand-Rossi basis, then
// multiplies by the SU(3) link (2 colour matrix-vector products instead of 4)
// and rebuilds the lower spin components as -/+ A_mu^dag (U h).
#pragma once

#include "fields.h"

namespace wd {

// h = psi_u + S * A_mu psi_l (S = -1 forward hop, +1 backward hop). psi is
// indexed 3*spin + colour; h is indexed 3*halfspin + colour.
//   A_x = [[0, i], [i, 0]]   A_y = [[0, -1], [1, 0]]
//   A_z = [[i, 0], [0, -i]]  A_t = [[1, 0], [0, 1]]
template <int MU, int S, typename R>
__device__ __forceinline__ void project(const cx<R> (&p)[12], cx<R> (&h)[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<R> p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
    if constexpr (MU == 0) {
      h[a] = S > 0 ? addi(p0, p3) : subi(p0, p3);
      h[3 + a] = S > 0 ? addi(p1, p2) : subi(p1, p2);
    } else if constexpr (MU == 1) {
      h[a] = S > 0 ? p0 - p3 : p0 + p3;
      h[3 + a] = S > 0 ? p1 + p2 : p1 - p2;
    } else if constexpr (MU == 2) {
      h[a] = S > 0 ? addi(p0, p2) : subi(p0, p2);
      h[3 + a] = S > 0 ? subi(p1, p3) : addi(p1, p3);
    } else {
      h[a] = S > 0 ? p0 + p2 : p0 - p2;
      h[3 + a] = S > 0 ? p1 + p3 : p1 - p3;
    }
  }
}

// acc += (U h, S * A_mu^dag (U h)); g = U h (or U^dag h) indexed like h.
//   A_x^dag = [[0, -i], [-i, 0]]   A_y^dag = [[0, 1], [-1, 0]]
//   A_z^dag = [[-i, 0], [0, i]]    A_t^dag = 1
template <int MU, int S, typename R>
__device__ __forceinline__ void reconstruct_add(const cx<R> (&g)[6], cx<R> (&acc)[12]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<R> g0 = g[a], g1 = g[3 + a];
    acc[a] = acc[a] + g0;
    acc[3 + a] = acc[3 + a] + g1;
    if constexpr (MU == 0) {  // lower = S * (-i g1, -i g0)
      acc[6 + a] = S > 0 ? subi(acc[6 + a], g1) : addi(acc[6 + a], g1);
      acc[9 + a] = S > 0 ? subi(acc[9 + a], g0) : addi(acc[9 + a], g0);
    } else if constexpr (MU == 1) {  // lower = S * (g1, -g0)
      acc[6 + a] = S > 0 ? acc[6 + a] + g1 : acc[6 + a] - g1;
      acc[9 + a] = S > 0 ? acc[9 + a] - g0 : acc[9 + a] + g0;
    } else if constexpr (MU == 2) {  // lower = S * (-i g0, i g1)
      acc[6 + a] = S > 0 ? subi(acc[6 + a], g0) : addi(acc[6 + a], g0);
      acc[9 + a] = S > 0 ? addi(acc[9 + a], g1) : subi(acc[9 + a], g1);
    } else {  // lower = S * (g0, g1)
      acc[6 + a] = S > 0 ? acc[6 + a] + g0 : acc[6 + a] - g0;
      acc[9 + a] = S > 0 ? acc[9 + a] + g1 : acc[9 + a] - g1;
    }
  }
}

// g = U h (DAG = false) or U^dag h (DAG = true), on both colour vectors of h.
template <bool DAG, typename R>
__device__ __forceinline__ void su3_mul(const cx<R> (&u)[9], const cx<R> (&h)[6], cx<R> (&g)[6]) {
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if constexpr (!DAG) {
        cx<R> r = mul(u[3 * a], h[3 * s]);
        r = fma(u[3 * a + 1], h[3 * s + 1], r);
        g[3 * s + a] = fma(u[3 * a + 2], h[3 * s + 2], r);
      } else {
        cx<R> r = cmul(u[a], h[3 * s]);
        r = cfma(u[3 + a], h[3 * s + 1], r);
        g[3 * s + a] = cfma(u[6 + a], h[3 * s + 2], r);
      }
    }
  }
}

// One hop with the neighbour spinor already in registers and the link of
// direction MU at site ls loaded from the packed gauge field.
template <int MU, int S, bool C12, typename LV, typename R>
__device__ __forceinline__ void hop_psi(const cx<R> (&psi)[12], const LV* __restrict__ links, long V,
                                        int ls, cx<R> (&acc)[12]) {
  cx<R> u[9];
  load_link<C12>(links, V, MU, ls, u);
  cx<R> h[6];
  project<MU, S>(psi, h);
  cx<R> g[6];
  su3_mul<(S > 0)>(u, h, g);
  reconstruct_add<MU, S>(g, acc);
}

// One hop: neighbour spinor at site n, link of direction MU at site ls.
template <int MU, int S, bool C12, typename SV, typename LV, typename R>
__device__ __forceinline__ void hop(const SV* __restrict__ in, const LV* __restrict__ links, long V,
                                    int n, int ls, cx<R> (&acc)[12]) {
  cx<R> psi[12];
  load_spinor(in, V, n, psi);
  hop_psi<MU, S, C12>(psi, links, V, ls, acc);
}

// out = diag * psi - acc / 2, optionally times gamma5 (negates spins 2, 3).
template <typename R>
__device__ __forceinline__ void epilogue(const cx<R> (&psi)[12], const cx<R> (&acc)[12], R diag,
                                         int gamma5, cx<R> (&o)[12]) {
  const R half = R(0.5);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    cx<R> r = {fmar(diag, psi[c].re, -half * acc[c].re), fmar(diag, psi[c].im, -half * acc[c].im)};
    if (gamma5 && c >= 6) r = -r;
    o[c] = r;
  }
}

}  // namespace wd
