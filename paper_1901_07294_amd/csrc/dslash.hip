// The Wilson-Dirac operator on gfx950: one lane per lattice site.
//
//   out(x) = (4+m) psi(x) - 1/2 sum_mu [ (1-g_mu) U_mu(x) psi(x+mu)
//                                       + (1+g_mu) U_mu(x-mu)^dag psi(x-mu) ]
//
// (the hopping term of eq. (1), Sec. II-A, with the opposite sign of gamma_mu
// and the (4+m) normalisation), optionally multiplied by gamma5 = diag(1,1,-1,-1).
//
// The stencil is bound by HBM bandwidth (1320 flop against >= 960 compulsory
// bytes per site in FP64), so there is no matrix-core work here: every lane
// streams its site's links and spinor planes, coalesced across the wave.
// Each hop first projects the 4-spinor to a 2-spinor, h = psi_u -/+ A_mu psi_l
// with gamma_mu = [[0, A_mu], [A_mu^dag, 0]] in the DeGrand-Rossi basis, then
// multiplies by the SU(3) link (2 colour matrix-vector products instead of 4)
// and rebuilds the lower spin components as -/+ A_mu^dag (U h).
#include "fields.h"
#include "wd_internal.h"

namespace wd {
namespace {

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

// One hop: neighbour spinor at site n, link of direction MU at site ls.
template <int MU, int S, bool C12, typename R>
__device__ __forceinline__ void hop(const typename Packed<R>::S* __restrict__ in,
                                    const typename Packed<R>::L* __restrict__ links, long V, int n,
                                    int ls, cx<R> (&acc)[12]) {
  cx<R> psi[12];
  load_spinor(in, V, n, psi);
  cx<R> u[9];
  load_link<C12>(links, V, MU, ls, u);
  cx<R> h[6];
  project<MU, S>(psi, h);
  cx<R> g[6];
  su3_mul<(S > 0)>(u, h, g);
  reconstruct_add<MU, S>(g, acc);
}

// Workgroup -> tile of kBlock consecutive sites. Consecutive workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2; with
// group > 0 the mapping gives every XCD runs of `group` consecutive tiles, so
// that neighbours in y and z, which sit a few tiles away, share an L2.
__device__ __forceinline__ int tile_of_block(int group) {
  const int b = blockIdx.x;
  const int nb = gridDim.x;
  if (group <= 0 || nb % (kNumXcd * group) != 0) return b;
  const int xcd = b % kNumXcd;
  const int l = b / kNumXcd;
  return ((l / group) * kNumXcd + xcd) * group + (l % group);
}

template <typename R, bool C12>
__global__ __launch_bounds__(kBlock) void dslash_kernel(const typename Packed<R>::S* __restrict__ in,
                                                        typename Packed<R>::S* __restrict__ out,
                                                        const typename Packed<R>::L* __restrict__ links,
                                                        Geo geo, R diag, int gamma5, int group) {
  const int s = tile_of_block(group) * kBlock + static_cast<int>(threadIdx.x);
  if (s >= geo.V) return;
  const long V = geo.V;

  const int x = s % geo.X;
  const int y = (s / geo.X) % geo.Y;
  const int z = (s / geo.XY) % geo.Z;
  const int t = s / geo.XYZ;
  // periodic neighbours (extent 1 wraps onto the site itself)
  const int xp = x + 1 == geo.X ? s - (geo.X - 1) : s + 1;
  const int xm = x == 0 ? s + (geo.X - 1) : s - 1;
  const int yp = y + 1 == geo.Y ? s - (geo.Y - 1) * geo.X : s + geo.X;
  const int ym = y == 0 ? s + (geo.Y - 1) * geo.X : s - geo.X;
  const int zp = z + 1 == geo.Z ? s - (geo.Z - 1) * geo.XY : s + geo.XY;
  const int zm = z == 0 ? s + (geo.Z - 1) * geo.XY : s - geo.XY;
  const int tp = t + 1 == geo.T ? s - (geo.T - 1) * geo.XYZ : s + geo.XYZ;
  const int tm = t == 0 ? s + (geo.T - 1) * geo.XYZ : s - geo.XYZ;

  cx<R> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};

  hop<0, -1, C12, R>(in, links, V, xp, s, acc);
  hop<0, +1, C12, R>(in, links, V, xm, xm, acc);
  hop<1, -1, C12, R>(in, links, V, yp, s, acc);
  hop<1, +1, C12, R>(in, links, V, ym, ym, acc);
  hop<2, -1, C12, R>(in, links, V, zp, s, acc);
  hop<2, +1, C12, R>(in, links, V, zm, zm, acc);
  hop<3, -1, C12, R>(in, links, V, tp, s, acc);
  hop<3, +1, C12, R>(in, links, V, tm, tm, acc);

  cx<R> psi[12];
  load_spinor(in, V, s, psi);
  const R half = R(0.5);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    cx<R> r = {diag * psi[c].re - half * acc[c].re, diag * psi[c].im - half * acc[c].im};
    if (gamma5 && c >= 6) r = -r;
    psi[c] = r;
  }
  store_spinor(out, V, s, psi);
}

int default_xcd_group(int nblocks) {
  // runs of 4 tiles (1024 sites) per XCD, when the grid allows it
  return nblocks % (kNumXcd * 4) == 0 ? 4 : 0;
}

}  // namespace

hipError_t launch_dslash(const wd_gauge* g, double mass, const void* in, void* out, int flags,
                         hipStream_t st) {
  const Geo geo = make_geo(g->dims);
  const unsigned nb = static_cast<unsigned>((geo.V + kBlock - 1) / kBlock);
  const int group = default_xcd_group(static_cast<int>(nb));
  const int g5 = (flags & WD_FLAG_GAMMA5) ? 1 : 0;
  if (g->prec == WD_FP64) {
    const auto* i = static_cast<const double2*>(in);
    auto* o = static_cast<double2*>(out);
    const auto* u = static_cast<const double2*>(g->links);
    const double d = 4.0 + mass;
    if (g->c12) dslash_kernel<double, true><<<nb, kBlock, 0, st>>>(i, o, u, geo, d, g5, group);
    else dslash_kernel<double, false><<<nb, kBlock, 0, st>>>(i, o, u, geo, d, g5, group);
  } else {
    const auto* i = static_cast<const float4*>(in);
    auto* o = static_cast<float4*>(out);
    const auto* u = static_cast<const float2*>(g->links);
    const float d = static_cast<float>(4.0 + mass);
    if (g->c12) dslash_kernel<float, true><<<nb, kBlock, 0, st>>>(i, o, u, geo, d, g5, group);
    else dslash_kernel<float, false><<<nb, kBlock, 0, st>>>(i, o, u, geo, d, g5, group);
  }
  return hipGetLastError();
}

}  // namespace wd
