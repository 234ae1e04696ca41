// Solving the Wilson system D x = b (the operator of eq. (1), Sec. II-A, in
// the (4+m) - H/2 normalisation) with the conjugate-gradient solver of cg.hip.
//
// Full-lattice gauge field: x solves the normal equations D^dag D x = D^dag b,
// with D^dag b = gamma5 D gamma5 b formed on the device.
//
// Even-odd gauge field (eo.h): with A = 4 + m, the odd sites solve
// S x_o = b^_o, S = A - H_oe H_eo / (4A), b^_o = b_o + H_oe b_e / (2A), through
// S^dag S x_o = S^dag b^_o (S^dag = gamma5 S gamma5), and the even sites follow
// as x_e = (b_e + H_eo x_o / 2) / A. S is better conditioned than D, so CG
// needs fewer iterations, each of which costs about 1.7 applications of D.
//
// Either way the call ends on the FP64 residual of the system itself,
// |b - D x| / |b|: CG first runs to the tolerance on its own residual (normal
// equations); where the system's residual is still above it, CG resumes from
// x with its tolerance tightened by the ratio found, a few times at most.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>

#include "cg_engine.h"
#include "eo.h"
#include "fields.h"

namespace wd {
namespace {

constexpr int kMaxRounds = 6;

char* at(void* base, size_t off) { return static_cast<char*>(base) + off; }

// Offsets (bytes) of the workspace: the CG solver's own, the right-hand side
// of the normal equations, a full FP64 field for D^dag b and b - D x, the
// reductions, and with even-odd the FP64 half fields b_e, b_o, x_o and three
// temporaries. Every vector holds nrhs fields.
struct WsLayout {
  size_t cg = 0, bn = 0, full = 0, partials = 0, scal = 0, be = 0, bo = 0, xo = 0, t1 = 0, t2 = 0, t3 = 0;
  size_t bytes = 0;
};

WsLayout ws_layout(const int32_t dims[4], int nrhs, int inner, bool eo) {
  WsLayout w;
  const long V = static_cast<long>(dims[0]) * dims[1] * dims[2] * dims[3];
  const size_t full = align256(static_cast<size_t>(packed_sites(V)) * nrhs * spinor_site_bytes(WD_FP64));
  const size_t half = align256(static_cast<size_t>(packed_sites(V / 2)) * nrhs * spinor_site_bytes(WD_FP64));
  size_t o = 0;
  w.cg = o; o += cg_layout(dims, nrhs, inner, eo).bytes;
  w.bn = o; o += eo ? half : full;
  w.full = o; o += full;
  w.partials = o; o += align256(static_cast<size_t>(nrhs) * kMaxPartials * sizeof(double));
  w.scal = o; o += align256(static_cast<size_t>(nrhs) * kScalars * sizeof(double));
  if (eo) {
    w.be = o; o += half;
    w.bo = o; o += half;
    w.xo = o; o += half;
    w.t1 = o; o += half;
    w.t2 = o; o += half;
    w.t3 = o; o += half;
  }
  w.bytes = o;
  return w;
}

struct Solver {
  const wd_gauge* ghi;
  const wd_gauge* glo;
  const double* masses;
  int nrhs;
  const void* b;
  void* x;
  void* ws;
  hipStream_t st;
  bool eo;
  WsLayout lay;
  RhsSet all;
  long V, Vh;

  int status(hipError_t e, const char* what) const { return launch_status(e, what); }

  // bn = D^dag b (full) or S^dag b^_o (even-odd); with even-odd also b_e, b_o.
  int prepare() {
    const long nfull = spinor_units<double>(V);
    if (!eo) {
      int rc = status(blas_gamma5(at(ws, lay.full), b, nfull, all, st), "wilson: gamma5 b");
      if (rc == WD_OK)
        rc = status(launch_dslash_multi(ghi, masses, nrhs, nullptr, at(ws, lay.full), at(ws, lay.bn),
                                        WD_FLAG_GAMMA5, st),
                    "wilson: D^dag b");
      return rc;
    }
    const EoGeo g = make_eo_geo(ghi->dims);
    int rc = status(launch_split_eo(b, at(ws, lay.be), at(ws, lay.bo), g, all, false, st), "wilson: split b");
    double d[kMaxRhs], c[kMaxRhs];
    for (int k = 0; k < nrhs; ++k) {
      d[k] = 1.0;
      c[k] = 1.0 / (2.0 * (4.0 + masses[k]));
    }
    // t1 = b^_o = b_o + H_oe b_e / (2A); t2 = gamma5 t1; bn = gamma5 S t2
    if (rc == WD_OK)
      rc = status(launch_eo_hop(ghi, 1, at(ws, lay.be), at(ws, lay.bo), at(ws, lay.t1), all, d, c, 0, st),
                  "wilson: odd source");
    if (rc == WD_OK)
      rc = status(blas_gamma5(at(ws, lay.t2), at(ws, lay.t1), spinor_units<double>(Vh), all, st),
                  "wilson: gamma5 source");
    if (rc == WD_OK)
      rc = status(launch_schur_q(ghi, masses, all, at(ws, lay.t2), at(ws, lay.t1), at(ws, lay.bn), st),
                  "wilson: S^dag source");
    return rc;
  }

  // x_o from x (a given start vector)
  int split_x() {
    return status(launch_split_eo(x, at(ws, lay.t1), at(ws, lay.xo), make_eo_geo(ghi->dims), all, false, st),
                  "wilson: split x");
  }

  // full solution from x_o: x_e = (b_e + H_eo x_o / 2) / A, merged with x_o into x
  int finish_x() {
    double d[kMaxRhs], c[kMaxRhs];
    for (int k = 0; k < nrhs; ++k) {
      d[k] = 1.0 / (4.0 + masses[k]);
      c[k] = 1.0 / (2.0 * (4.0 + masses[k]));
    }
    int rc = status(launch_eo_hop(ghi, 0, at(ws, lay.xo), at(ws, lay.be), at(ws, lay.t1), all, d, c, 0, st),
                    "wilson: even sites");
    if (rc == WD_OK)
      rc = status(launch_split_eo(x, at(ws, lay.t1), at(ws, lay.xo), make_eo_geo(ghi->dims), all, true, st),
                  "wilson: merge x");
    return rc;
  }

  // |b - D x|^2 and |b|^2 of every field into scal (kRrTrue, kB2), read back.
  int residual(double* host) {
    const long nfull = spinor_units<double>(V);
    double* partials = reinterpret_cast<double*>(at(ws, lay.partials));
    double* scal = reinterpret_cast<double*>(at(ws, lay.scal));
    int rc = WD_OK;
    if (!eo) {
      rc = status(launch_dslash_multi(ghi, masses, nrhs, nullptr, x, at(ws, lay.full), 0, st), "wilson: D x");
    } else {
      // (D x)_e = A x_e - H_eo x_o / 2 and (D x)_o = A x_o - H_oe x_e / 2, from x itself
      const EoGeo g = make_eo_geo(ghi->dims);
      double d[kMaxRhs], c[kMaxRhs];
      for (int k = 0; k < nrhs; ++k) {
        d[k] = 4.0 + masses[k];
        c[k] = -0.5;
      }
      rc = status(launch_split_eo(x, at(ws, lay.t1), at(ws, lay.xo), g, all, false, st), "wilson: split x");
      if (rc == WD_OK)
        rc = status(launch_eo_hop(ghi, 0, at(ws, lay.xo), at(ws, lay.t1), at(ws, lay.t2), all, d, c, 0, st),
                    "wilson: (D x)_e");
      if (rc == WD_OK)
        rc = status(launch_eo_hop(ghi, 1, at(ws, lay.t1), at(ws, lay.xo), at(ws, lay.t3), all, d, c, 0, st),
                    "wilson: (D x)_o");
      if (rc == WD_OK)
        rc = status(launch_split_eo(at(ws, lay.full), at(ws, lay.t2), at(ws, lay.t3), g, all, true, st),
                    "wilson: merge D x");
    }
    if (rc == WD_OK)
      rc = status(blas_zero(scal, WD_FP64, static_cast<long>(kScalars / 2), all, st), "wilson: scalars");
    if (rc == WD_OK)
      rc = status(blas_residual(at(ws, lay.full), b, nfull, V, all, partials, scal, st), "wilson: b - D x");
    if (rc == WD_OK) rc = status(blas_norm2(b, WD_FP64, nfull, V, all, partials, scal, kFinNorm, st), "wilson: |b|");
    if (rc != WD_OK) return rc;
    const hipError_t e = hipMemcpyAsync(host, scal, static_cast<size_t>(nrhs) * kScalars * sizeof(double),
                                        hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return set_error(WD_ERR_DEVICE, "wilson: scalar copy: %s", hipGetErrorString(e));
    const hipError_t e2 = hipStreamSynchronize(st);
    if (e2 != hipSuccess) return set_error(WD_ERR_DEVICE, "wilson: device error: %s", hipGetErrorString(e2));
    return WD_OK;
  }
};

}  // namespace
}  // namespace wd

using namespace wd;

extern "C" {

size_t wilson_workspace_bytes(const int32_t dims[4], int32_t nrhs, int32_t inner, int32_t eo) {
  long V = 0;
  if (check_dims(dims, &V) != WD_OK || nrhs < 1 || nrhs > kMaxRhs) return 0;
  if (inner != WD_FP64 && inner != WD_FP32 && inner != WD_FP16) return 0;
  if (eo && check_even_dims(dims) != WD_OK) return 0;
  return ws_layout(dims, nrhs, inner, eo != 0).bytes;
}

int cg_solve_wilson(const wd_gauge* g_hi, const wd_gauge* g_lo, const double* masses_host, int32_t nrhs,
                    const void* b_dev, void* x_dev, const wd_cg_params* params, wd_cg_stats* stats_host,
                    void* ws_dev, size_t ws_bytes, hipStream_t stream) {
  try {
    clear_error();
    const auto t_start = std::chrono::steady_clock::now();
    int rc = check_gauge(g_hi);
    if (rc != WD_OK) return rc;
    if (g_hi->prec != WD_FP64) return set_error(WD_ERR_INVALID_ARG, "g_hi must be an FP64 gauge field");
    const bool eo = g_hi->eo != 0;
    if (params == nullptr || masses_host == nullptr)
      return set_error(WD_ERR_INVALID_ARG, "params and masses_host must not be NULL");
    const wd_cg_params& p = *params;
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(WD_ERR_UNSUPPORTED, "nrhs %d outside 1..%d", nrhs, kMaxRhs);
    if (!(p.tol > 0.0) || p.max_iter < 1 || p.check_every < 1)
      return set_error(WD_ERR_INVALID_ARG, "need tol > 0, max_iter >= 1, check_every >= 1");
    if (p.inner != WD_FP64 && p.inner != WD_FP32 && p.inner != WD_FP16)
      return set_error(WD_ERR_INVALID_ARG, "unknown inner precision %d", p.inner);
    if (p.inner != WD_FP64) {
      if ((rc = check_gauge(g_lo)) != WD_OK) return rc;
      if ((rc = check_layout(g_lo, g_hi->eo, "cg_solve_wilson (g_lo like g_hi)")) != WD_OK) return rc;
      if (g_lo->prec != p.inner)
        return set_error(WD_ERR_INVALID_ARG, "g_lo must be a gauge field of the inner precision %d", p.inner);
      for (int i = 0; i < 4; ++i)
        if (g_lo->dims[i] != g_hi->dims[i]) return set_error(WD_ERR_SHAPE, "g_lo and g_hi have different lattices");
      if (!(p.delta > 0.0 && p.delta < 1.0)) return set_error(WD_ERR_INVALID_ARG, "delta must lie in (0, 1)");
    }
    for (int k = 0; k < nrhs; ++k) {
      if (!std::isfinite(masses_host[k])) return set_error(WD_ERR_INVALID_ARG, "mass %d is not finite", k);
      if (eo && masses_host[k] == -4.0)
        return set_error(WD_ERR_INVALID_ARG, "mass %d is -4: the Schur complement divides by 4 + m", k);
    }
    const long V = g_hi->V;
    const size_t vec = static_cast<size_t>(packed_sites(V)) * nrhs * spinor_site_bytes(WD_FP64);
    if ((rc = check_device_range(b_dev, vec, "b_dev")) != WD_OK) return rc;
    if ((rc = check_device_range(x_dev, vec, "x_dev")) != WD_OK) return rc;
    const WsLayout lay = ws_layout(g_hi->dims, nrhs, p.inner, eo);
    if (ws_bytes < lay.bytes) return set_error(WD_ERR_INVALID_ARG, "ws_bytes %zu < %zu needed", ws_bytes, lay.bytes);
    if ((rc = check_device_range(ws_dev, lay.bytes, "ws_dev")) != WD_OK) return rc;
    if (overlaps(b_dev, vec, x_dev, vec) || overlaps(b_dev, vec, ws_dev, lay.bytes) ||
        overlaps(x_dev, vec, ws_dev, lay.bytes))
      return set_error(WD_ERR_INVALID_ARG, "b_dev, x_dev and ws_dev must not overlap");

    Solver sv{g_hi, p.inner != WD_FP64 ? g_lo : g_hi, masses_host, nrhs, b_dev, x_dev, ws_dev, stream, eo, lay,
              RhsSet{}, V, V / 2};
    sv.all.n = nrhs;
    for (int k = 0; k < nrhs; ++k) sv.all.idx[k] = k;
    if ((rc = sv.prepare()) != WD_OK) return rc;
    if (eo && p.x0_given && (rc = sv.split_x()) != WD_OK) return rc;

    int iters[kMaxRhs] = {}, updates[kMaxRhs] = {}, status[kMaxRhs] = {};
    double res[kMaxRhs] = {};
    double host[kMaxRhs * kScalars];
    wd_cg_stats cg[kMaxRhs];
    wd_cg_params prm = p;
    int used = 0;
    int worst = WD_OK;
    for (int round = 0; round < kMaxRounds; ++round) {
      prm.x0_given = (round > 0 || p.x0_given) ? 1 : 0;
      prm.max_iter = p.max_iter - used;
      rc = solve_sync(sv.ghi, sv.glo, masses_host, nrhs, at(ws_dev, lay.bn), eo ? at(ws_dev, lay.xo) : x_dev, prm,
                      cg, at(ws_dev, lay.cg), stream, nullptr);
      if (rc != WD_OK && rc != WD_ERR_NOT_CONVERGED && rc != WD_ERR_NUMERIC) return rc;
      int most = 0;
      for (int k = 0; k < nrhs; ++k) {
        iters[k] += cg[k].iters;
        updates[k] += cg[k].reliable_updates;
        most = cg[k].iters > most ? cg[k].iters : most;
      }
      used += most;
      if (eo && (rc = sv.finish_x()) != WD_OK) return rc;
      if ((rc = sv.residual(host)) != WD_OK) return rc;
      double worst_ratio = 0.0;
      worst = WD_OK;
      for (int k = 0; k < nrhs; ++k) {
        const double b2 = host[k * kScalars + kB2];
        const double r2 = host[k * kScalars + kRrTrue];
        res[k] = b2 > 0.0 ? std::sqrt(r2 / b2) : 0.0;
        status[k] = cg[k].status;
        if (!std::isfinite(res[k])) status[k] = WD_ERR_NUMERIC;
        if (status[k] == WD_OK && res[k] > p.tol) {
          status[k] = WD_ERR_NOT_CONVERGED;
          worst_ratio = res[k] / p.tol > worst_ratio ? res[k] / p.tol : worst_ratio;
        }
        if (status[k] != WD_OK && (worst == WD_OK || status[k] == WD_ERR_NUMERIC)) worst = status[k];
      }
      // done, failed, out of iterations, or the system's residual above tol
      // with CG converged: tighten CG's tolerance by the ratio and resume
      bool resume = worst_ratio > 0.0 && used < p.max_iter;
      for (int k = 0; k < nrhs; ++k)
        if (status[k] == WD_ERR_NUMERIC || (cg[k].status != WD_OK)) resume = false;
      if (!resume) break;
      prm.tol = prm.tol / (2.0 * worst_ratio);
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (stats_host != nullptr)
      for (int k = 0; k < nrhs; ++k) {
        stats_host[k].status = status[k];
        stats_host[k].iters = iters[k];
        stats_host[k].reliable_updates = updates[k];
        stats_host[k].reserved = 0;
        stats_host[k].true_rel_residual = res[k];
        stats_host[k].seconds = secs;
      }
    if (worst == WD_ERR_NOT_CONVERGED)
      set_error(worst, "cg_solve_wilson: |b - D x| / |b| above %g after %d iterations", p.tol, used);
    else if (worst == WD_ERR_NUMERIC)
      set_error(worst, "cg_solve_wilson: non-finite or non-positive value in the iteration");
    return worst;
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in cg_solve_wilson");
  }
}

}  // extern "C"
