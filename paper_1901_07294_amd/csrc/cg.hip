// Conjugate gradient on the normal equations D^dag D x = b, plain FP64 or
// with FP32 inner iterations and FP64 reliable updates.
//
// The paper (Sec. II-A) names iterative solvers such as conjugate gradient as
// where lattice QCD spends its time, dominated by the Dirac operator applied
// to a quark field; its related work cites mixed-precision GPU solvers. Here
// A = D^dag D = Q^2 with the Hermitian Q = gamma5 D, so one CG iteration is two
// dslash applications (gamma5 folded into their epilogue) and <p, A p> =
// |Q p|^2. With FP32 inner iterations the solution is accumulated in FP64, and
// whenever the iterated FP32 residual has fallen by the factor delta since the
// last true residual (or claims convergence), the residual is recomputed in
// FP64 as b - A x ("reliable update") and the FP32 residual restarted from it.
// Convergence is always judged on that FP64 true residual.
//
// Scalars (alpha, beta, <r,r>) stay on the device; the host reads them only
// every check_every iterations. All right-hand sides of a call iterate in
// lock step, each with its own mass and scalars; a converged one leaves the
// set of launched right-hand sides.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "blas.h"
#include "fields.h"
#include "wd_internal.h"

namespace wd {
namespace {

size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

struct Workspace {
  size_t bytes = 0;
  // offsets
  size_t r_hi = 0, t_hi = 0, r = 0, p = 0, t = 0, ap = 0, partials = 0, scal = 0;
};

// Layout of the caller's workspace. Plain FP64 CG keeps r, p, t, Ap in FP64
// (the true-residual recompute reuses t and Ap); mixed CG adds FP64 r and t.
Workspace layout(long V, int nrhs, int inner) {
  Workspace w;
  const size_t hi = align256(static_cast<size_t>(packed_sites(V)) * nrhs * spinor_site_bytes(WD_FP64));
  const size_t lo = align256(static_cast<size_t>(packed_sites(V)) * nrhs * spinor_site_bytes(inner));
  size_t o = 0;
  if (inner == WD_FP32) {
    w.r_hi = o; o += hi;
    w.t_hi = o; o += hi;
  }
  w.r = o; o += lo;
  w.p = o; o += lo;
  w.t = o; o += lo;
  w.ap = o; o += lo;
  if (inner != WD_FP32) {
    w.r_hi = w.r;
    w.t_hi = w.t;
  }
  w.partials = o; o += align256(static_cast<size_t>(nrhs) * kMaxPartials * sizeof(double));
  w.scal = o; o += align256(static_cast<size_t>(nrhs) * kScalars * sizeof(double));
  w.bytes = o;
  return w;
}

char* at(void* base, size_t off) { return static_cast<char*>(base) + off; }

class Solver {
 public:
  Solver(const wd_gauge* ghi, const wd_gauge* glo, const double* masses, int nrhs, const void* b,
         void* x, const wd_cg_params& prm, void* ws, hipStream_t st)
      : ghi_(ghi), glo_(glo ? glo : ghi), masses_(masses), nrhs_(nrhs), b_(b), x_(x), prm_(prm),
        ws_(ws), st_(st) {
    V_ = ghi->V;
    inner_ = prm.inner;
    nhi_ = packed_sites(V_) * 12;
    nlo_ = packed_sites(V_) * (inner_ == WD_FP64 ? 12 : 6);
    lay_ = layout(V_, nrhs, inner_);
    partials_ = reinterpret_cast<double*>(at(ws_, lay_.partials));
    scal_ = reinterpret_cast<double*>(at(ws_, lay_.scal));
    host_scal_.assign(static_cast<size_t>(nrhs) * kScalars, 0.0);
  }

  int run(wd_cg_stats* stats) {
    const auto t_start = std::chrono::steady_clock::now();
    std::vector<int> status(nrhs_, WD_PENDING), iters(nrhs_, 0), updates(nrhs_, 0);
    RhsSet all = set_of_all();
    int rc = WD_OK;

#define WD_TRY(expr)                           \
  do {                                         \
    rc = (expr);                               \
    if (rc != WD_OK) return finish(rc, stats); \
  } while (0)

    WD_TRY(launch_status(blas_zero(scal_, WD_FP64, kScalars / 2, all, st_), "cg: scalars"));
    WD_TRY(launch_status(blas_norm2(b_, WD_FP64, nhi_, V_, all, partials_, scal_, kFinNorm, st_), "cg: |b|"));
    if (prm_.x0_given) {
      WD_TRY(true_residual(all));
    } else {
      WD_TRY(launch_status(blas_zero(x_, WD_FP64, nhi_, all, st_), "cg: x0"));
      WD_TRY(launch_status(blas_copy(at(ws_, lay_.r_hi), b_, WD_FP64, nhi_, all, st_), "cg: r0"));
      WD_TRY(launch_status(blas_norm2(at(ws_, lay_.r_hi), WD_FP64, nhi_, V_, all, partials_, scal_,
                                      kFinTrueRr, st_), "cg: |r0|"));
      if (inner_ == WD_FP32)
        WD_TRY(launch_status(blas_demote(at(ws_, lay_.r), at(ws_, lay_.r_hi), nlo_, nhi_, all, st_), "cg: demote"));
    }
    WD_TRY(launch_status(blas_copy(at(ws_, lay_.p), at(ws_, lay_.r), inner_, nlo_, all, st_), "cg: p0"));
    WD_TRY(read_scalars());

    // right-hand sides that are already solved (b = 0, or x0 good enough)
    std::vector<int> active;
    for (int k = 0; k < nrhs_; ++k) {
      const double b2 = sc(k, kB2), rr = sc(k, kRr);
      if (!std::isfinite(b2) || !std::isfinite(rr)) {
        status[k] = WD_ERR_NUMERIC;
      } else if (b2 == 0.0 || rr <= tol2(k)) {
        status[k] = WD_OK;
      } else {
        active.push_back(k);
      }
    }

    int it = 0;
    while (!active.empty() && it < prm_.max_iter) {
      const RhsSet set = set_of(active);
      WD_TRY(iteration(set));
      ++it;
      for (int k : active) iters[k] = it;
      if (it % prm_.check_every != 0 && it < prm_.max_iter) continue;

      WD_TRY(read_scalars());
      std::vector<int> refresh, keep;
      for (int k : active) {
        if (sc(k, kFlag) != 0.0 || !std::isfinite(sc(k, kRr))) {
          status[k] = WD_ERR_NUMERIC;
          continue;
        }
        const double rr = sc(k, kRr);
        const bool small = rr <= tol2(k);
        const bool dropped = inner_ == WD_FP32 && rr < prm_.delta * prm_.delta * sc(k, kRrMax);
        if (small || dropped || it >= prm_.max_iter) refresh.push_back(k);
        keep.push_back(k);
      }
      active = keep;
      if (refresh.empty()) continue;
      const RhsSet rs = set_of(refresh);
      WD_TRY(true_residual(rs));
      WD_TRY(read_scalars());
      std::vector<int> still;
      for (int k : active) {
        const bool refreshed = std::find(refresh.begin(), refresh.end(), k) != refresh.end();
        if (refreshed) ++updates[k];
        if (refreshed && sc(k, kRrTrue) <= tol2(k)) {
          status[k] = WD_OK;
        } else if (refreshed && (sc(k, kFlag) != 0.0 || !std::isfinite(sc(k, kRrTrue)))) {
          status[k] = WD_ERR_NUMERIC;
        } else {
          still.push_back(k);
        }
      }
      active = still;
    }
    for (int k : active) status[k] = WD_ERR_NOT_CONVERGED;

    WD_TRY(read_scalars());
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    int worst = WD_OK;
    for (int k = 0; k < nrhs_; ++k) {
      if (stats != nullptr) {
        stats[k].status = status[k];
        stats[k].iters = iters[k];
        stats[k].reliable_updates = updates[k];
        const double b2 = sc(k, kB2);
        stats[k].true_rel_residual = b2 > 0.0 ? std::sqrt(sc(k, kRrTrue) / b2) : 0.0;
        stats[k].seconds = secs;
      }
      if (status[k] != WD_OK && (worst == WD_OK || status[k] == WD_ERR_NUMERIC)) worst = status[k];
    }
    if (worst == WD_ERR_NOT_CONVERGED)
      set_error(worst, "cg_solve_normal: not converged to %g within %d iterations", prm_.tol,
                prm_.max_iter);
    else if (worst == WD_ERR_NUMERIC)
      set_error(worst, "cg_solve_normal: non-finite or non-positive value in the iteration");
    return worst;
#undef WD_TRY
  }

 private:
  // One CG iteration on the right-hand sides of set (inner precision).
  int iteration(const RhsSet& set) {
    const size_t vb = static_cast<size_t>(nlo_) * 16;
    for (int i = 0; i < set.n; ++i) {
      const int k = set.idx[i];
      const size_t off = k * vb;
      int rc = launch_status(launch_dslash(glo_, masses_[k], at(ws_, lay_.p + off),
                                           at(ws_, lay_.t + off), WD_FLAG_GAMMA5, st_), "cg: Q p");
      if (rc != WD_OK) return rc;
      rc = launch_status(launch_dslash(glo_, masses_[k], at(ws_, lay_.t + off),
                                       at(ws_, lay_.ap + off), WD_FLAG_GAMMA5, st_), "cg: Q Q p");
      if (rc != WD_OK) return rc;
    }
    int rc = launch_status(blas_norm2(at(ws_, lay_.t), inner_, nlo_, V_, set, partials_, scal_,
                                      kFinPap, st_), "cg: pAp");
    if (rc != WD_OK) return rc;
    rc = launch_status(blas_update_xr(x_, at(ws_, lay_.r), at(ws_, lay_.p), at(ws_, lay_.ap), inner_,
                                      nlo_, nhi_, V_, set, partials_, scal_, st_), "cg: x, r");
    if (rc != WD_OK) return rc;
    return launch_status(blas_update_p(at(ws_, lay_.p), at(ws_, lay_.r), inner_, nlo_, set, scal_, st_),
                         "cg: p");
  }

  // r_hi = b - A x in FP64 (and the inner residual restarted from it).
  int true_residual(const RhsSet& set) {
    const size_t vb = static_cast<size_t>(nhi_) * 16;
    for (int i = 0; i < set.n; ++i) {
      const int k = set.idx[i];
      const size_t off = k * vb;
      int rc = launch_status(launch_dslash(ghi_, masses_[k], at(x_, off), at(ws_, lay_.t_hi + off),
                                           WD_FLAG_GAMMA5, st_), "cg: Q x");
      if (rc != WD_OK) return rc;
      rc = launch_status(launch_dslash(ghi_, masses_[k], at(ws_, lay_.t_hi + off),
                                       at(ws_, lay_.r_hi + off), WD_FLAG_GAMMA5, st_), "cg: Q Q x");
      if (rc != WD_OK) return rc;
    }
    int rc = launch_status(blas_residual(at(ws_, lay_.r_hi), b_, nhi_, V_, set, partials_, scal_, st_),
                           "cg: b - A x");
    if (rc != WD_OK) return rc;
    if (inner_ == WD_FP32)
      rc = launch_status(blas_demote(at(ws_, lay_.r), at(ws_, lay_.r_hi), nlo_, nhi_, set, st_),
                         "cg: demote");
    return rc;
  }

  int read_scalars() {
    hipError_t e = hipMemcpyAsync(host_scal_.data(), scal_, host_scal_.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, st_);
    if (e == hipSuccess) e = hipStreamSynchronize(st_);
    if (e != hipSuccess) return set_error(WD_ERR_DEVICE, "cg: device error: %s", hipGetErrorString(e));
    return WD_OK;
  }

  int finish(int rc, wd_cg_stats* stats) {
    if (stats != nullptr)
      for (int k = 0; k < nrhs_; ++k) stats[k].status = rc;
    return rc;
  }

  double sc(int k, int i) const { return host_scal_[static_cast<size_t>(k) * kScalars + i]; }
  double tol2(int k) const { return prm_.tol * prm_.tol * sc(k, kB2); }

  RhsSet set_of_all() const {
    RhsSet s{};
    s.n = nrhs_;
    for (int k = 0; k < nrhs_; ++k) s.idx[k] = k;
    return s;
  }
  static RhsSet set_of(const std::vector<int>& ks) {
    RhsSet s{};
    s.n = static_cast<int>(ks.size());
    for (size_t i = 0; i < ks.size(); ++i) s.idx[i] = ks[i];
    return s;
  }

  const wd_gauge* ghi_;
  const wd_gauge* glo_;
  const double* masses_;
  int nrhs_;
  const void* b_;
  void* x_;
  wd_cg_params prm_;
  void* ws_;
  hipStream_t st_;
  long V_ = 0, nhi_ = 0, nlo_ = 0;
  int inner_ = WD_FP64;
  Workspace lay_;
  double* partials_ = nullptr;
  double* scal_ = nullptr;
  std::vector<double> host_scal_;
};

}  // namespace
}  // namespace wd

using namespace wd;

extern "C" {

size_t cg_workspace_bytes(const int32_t dims[4], int32_t nrhs, int32_t inner) {
  long V = 0;
  if (check_dims(dims, &V) != WD_OK || nrhs < 1 || nrhs > kMaxRhs) return 0;
  if (inner != WD_FP64 && inner != WD_FP32) return 0;
  return layout(V, nrhs, inner).bytes;
}

int cg_solve_normal(const wd_gauge* g_hi, const wd_gauge* g_lo, const double* masses_host,
                    int32_t nrhs, const void* b_dev, void* x_dev, const wd_cg_params* params,
                    wd_cg_stats* stats_host, void* ws_dev, size_t ws_bytes, hipStream_t stream) {
  try {
    clear_error();
    int rc = check_gauge(g_hi);
    if (rc != WD_OK) return rc;
    if (g_hi->prec != WD_FP64) return set_error(WD_ERR_INVALID_ARG, "g_hi must be an FP64 gauge field");
    if (params == nullptr || masses_host == nullptr)
      return set_error(WD_ERR_INVALID_ARG, "params and masses_host must not be NULL");
    const wd_cg_params& p = *params;
    if (nrhs < 1 || nrhs > kMaxRhs)
      return set_error(WD_ERR_UNSUPPORTED, "nrhs %d outside 1..%d", nrhs, kMaxRhs);
    if (!(p.tol > 0.0) || p.max_iter < 1 || p.check_every < 1)
      return set_error(WD_ERR_INVALID_ARG, "need tol > 0, max_iter >= 1, check_every >= 1");
    if (p.inner != WD_FP64 && p.inner != WD_FP32)
      return set_error(WD_ERR_UNSUPPORTED, "inner precision %d not supported", p.inner);
    if (p.inner == WD_FP32) {
      if ((rc = check_gauge(g_lo)) != WD_OK) return rc;
      if (g_lo->prec != WD_FP32) return set_error(WD_ERR_INVALID_ARG, "g_lo must be an FP32 gauge field");
      for (int i = 0; i < 4; ++i)
        if (g_lo->dims[i] != g_hi->dims[i])
          return set_error(WD_ERR_SHAPE, "g_lo and g_hi have different lattices");
      if (!(p.delta > 0.0 && p.delta < 1.0))
        return set_error(WD_ERR_INVALID_ARG, "delta must lie in (0, 1)");
    }
    for (int k = 0; k < nrhs; ++k)
      if (!std::isfinite(masses_host[k]))
        return set_error(WD_ERR_INVALID_ARG, "mass %d is not finite", k);
    const long V = g_hi->V;
    const size_t vec = static_cast<size_t>(packed_sites(V)) * nrhs * spinor_site_bytes(WD_FP64);
    if ((rc = check_device_range(b_dev, vec, "b_dev")) != WD_OK) return rc;
    if ((rc = check_device_range(x_dev, vec, "x_dev")) != WD_OK) return rc;
    const size_t need = layout(V, nrhs, p.inner).bytes;
    if (ws_bytes < need) return set_error(WD_ERR_INVALID_ARG, "ws_bytes %zu < %zu needed", ws_bytes, need);
    if ((rc = check_device_range(ws_dev, need, "ws_dev")) != WD_OK) return rc;
    if (overlaps(b_dev, vec, x_dev, vec) || overlaps(b_dev, vec, ws_dev, need) ||
        overlaps(x_dev, vec, ws_dev, need))
      return set_error(WD_ERR_INVALID_ARG, "b_dev, x_dev and ws_dev must not overlap");
    Solver s(g_hi, p.inner == WD_FP32 ? g_lo : g_hi, masses_host, nrhs, b_dev, x_dev, p, ws_dev, stream);
    return s.run(stats_host);
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in cg_solve_normal");
  }
}

}  // extern "C"
