// Conjugate gradient on the normal equations D^dag D x = b, plain FP64 or
// with FP32 or FP16-storage inner iterations and FP64 reliable updates.
//
// The paper (Sec. II-A) names iterative solvers such as conjugate gradient as
// where lattice QCD spends its time, dominated by the Dirac operator applied
// to a quark field; its related work cites mixed-precision GPU solvers. Here
// A = D^dag D = Q^2 with the Hermitian Q = gamma5 D, so one CG iteration is two
// dslash applications (gamma5 folded into their epilogue) and <p, A p> =
// |Q p|^2. With lower-precision inner iterations (FP32, or FP16 storage with
// FP32 arithmetic) the solution increments are accumulated in an FP32 vector,
// and whenever the iterated residual has fallen by the factor delta since the
// last true residual (or claims convergence), that vector is added into the
// FP64 solution, the residual is recomputed in FP64 as b - A x ("reliable
// update") and the inner residual restarted from it.
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
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "cg_engine.h"
#include "eo.h"
#include "fields.h"

// Workspace of cg_solve_normal_noalloc (see the note above scratch_address).
static __device__ __align__(256) unsigned char scratch[WD_NOALLOC_SCRATCH_BYTES];

namespace wd {

size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Plain FP64 CG keeps r, p, t, Ap in FP64 (the true-residual recompute reuses
// r and t); mixed CG adds FP64 r and t and the FP32 solution accumulator.
CgLayout cg_layout(const int32_t dims[4], int slots, int inner, bool eo) {
  CgLayout w;
  const long V = static_cast<long>(dims[0]) * dims[1] * dims[2] * dims[3] / (eo ? 2 : 1);
  w.nslices = eo ? 0 : cg_fuse_slices(dims, inner);
  const size_t hi = align256(static_cast<size_t>(packed_sites(V)) * slots * spinor_site_bytes(WD_FP64));
  const size_t lo = align256(static_cast<size_t>(packed_sites(V)) * slots * spinor_site_bytes(inner));
  const size_t acc = align256(static_cast<size_t>(packed_sites(V)) * slots * spinor_site_bytes(WD_FP32));
  size_t o = 0;
  if (inner != WD_FP64) {
    w.r_hi = o; o += hi;
    w.t_hi = o; o += hi;
    w.x_lo = o; o += acc;
  }
  w.r = o; o += lo;
  w.p = o; o += lo;
  w.p2 = w.p;
  if (w.nslices > 0 && inner != WD_FP64) {  // the direction of an iteration whose x update waits
    w.p2 = o;
    o += lo;
  }
  w.t = o; o += lo;
  if (w.nslices == 0 || inner == WD_FP64) {  // FP64 keeps A p (the update is not fused)
    w.ap = o;
    o += lo;
  }
  if (inner == WD_FP64) {
    w.r_hi = w.r;
    w.t_hi = w.t;
  }
  if (eo) {
    w.e_lo = o; o += lo;
    if (inner != WD_FP64) {
      w.e_hi = o;
      o += hi;
    } else {
      w.e_hi = w.e_lo;
    }
  }
  w.partials = o; o += align256(static_cast<size_t>(slots) * kMaxPartials * sizeof(double));
  w.pap = o; o += align256(static_cast<size_t>(slots) * kMaxPartials * sizeof(double));
  w.scal = o; o += align256(static_cast<size_t>(slots) * kScalars * sizeof(double));
  w.rr = o; o += align256(static_cast<size_t>(slots) * w.nslices * sizeof(double));
  w.paps = o; o += align256(static_cast<size_t>(slots) * w.nslices * sizeof(double));
  w.bytes = o;
  return w;
}

CgAction cg_check(const double* sc, double tol, bool mixed, double delta, bool at_max) {
  const double rr = sc[kRr];
  if (sc[kFlag] != 0.0 || !std::isfinite(rr)) return kCgNumeric;
  const bool small = rr <= tol * tol * sc[kB2];
  const bool dropped = mixed && rr < delta * delta * sc[kRrMax];
  return (small || dropped || at_max) ? kCgRefresh : kCgContinue;
}

CgOutcome cg_after_refresh(const double* sc, double tol, bool at_max) {
  if (sc[kRrTrue] <= tol * tol * sc[kB2]) return kCgConverged;
  if (sc[kFlag] != 0.0 || !std::isfinite(sc[kRrTrue])) return kCgFailed;
  return at_max ? kCgNotConverged : kCgKeepGoing;
}

namespace {
char* at(void* base, size_t off) { return static_cast<char*>(base) + off; }
}  // namespace

CgEngine::CgEngine(const wd_gauge* ghi, const wd_gauge* glo, int inner, int slots, const void* b,
                   void* x, void* ws, hipStream_t st)
    : ghi_(ghi), glo_(glo ? glo : ghi), inner_(inner), slots_(slots), b_(b), x_(x), ws_(ws), st_(st) {
  eo_ = ghi->eo != 0;
  V_ = eo_ ? ghi->V / 2 : ghi->V;
  nhi_ = packed_sites(V_) * 12;
  nlo_ = inner_ == WD_FP64 ? spinor_units<double>(V_)
                           : inner_ == WD_FP32 ? spinor_units<float>(V_) : spinor_units<_Float16>(V_);
  n32_ = spinor_units<float>(V_);
  lay_ = cg_layout(ghi->dims, slots, inner_, eo_);
  partials_ = reinterpret_cast<double*>(at(ws_, lay_.partials));
  rr_ = reinterpret_cast<double*>(at(ws_, lay_.rr));
  paps_ = reinterpret_cast<double*>(at(ws_, lay_.paps));
  pap_ = reinterpret_cast<double*>(at(ws_, lay_.pap));
  scal_ = reinterpret_cast<double*>(at(ws_, lay_.scal));
}

int CgEngine::apply_q(const wd_gauge* g, const double* m, const RhsSet& set, const void* in, void* tmp,
                      void* out, const char* what) const {
  return launch_status(eo_ ? launch_schur_q(g, m, set, in, tmp, out, st_)
                           : launch_dslash_multi(g, m, set.n, set.idx, in, out, WD_FLAG_GAMMA5, st_),
                       what);
}

int CgEngine::start(const RhsSet& set, bool x0_given) {
  int rc = launch_status(blas_zero(scal_, WD_FP64, kScalars / 2, set, st_), "cg: scalars");
  if (rc == WD_OK)
    rc = launch_status(blas_norm2(b_, WD_FP64, nhi_, V_, set, partials_, scal_, kFinNorm, st_), "cg: |b|");
  if (rc == WD_OK && inner_ != WD_FP64)
    rc = launch_status(blas_zero(at(ws_, lay_.x_lo), WD_FP32, n32_, set, st_), "cg: x_lo");
  if (rc != WD_OK) return rc;
  if (x0_given) {
    rc = refresh(set);
  } else {
    rc = launch_status(blas_zero(x_, WD_FP64, nhi_, set, st_), "cg: x0");
    if (rc == WD_OK)
      rc = launch_status(blas_copy(at(ws_, lay_.r_hi), b_, WD_FP64, nhi_, set, st_), "cg: r0");
    if (rc == WD_OK)
      rc = launch_status(blas_norm2(at(ws_, lay_.r_hi), WD_FP64, nhi_, V_, set, partials_, scal_,
                                    kFinTrueRr, st_), "cg: |r0|");
    if (rc == WD_OK && inner_ != WD_FP64)
      rc = launch_status(blas_demote(at(ws_, lay_.r), at(ws_, lay_.r_hi), inner_, nlo_, nhi_, V_, set, st_),
                         "cg: demote");
  }
  if (rc != WD_OK) return rc;
  return launch_status(blas_copy(at(ws_, lay_.p), at(ws_, lay_.r), inner_, nlo_, set, st_), "cg: p0");
}

int CgEngine::chunk(const RhsSet& set, int n) {
  int rc = WD_OK;
  for (int j = 0; j < n && rc == WD_OK; ++j) rc = iterate(set, j, n);
  return rc;
}

int CgEngine::iterate(const RhsSet& set, int j, int n) {
  double m[kMaxRhs];
  for (int i = 0; i < set.n; ++i) m[i] = masses_[set.idx[i]];
  if (lay_.nslices > 0 && inner_ == WD_FP64) {
    // t = Q p with <p, A p> = |t|^2 summed per tile slice in the same launch;
    // A p = Q t; then r -= alpha A p (reducing those sums to alpha), and x and
    // p together (p is read once)
    CgFuse f{};
    f.mode = kCgNorm;
    f.rr = paps_;
    f.nslices = lay_.nslices;
    int rc = launch_status(launch_dslash_cg(glo_, m, set.n, set.idx, at(ws_, lay_.p), at(ws_, lay_.t), f,
                                            st_), "cg: Q p with |Q p|^2");
    if (rc == WD_OK)
      rc = launch_status(launch_dslash_multi(glo_, m, set.n, set.idx, at(ws_, lay_.t), at(ws_, lay_.ap),
                                             WD_FLAG_GAMMA5, st_), "cg: Q Q p");
    int nrr = 0;
    if (rc == WD_OK)
      rc = launch_status(blas_update_r(at(ws_, lay_.r), at(ws_, lay_.ap), nlo_, V_, set, paps_,
                                       lay_.nslices, partials_, &nrr, scal_, st_), "cg: r");
    if (rc == WD_OK)
      rc = launch_status(blas_update_xp(x_, at(ws_, lay_.p), at(ws_, lay_.r), nlo_, set, partials_, nrr,
                                        scal_, st_), "cg: x, p");
    return rc;
  }
  if (lay_.nslices > 0) {
    // t = Q p, with <p, A p> = |t|^2 summed per tile slice in the same launch;
    // then Q t = A p used at once for r -= alpha A p, with <r, r> per tile
    // slice (A p is never stored); then x += alpha p and p = r + beta p
    // together (p is read once). In iteration j = 0, 2, ... of the chunk,
    // unless it is the last, p moves to p2 and x += alpha p waits for
    // iteration j + 1, which adds both directions' terms and moves p back
    // (x_lo is read and written once per two iterations).
    void* const p1 = at(ws_, lay_.p);
    void* const p2 = at(ws_, lay_.p2);
    const bool second = (j & 1) != 0;
    const int kind = second ? kXpPair : (j + 1 < n ? kXpDefer : kXpNow);
    void* const pc = second ? p2 : p1;
    CgFuse f{};
    f.mode = kCgNorm;
    f.rr = paps_;
    f.nslices = lay_.nslices;
    int rc = launch_status(launch_dslash_cg(glo_, m, set.n, set.idx, pc, at(ws_, lay_.t), f, st_),
                           "cg: Q p with |Q p|^2");
    f.mode = kCgUpdate;
    f.r = at(ws_, lay_.r);
    f.pap = paps_;
    f.npap = lay_.nslices;
    f.rr = rr_;
    f.scal = scal_;
    if (rc == WD_OK)
      rc = launch_status(launch_dslash_cg(glo_, m, set.n, set.idx, at(ws_, lay_.t), nullptr, f, st_),
                         "cg: Q Q p with r");
    if (rc == WD_OK)
      rc = launch_status(blas_update_xp_lo(at(ws_, lay_.x_lo), kind == kXpDefer ? p2 : p1, pc, p1,
                                           at(ws_, lay_.r), kind, inner_, nlo_, n32_, V_, set, rr_,
                                           lay_.nslices, scal_, st_),
                         "cg: x, p");
    return rc;
  }
  int rc = apply_q(glo_, m, set, at(ws_, lay_.p), at(ws_, lay_.e_lo), at(ws_, lay_.t), "cg: Q p");
  if (rc == WD_OK) rc = apply_q(glo_, m, set, at(ws_, lay_.t), at(ws_, lay_.e_lo), at(ws_, lay_.ap), "cg: Q Q p");
  // <p, A p> = |Q p|^2: partial sums here, reduced (with alpha) inside the r update
  int npap = 0;
  if (rc == WD_OK)
    rc = launch_status(blas_norm2_partials(at(ws_, lay_.t), inner_, nlo_, V_, set, pap_, &npap, st_),
                       "cg: pAp");
  // <r, r> likewise: partial sums in the r update, reduced (with beta) inside the p update
  int nrr = 0;
  if (inner_ == WD_FP64) {  // r first, then x and p together (p read once)
    if (rc == WD_OK)
      rc = launch_status(blas_update_r(at(ws_, lay_.r), at(ws_, lay_.ap), nlo_, V_, set, pap_, npap,
                                       partials_, &nrr, scal_, st_), "cg: r");
    if (rc == WD_OK)
      rc = launch_status(blas_update_xp(x_, at(ws_, lay_.p), at(ws_, lay_.r), nlo_, set, partials_, nrr,
                                        scal_, st_), "cg: x, p");
    return rc;
  }
  if (rc == WD_OK)
    rc = launch_status(blas_update_xr(at(ws_, lay_.x_lo), at(ws_, lay_.r),
                                      at(ws_, lay_.p), at(ws_, lay_.ap), inner_, nlo_, n32_, V_, set,
                                      pap_, npap, partials_, &nrr, scal_, st_), "cg: x, r");
  if (rc == WD_OK)
    rc = launch_status(blas_update_p(at(ws_, lay_.p), at(ws_, lay_.r), inner_, nlo_, V_, set, partials_,
                                     nrr, scal_, st_), "cg: p");
  return rc;
}

int CgEngine::refresh(const RhsSet& set) {
  double m[kMaxRhs];
  for (int i = 0; i < set.n; ++i) m[i] = masses_[set.idx[i]];
  int rc = WD_OK;
  if (inner_ != WD_FP64)  // the FP32 accumulator joins the FP64 solution
    rc = launch_status(blas_flush_x(x_, at(ws_, lay_.x_lo), n32_, nhi_, set, st_), "cg: flush x");
  if (rc == WD_OK) rc = apply_q(ghi_, m, set, x_, at(ws_, lay_.e_hi), at(ws_, lay_.t_hi), "cg: Q x");
  if (rc == WD_OK)
    rc = apply_q(ghi_, m, set, at(ws_, lay_.t_hi), at(ws_, lay_.e_hi), at(ws_, lay_.r_hi), "cg: Q Q x");
  if (rc != WD_OK) return rc;
  if (inner_ == WD_FP64)  // r_hi is the iteration's residual
    return launch_status(blas_residual(at(ws_, lay_.r_hi), b_, nhi_, V_, set, partials_, scal_, st_),
                         "cg: b - A x");
  // mixed: only the inner-precision residual is kept (r_hi holds A x)
  return launch_status(blas_residual_demote(at(ws_, lay_.r), b_, at(ws_, lay_.r_hi), inner_, nlo_, nhi_, V_,
                                            set, partials_, scal_, st_),
                       "cg: b - A x, demoted");
}

int CgEngine::fetch_scalars(double* host) const {
  const hipError_t e = hipMemcpyAsync(host, scal_, static_cast<size_t>(slots_) * kScalars * sizeof(double),
                                      hipMemcpyDeviceToHost, st_);
  if (e != hipSuccess) return set_error(WD_ERR_DEVICE, "cg: scalar copy: %s", hipGetErrorString(e));
  return WD_OK;
}

namespace {

// Chunks of CG iterations captured as HIP graphs and replayed: one graph per
// (set of active right-hand sides, chunk length). The scalars never leave the
// device inside a chunk, so a replay needs no host work between iterations.
// (The scalar copy after a chunk stays outside the graph: as the graph's last
// node it delayed the host's view of completion.)
class ChunkGraphs {
 public:
  explicit ChunkGraphs(hipStream_t st) : st_(st) {}
  ~ChunkGraphs() {
    for (auto& e : execs_) (void)hipGraphExecDestroy(e.second);
  }
  ChunkGraphs(const ChunkGraphs&) = delete;
  ChunkGraphs& operator=(const ChunkGraphs&) = delete;

  // n iterations of eng on set, captured the first time (set, n) is seen
  int run(CgEngine& eng, const RhsSet& set, int n) {
    std::vector<int> key(set.idx, set.idx + set.n);
    key.push_back(-n);
    auto it = execs_.find(key);
    if (it == execs_.end()) {
      hipError_t e = hipStreamBeginCapture(st_, hipStreamCaptureModeRelaxed);
      if (e != hipSuccess) return set_error(WD_ERR_DEVICE, "cg: graph capture: %s", hipGetErrorString(e));
      const int rc = eng.chunk(set, n);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(st_, &graph);
      hipGraphExec_t exec = nullptr;
      if (rc == WD_OK && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (graph != nullptr) (void)hipGraphDestroy(graph);
      if (rc != WD_OK) return rc;
      if (e != hipSuccess) return set_error(WD_ERR_DEVICE, "cg: graph: %s", hipGetErrorString(e));
      it = execs_.emplace(std::move(key), exec).first;
    }
    const hipError_t e = hipGraphLaunch(it->second, st_);
    return e == hipSuccess ? WD_OK : set_error(WD_ERR_DEVICE, "cg: graph launch: %s", hipGetErrorString(e));
  }

 private:
  hipStream_t st_;
  std::map<std::vector<int>, hipGraphExec_t> execs_;
};

// A stream of the library's own for graph capture (the caller's may be the
// null stream, which cannot be captured), ordered after the caller's work.
class OwnStream {
 public:
  explicit OwnStream(hipStream_t after) {
    if (hipStreamCreateWithFlags(&st_, hipStreamNonBlocking) != hipSuccess) { st_ = nullptr; return; }
    if (hipEventCreateWithFlags(&ev_, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev_, after) != hipSuccess || hipStreamWaitEvent(st_, ev_, 0) != hipSuccess)
      ok_ = false;
  }
  ~OwnStream() {
    if (st_ != nullptr) {
      (void)hipStreamSynchronize(st_);
      (void)hipStreamDestroy(st_);
    }
    if (ev_ != nullptr) (void)hipEventDestroy(ev_);
  }
  OwnStream(const OwnStream&) = delete;
  OwnStream& operator=(const OwnStream&) = delete;
  bool ok() const { return st_ != nullptr && ok_; }
  hipStream_t get() const { return st_; }

 private:
  hipStream_t st_ = nullptr;
  hipEvent_t ev_ = nullptr;
  bool ok_ = true;
};

// Page-locked host buffers for the scalars the synchronous solver reads after
// each chunk of iterations (a copy into pageable memory is staged through the
// runtime; with page-locked memory the graph-replayed 8^4 solve went from 5.2
// to 5.0 ms). Each holds kMaxRhs slots; buffers are kept for the life of the
// process and reused by later solves, except one whose last copy may not have
// completed (a device error), which is dropped.
class HostScalars {
 public:
  explicit HostScalars(bool take) {
    if (!take) return;
    {
      std::lock_guard<std::mutex> lk(mu());
      if (!pool().empty()) {
        p_ = pool().back();
        pool().pop_back();
      }
    }
    if (p_ == nullptr && hipHostMalloc(reinterpret_cast<void**>(&p_), kBytes, hipHostMallocPortable) != hipSuccess)
      p_ = nullptr;
    if (p_ != nullptr) std::memset(p_, 0, kBytes);
  }
  ~HostScalars() {
    if (p_ == nullptr || !reusable_) return;
    std::lock_guard<std::mutex> lk(mu());
    pool().push_back(p_);
  }
  HostScalars(const HostScalars&) = delete;
  HostScalars& operator=(const HostScalars&) = delete;
  double* get() const { return p_; }
  void drop() { reusable_ = false; }

 private:
  static constexpr size_t kBytes = sizeof(double) * kMaxRhs * kScalars;
  static std::mutex& mu() {
    static std::mutex m;
    return m;
  }
  static std::vector<double*>& pool() {
    static auto* v = new std::vector<double*>;  // never destroyed: process lifetime
    return *v;
  }
  double* p_ = nullptr;
  bool reusable_ = true;
};

// Waits for the stream by polling it: after a blocking wait the host takes
// tens of microseconds to wake up, during which the device idles, once per
// chunk of iterations. Ends when the stream's work has completed or failed.
// Used for eager chunks (24^4 FP16-storage inner 62.5-63.0 -> 65.2 solves/s,
// 8^4 FP32 inner 5.3 -> 4.9 ms per solve); after a graph replay polling
// measured slower than a blocking wait (8^4: 5.0 -> 5.4-6.1 ms), so replays
// keep the blocking wait.
hipError_t poll_stream(hipStream_t st) {
  for (;;) {
    const hipError_t e = hipStreamQuery(st);
    if (e != hipErrorNotReady) return e;
    std::this_thread::yield();
  }
}

}  // namespace

// Right-hand-side indices of a solve, in a fixed-capacity list (no heap use).
struct IdxList {
  int n = 0;
  int k[kMaxRhs] = {};
  void push(int v) { k[n++] = v; }
  bool has(int v) const {
    for (int i = 0; i < n; ++i)
      if (k[i] == v) return true;
    return false;
  }
  RhsSet set() const {
    RhsSet s{};
    s.n = n;
    for (int i = 0; i < n; ++i) s.idx[i] = k[i];
    return s;
  }
};

// The synchronous solver: all right-hand sides start together; every
// check_every iterations the host reads the scalars, recomputes the true
// residual of those that need it, and drops the finished ones. With
// use_graph, each chunk of iterations between two reads is a graph replay.
// host: where the scalars are read to (kMaxRhs * kScalars doubles), or null
// for a page-locked buffer from the pool.
int solve_sync(const wd_gauge* ghi, const wd_gauge* glo, const double* masses, int nrhs,
               const void* b, void* x, const wd_cg_params& prm, wd_cg_stats* stats, void* ws,
               hipStream_t caller, double* host) {
  const auto t_start = std::chrono::steady_clock::now();
  std::unique_ptr<OwnStream> own;
  if (prm.use_graph) {
    own = std::make_unique<OwnStream>(caller);
    if (!own->ok()) return set_error(WD_ERR_DEVICE, "cg: cannot create a stream for graph capture");
  }
  const hipStream_t st = own ? own->get() : caller;
  std::unique_ptr<ChunkGraphs> graphs;
  if (own) graphs = std::make_unique<ChunkGraphs>(st);
  CgEngine eng(ghi, glo, prm.inner, nrhs, b, x, ws, st);
  for (int k = 0; k < nrhs; ++k) eng.set_mass(k, masses[k]);
  HostScalars hs(host == nullptr);
  double* const scal = host != nullptr ? host : hs.get();
  if (scal == nullptr) return set_error(WD_ERR_NOMEM, "cg: cannot allocate page-locked host memory");
  auto sc = [&](int k) { return scal + static_cast<size_t>(k) * kScalars; };
  auto read = [&]() -> int {
    const int rc = eng.fetch_scalars(scal);
    if (rc != WD_OK) {
      hs.drop();
      return rc;
    }
    const hipError_t e = graphs ? hipStreamSynchronize(st) : poll_stream(st);
    if (e == hipSuccess) return WD_OK;
    hs.drop();
    return set_error(WD_ERR_DEVICE, "cg: device error: %s", hipGetErrorString(e));
  };
  int status[kMaxRhs], iters[kMaxRhs], updates[kMaxRhs];
  IdxList all;
  for (int k = 0; k < nrhs; ++k) {
    status[k] = WD_PENDING;
    iters[k] = updates[k] = 0;
    all.push(k);
  }
  const bool mixed = prm.inner != WD_FP64;

  int rc = eng.start(all.set(), prm.x0_given != 0);
  if (rc == WD_OK) rc = read();
  IdxList active;
  for (int k = 0; rc == WD_OK && k < nrhs; ++k) {
    const double b2 = sc(k)[kB2], rr = sc(k)[kRr];
    if (!std::isfinite(b2) || !std::isfinite(rr)) status[k] = WD_ERR_NUMERIC;
    else if (b2 == 0.0 || rr <= prm.tol * prm.tol * b2) status[k] = WD_OK;
    else active.push(k);
  }
  int it = 0;
  // Right-hand sides whose true residual was recomputed before the last chunk
  // without the host waiting for it (refresh_it: the iterations then). The
  // recompute leaves its scalars (kRrTrue, kFlag) to the next read; one that
  // has converged keeps its FP64 x from then (the chunk only added to x_lo,
  // which is never flushed again).
  IdxList unread;
  int refresh_it[kMaxRhs] = {};
  while (rc == WD_OK && active.n > 0 && it < prm.max_iter) {
    // iterations up to the next check (a multiple of check_every, or max_iter)
    const int n = std::min(prm.check_every - it % prm.check_every, prm.max_iter - it);
    const RhsSet set = active.set();
    rc = graphs ? graphs->run(eng, set, n) : eng.chunk(set, n);
    if (rc != WD_OK) break;
    it += n;
    for (int i = 0; i < active.n; ++i) iters[active.k[i]] = it;
    const bool at_max = it >= prm.max_iter;
    if ((rc = read()) != WD_OK) break;
    if (unread.n > 0) {
      IdxList going;
      for (int i = 0; i < active.n; ++i) {
        const int k = active.k[i];
        if (!unread.has(k)) {
          going.push(k);
          continue;
        }
        ++updates[k];
        switch (cg_after_refresh(sc(k), prm.tol, false)) {
          case kCgConverged: status[k] = WD_OK; iters[k] = refresh_it[k]; break;
          case kCgFailed: status[k] = WD_ERR_NUMERIC; iters[k] = refresh_it[k]; break;
          default: going.push(k); break;
        }
      }
      active = going;
      unread = IdxList{};
    }
    IdxList refresh, keep;
    for (int i = 0; i < active.n; ++i) {
      const int k = active.k[i];
      const CgAction a = cg_check(sc(k), prm.tol, mixed, prm.delta, at_max);
      if (a == kCgNumeric) { status[k] = WD_ERR_NUMERIC; continue; }
      if (a == kCgRefresh) refresh.push(k);
      keep.push(k);
    }
    active = keep;
    if (refresh.n == 0) continue;
    if ((rc = eng.refresh(refresh.set())) != WD_OK) break;
    // A recompute that follows a drop of the iterated residual by delta, with
    // no right-hand side claiming convergence and iterations left, almost
    // never ends a solve: the next chunk goes out at once and its read brings
    // the outcome (one wait for the device fewer per reliable update; a solve
    // that did converge there has run one chunk for nothing)
    bool wait = at_max;
    for (int i = 0; i < refresh.n; ++i) {
      const double* c = sc(refresh.k[i]);
      if (c[kRr] <= prm.tol * prm.tol * c[kB2]) wait = true;
    }
    if (!wait) {
      unread = refresh;
      for (int i = 0; i < refresh.n; ++i) refresh_it[refresh.k[i]] = it;
      continue;
    }
    if ((rc = read()) != WD_OK) break;
    IdxList still;
    for (int i = 0; i < active.n; ++i) {
      const int k = active.k[i];
      if (!refresh.has(k)) {
        still.push(k);
        continue;
      }
      ++updates[k];
      switch (cg_after_refresh(sc(k), prm.tol, at_max)) {
        case kCgConverged: status[k] = WD_OK; break;
        case kCgFailed: status[k] = WD_ERR_NUMERIC; break;
        case kCgNotConverged: status[k] = WD_ERR_NOT_CONVERGED; break;
        case kCgKeepGoing: still.push(k); break;
      }
    }
    active = still;
  }
  if (rc == WD_OK) {
    for (int i = 0; i < active.n; ++i) status[active.k[i]] = WD_ERR_NOT_CONVERGED;
    rc = read();
  }
  if (rc != WD_OK) {
    if (stats != nullptr)
      for (int k = 0; k < nrhs; ++k) stats[k].status = rc;
    return rc;
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  int worst = WD_OK;
  for (int k = 0; k < nrhs; ++k) {
    if (stats != nullptr) {
      stats[k].status = status[k];
      stats[k].iters = iters[k];
      stats[k].reliable_updates = updates[k];
      stats[k].reserved = 0;
      const double b2 = sc(k)[kB2];
      stats[k].true_rel_residual = b2 > 0.0 ? std::sqrt(sc(k)[kRrTrue] / b2) : 0.0;
      stats[k].seconds = secs;
    }
    if (status[k] != WD_OK && (worst == WD_OK || status[k] == WD_ERR_NUMERIC)) worst = status[k];
  }
  if (worst == WD_ERR_NOT_CONVERGED)
    set_error(worst, "cg_solve_normal: not converged to %g within %d iterations", prm.tol, prm.max_iter);
  else if (worst == WD_ERR_NUMERIC)
    set_error(worst, "cg_solve_normal: non-finite or non-positive value in the iteration");
  return worst;
}

namespace {

// Argument checks of the synchronous solver, shared by its two entry points;
// on success *vec is the bytes of b_dev and x_dev and *need the workspace's.
int check_solve_args(const wd_gauge* g_hi, const wd_gauge* g_lo, const double* masses, int32_t nrhs,
                     const void* b_dev, const void* x_dev, const wd_cg_params* params, size_t* vec,
                     size_t* need) {
  int rc = check_gauge(g_hi);
  if (rc != WD_OK) return rc;
  if ((rc = check_layout(g_hi, 0, "cg_solve_normal")) != WD_OK) return rc;
  if (g_hi->prec != WD_FP64) return set_error(WD_ERR_INVALID_ARG, "g_hi must be an FP64 gauge field");
  if (params == nullptr || masses == nullptr)
    return set_error(WD_ERR_INVALID_ARG, "params and masses_host must not be NULL");
  const wd_cg_params& p = *params;
  if (nrhs < 1 || nrhs > kMaxRhs) return set_error(WD_ERR_UNSUPPORTED, "nrhs %d outside 1..%d", nrhs, kMaxRhs);
  if (!(p.tol > 0.0) || p.max_iter < 1 || p.check_every < 1)
    return set_error(WD_ERR_INVALID_ARG, "need tol > 0, max_iter >= 1, check_every >= 1");
  if (p.inner != WD_FP64 && p.inner != WD_FP32 && p.inner != WD_FP16)
    return set_error(WD_ERR_INVALID_ARG, "unknown inner precision %d", p.inner);
  if (p.inner != WD_FP64) {
    if ((rc = check_gauge(g_lo)) != WD_OK) return rc;
    if ((rc = check_layout(g_lo, 0, "cg_solve_normal")) != WD_OK) return rc;
    if (g_lo->prec != p.inner)
      return set_error(WD_ERR_INVALID_ARG, "g_lo must be a gauge field of the inner precision %d", p.inner);
    for (int i = 0; i < 4; ++i)
      if (g_lo->dims[i] != g_hi->dims[i]) return set_error(WD_ERR_SHAPE, "g_lo and g_hi have different lattices");
    if (!(p.delta > 0.0 && p.delta < 1.0)) return set_error(WD_ERR_INVALID_ARG, "delta must lie in (0, 1)");
  }
  for (int k = 0; k < nrhs; ++k)
    if (!std::isfinite(masses[k])) return set_error(WD_ERR_INVALID_ARG, "mass %d is not finite", k);
  *vec = static_cast<size_t>(packed_sites(g_hi->V)) * nrhs * spinor_site_bytes(WD_FP64);
  if ((rc = check_device_range(b_dev, *vec, "b_dev")) != WD_OK) return rc;
  if ((rc = check_device_range(x_dev, *vec, "x_dev")) != WD_OK) return rc;
  if (overlaps(b_dev, *vec, x_dev, *vec)) return set_error(WD_ERR_INVALID_ARG, "b_dev and x_dev overlap");
  *need = cg_layout(g_hi->dims, nrhs, p.inner).bytes;
  return WD_OK;
}

// ---------------------------------------------------------------------------
// Workspace of the entry point that allocates nothing: a static device array,
// one copy per GPU (the loader places it with the code object on each device;
// it is held until the process ends). Host code never passes the array's name
// to a kernel or a copy: it is only a host-side stand-in for the symbol. The
// device address comes from hipGetSymbolAddress, looked up once per device
// with that device current, and only that address is used.
constexpr size_t kScratchBytes = WD_NOALLOC_SCRATCH_BYTES;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
// Scalars of a solve are copied to this pageable host buffer (one per device).
double g_noalloc_host[kMaxDevices][kMaxRhs * kScalars];

// The scratch array's device address on the current device (looked up on the
// first call there) and the device index.
int scratch_address(void** out, int* device) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(WD_ERR_DEVICE, "no current HIP device");
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(WD_ERR_UNSUPPORTED, "device %d beyond the %d the static workspace serves", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return set_error(WD_ERR_DEVICE, "looking up the static workspace on device %d: %s", dev,
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  *device = dev;
  return WD_OK;
}

}  // namespace
}  // namespace wd

using namespace wd;

extern "C" {

size_t cg_workspace_bytes(const int32_t dims[4], int32_t nrhs, int32_t inner) {
  long V = 0;
  if (check_dims(dims, &V) != WD_OK || nrhs < 1 || nrhs > kMaxRhs) return 0;
  if (inner != WD_FP64 && inner != WD_FP32 && inner != WD_FP16) return 0;
  return cg_layout(dims, nrhs, inner).bytes;
}

int cg_solve_normal(const wd_gauge* g_hi, const wd_gauge* g_lo, const double* masses_host,
                    int32_t nrhs, const void* b_dev, void* x_dev, const wd_cg_params* params,
                    wd_cg_stats* stats_host, void* ws_dev, size_t ws_bytes, hipStream_t stream) {
  try {
    clear_error();
    size_t vec = 0, need = 0;
    int rc = check_solve_args(g_hi, g_lo, masses_host, nrhs, b_dev, x_dev, params, &vec, &need);
    if (rc != WD_OK) return rc;
    if (ws_bytes < need) return set_error(WD_ERR_INVALID_ARG, "ws_bytes %zu < %zu needed", ws_bytes, need);
    if ((rc = check_device_range(ws_dev, need, "ws_dev")) != WD_OK) return rc;
    if (overlaps(b_dev, vec, ws_dev, need) || overlaps(x_dev, vec, ws_dev, need))
      return set_error(WD_ERR_INVALID_ARG, "b_dev, x_dev and ws_dev must not overlap");
    const wd_cg_params& p = *params;
    return solve_sync(g_hi, p.inner != WD_FP64 ? g_lo : g_hi, masses_host, nrhs, b_dev, x_dev, p,
                      stats_host, ws_dev, stream, nullptr);
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in cg_solve_normal");
  }
}

int cg_solve_normal_noalloc(const wd_gauge* g_hi, const wd_gauge* g_lo, const double* masses_host,
                            int32_t nrhs, const void* b_dev, void* x_dev, const wd_cg_params* params,
                            wd_cg_stats* stats_host, hipStream_t stream) {
  try {
    clear_error();
    size_t vec = 0, need = 0;
    int rc = check_solve_args(g_hi, g_lo, masses_host, nrhs, b_dev, x_dev, params, &vec, &need);
    if (rc != WD_OK) return rc;
    if (params->use_graph)
      return set_error(WD_ERR_UNSUPPORTED, "use_graph allocates (graph instantiation); not available here");
    if (need > kScratchBytes)
      return set_error(WD_ERR_NOMEM, "the solve needs %zu bytes of workspace; the static workspace holds %zu",
                       need, kScratchBytes);
    void* ws = nullptr;
    int dev = 0;
    if ((rc = scratch_address(&ws, &dev)) != WD_OK) return rc;
    const wd_cg_params& p = *params;
    return solve_sync(g_hi, p.inner != WD_FP64 ? g_lo : g_hi, masses_host, nrhs, b_dev, x_dev, p,
                      stats_host, ws, stream, g_noalloc_host[dev]);
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in cg_solve_normal_noalloc");
  }
}

}  // extern "C"
