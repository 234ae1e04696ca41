// Request server: continuous batching of CG solves on resident gauge fields.
//
// Clients register gauge fields (packed once into the server's arena and kept
// there) and submit solve requests of 1..16 right-hand sides with their own
// masses and tolerance. A scheduler thread keeps, per gauge field in use, a
// group of right-hand-side slots that iterate CG together (one fused
// multi-right-hand-side dslash per operator application). Requests join a
// group at chunk boundaries as slots and arena memory free up and leave it
// when their residual has converged; groups of different lattices run on
// different streams, so their work overlaps on the device.
//
// Chunks are check_every CG iterations long and slots join only at chunk
// boundaries, so every right-hand side sees the same sequence of operations
// and decisions whether it runs alone or in a mix: results are bit-identical.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "cg_engine.h"
#include "fields.h"
#include "server_policy.h"

namespace wd {
namespace {

using Clock = std::chrono::steady_clock;
constexpr int kStarveSkips = 64;  // scheduling rounds a request may be passed over

struct GaugeEntry {
  uint64_t id = 0;
  int32_t dims[4] = {0, 0, 0, 0};
  long V = 0;
  char* mem = nullptr;
  wd_gauge* hi = nullptr;
  wd_gauge* lo = nullptr;
  int groups = 0;    // groups currently built on it
  int requests = 0;  // queued or running requests on it
  bool removing = false;
  double last_used = 0;  // server time of its registration or latest request
};

struct Request {
  uint64_t ticket = 0;
  wd_request r{};
  GaugeEntry* gauge = nullptr;
  double t_submit = 0, t_start = -1, t_done = -1;
  int status = WD_PENDING;
  int remaining = 0;
  int skipped = 0;
  wd_cg_stats stats[kMaxRhs] = {};
  int nrhs() const { return r.nrhs; }
};

struct Slot {
  Request* req = nullptr;
  int rhs = 0;
  int iters = 0;
  int updates = 0;
};

struct Group {
  GaugeEntry* gauge = nullptr;
  int S = 0;
  char* mem = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  double* host_scal = nullptr;  // pinned
  std::unique_ptr<CgEngine> eng;
  std::vector<Slot> slots;
  enum Phase { kReady, kChunk, kRefresh, kCopy } phase = kReady;
  std::vector<int> refreshing;
  std::vector<std::pair<Request*, int>> completing;  // (request, status) per finished slot
  int active() const {
    int n = 0;
    for (const Slot& s : slots) n += s.req != nullptr;
    return n;
  }
  int free_slots() const { return S - active(); }
  bool ready() const { return phase == kReady; }
};

}  // namespace

}  // namespace wd

struct wd_server {
  wd_server_cfg cfg{};
  int device = 0;
  wd::Arena arena;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1, next_gauge = 1;
  int evictions = 0;
  std::map<uint64_t, std::unique_ptr<wd::GaugeEntry>> gauges;
  std::deque<wd::Request*> submitted;                       // not yet seen by the scheduler
  std::map<uint64_t, std::unique_ptr<wd::Request>> requests;  // every unpolled request
  // scheduler-thread state
  std::deque<wd::Request*> pending;
  std::vector<std::unique_ptr<wd::Group>> groups;
  std::vector<hipStream_t> streams;
  size_t next_stream = 0;
  wd::Clock::time_point t0;
  std::atomic<int> running{0};
  std::atomic<int> fatal{WD_OK};

  double now() const { return std::chrono::duration<double>(wd::Clock::now() - t0).count(); }
  void loop();
  bool admit();
  bool advance(wd::Group& g);
  void launch_chunk(wd::Group& g);
  void finish_slot(wd::Group& g, int k, int status);
  void destroy_group(size_t i);
  wd::Group* make_group(wd::GaugeEntry* ge, int need);
  void complete(wd::Request* rq);
};

namespace wd {
namespace {

size_t vec_bytes(long V, int n) {
  return align256(static_cast<size_t>(packed_sites(V)) * n * spinor_site_bytes(WD_FP64));
}

// Arena bytes of the inner-precision copy of a gauge field (none for FP64).
size_t inner_gauge_bytes(const int32_t dims[4], int inner) {
  return inner == WD_FP64 ? 0 : align256(wd_gauge_bytes(dims, inner, 0));
}

size_t group_bytes(const int32_t dims[4], long V, int S, int inner) {
  return 2 * vec_bytes(V, S) + cg_layout(dims, S, inner).bytes;
}

RhsSet set_of(const std::vector<int>& ks) {
  RhsSet s{};
  s.n = static_cast<int>(ks.size());
  for (size_t i = 0; i < ks.size(); ++i) s.idx[i] = ks[i];
  return s;
}

}  // namespace
}  // namespace wd

using namespace wd;

// Marks a request finished (lock held by the caller).
void wd_server::complete(Request* rq) {
  rq->t_done = now();
  int st = WD_OK;
  for (int k = 0; k < rq->r.nrhs; ++k) {
    const int s = rq->stats[k].status;
    if (s != WD_OK && (st == WD_OK || s == WD_ERR_NUMERIC || s == WD_ERR_CANCELLED)) st = s;
  }
  rq->status = st;
  --rq->gauge->requests;  // a removed gauge field is freed by the scheduler at 0
  running.fetch_sub(1);
}

// A group of the configured number of slots if the arena has room for one,
// else one of just `need` slots (the request that asks for it), so that a
// request does not wait for memory a smaller group would not need.
Group* wd_server::make_group(GaugeEntry* ge, int need) {
  int S = cfg.max_rhs_per_group;
  char* mem;
  {
    std::lock_guard<std::mutex> lk(mu);
    mem = arena.alloc(group_bytes(ge->dims, ge->V, S, cfg.inner));
    if (mem == nullptr && need < S) {
      S = need;
      mem = arena.alloc(group_bytes(ge->dims, ge->V, S, cfg.inner));
    }
  }
  if (mem == nullptr) return nullptr;
  auto g = std::make_unique<Group>();
  g->gauge = ge;
  g->S = S;
  g->mem = mem;
  g->stream = streams[next_stream++ % streams.size()];
  if (hipEventCreateWithFlags(&g->ev, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&g->host_scal), S * kScalars * sizeof(double),
                    hipHostMallocDefault) != hipSuccess) {
    if (g->ev) (void)hipEventDestroy(g->ev);
    std::lock_guard<std::mutex> lk(mu);
    arena.release(mem);
    fatal = WD_ERR_DEVICE;
    return nullptr;
  }
  void* b = mem;
  void* x = mem + vec_bytes(ge->V, S);
  void* ws = mem + 2 * vec_bytes(ge->V, S);
  g->eng = std::make_unique<CgEngine>(ge->hi, cfg.inner != WD_FP64 ? ge->lo : ge->hi, cfg.inner, S, b,
                                      x, ws, g->stream);
  g->slots.assign(S, Slot{});
  {
    std::lock_guard<std::mutex> lk(mu);  // eviction reads the count under the lock
    ge->groups++;
  }
  groups.push_back(std::move(g));
  return groups.back().get();
}

void wd_server::destroy_group(size_t i) {
  Group& g = *groups[i];
  (void)hipStreamSynchronize(g.stream);
  (void)hipEventDestroy(g.ev);
  (void)hipHostFree(g.host_scal);
  {
    std::lock_guard<std::mutex> lk(mu);
    g.gauge->groups--;
    arena.release(g.mem);
  }
  groups.erase(groups.begin() + static_cast<long>(i));
}

// Admits waiting requests into groups (policy in server_policy.h): the right-hand
// sides of an admitted request are copied into free slots and started.
bool wd_server::admit() {
  struct Ops {
    wd_server* s;
    Group* make_group(GaugeEntry* ge, int need) { return s->make_group(ge, need); }
    void place(Group* target, Request* rq) {
      std::vector<int> ks;
      const size_t field = static_cast<size_t>(packed_sites(rq->gauge->V)) * spinor_site_bytes(WD_FP64);
      for (int k = 0; k < target->S && static_cast<int>(ks.size()) < rq->r.nrhs; ++k) {
        if (target->slots[k].req != nullptr) continue;
        const int j = static_cast<int>(ks.size());
        target->slots[k] = Slot{rq, j, 0, 0};
        target->eng->set_mass(k, rq->r.masses[j]);
        if (hipMemcpyAsync(target->mem + k * field, static_cast<const char*>(rq->r.b_dev) + j * field,
                           field, hipMemcpyDeviceToDevice, target->stream) != hipSuccess)
          s->fatal = WD_ERR_DEVICE;
        ks.push_back(k);
      }
      if (target->eng->start(set_of(ks), false) != WD_OK) s->fatal = WD_ERR_DEVICE;
      std::lock_guard<std::mutex> lk(s->mu);
      rq->t_start = s->now();
    }
  } ops{this};
  std::vector<Group*> current;
  for (auto& g : groups) current.push_back(g.get());
  return admit_requests(pending, current, ops, kStarveSkips);
}

void wd_server::launch_chunk(Group& g) {
  std::vector<int> ks;
  for (int k = 0; k < g.S; ++k)
    if (g.slots[k].req != nullptr) ks.push_back(k);
  const RhsSet set = set_of(ks);
  if (g.eng->chunk(set, cfg.check_every) != WD_OK) fatal = WD_ERR_DEVICE;
  for (int k : ks) g.slots[k].iters += cfg.check_every;
  if (g.eng->fetch_scalars(g.host_scal) != WD_OK || hipEventRecord(g.ev, g.stream) != hipSuccess)
    fatal = WD_ERR_DEVICE;
  g.phase = Group::kChunk;
}

// A slot is done: copy its solution out (stream ordered) and free it.
void wd_server::finish_slot(Group& g, int k, int status) {
  Slot& s = g.slots[k];
  Request* rq = s.req;
  const size_t field = static_cast<size_t>(packed_sites(g.gauge->V)) * spinor_site_bytes(WD_FP64);
  const double* sc = g.host_scal + k * kScalars;
  {
    std::lock_guard<std::mutex> lk(mu);
    wd_cg_stats& st = rq->stats[s.rhs];
    st.status = status;
    st.iters = s.iters;
    st.reliable_updates = s.updates;
    st.reserved = 0;
    st.true_rel_residual = sc[kB2] > 0.0 ? std::sqrt(sc[kRrTrue] / sc[kB2]) : 0.0;
    st.seconds = now() - rq->t_start;
  }
  if (status != WD_ERR_CANCELLED)
    (void)hipMemcpyAsync(static_cast<char*>(rq->r.x_dev) + s.rhs * field,
                         g.mem + vec_bytes(g.gauge->V, g.S) + k * field, field,
                         hipMemcpyDeviceToDevice, g.stream);
  g.completing.emplace_back(rq, s.rhs);
  s = Slot{};
}

// The group's event has completed: act on the scalars it brought back.
bool wd_server::advance(Group& g) {
  const bool mixed = cfg.inner != WD_FP64;
  if (g.phase == Group::kChunk) {
    g.refreshing.clear();
    for (int k = 0; k < g.S; ++k) {
      Slot& s = g.slots[k];
      if (s.req == nullptr) continue;
      const bool at_max = s.iters >= s.req->r.max_iter;
      const CgAction a = cg_check(g.host_scal + k * kScalars, s.req->r.tol, mixed, cfg.delta, at_max);
      if (a == kCgNumeric) finish_slot(g, k, WD_ERR_NUMERIC);
      else if (a == kCgRefresh) g.refreshing.push_back(k);
    }
    if (!g.refreshing.empty()) {
      if (g.eng->refresh(set_of(g.refreshing)) != WD_OK || g.eng->fetch_scalars(g.host_scal) != WD_OK ||
          hipEventRecord(g.ev, g.stream) != hipSuccess)
        fatal = WD_ERR_DEVICE;
      g.phase = Group::kRefresh;
      return true;
    }
  } else if (g.phase == Group::kRefresh) {
    for (int k : g.refreshing) {
      Slot& s = g.slots[k];
      s.updates++;
      const bool at_max = s.iters >= s.req->r.max_iter;
      switch (cg_after_refresh(g.host_scal + k * kScalars, s.req->r.tol, at_max)) {
        case kCgConverged: finish_slot(g, k, WD_OK); break;
        case kCgFailed: finish_slot(g, k, WD_ERR_NUMERIC); break;
        case kCgNotConverged: finish_slot(g, k, WD_ERR_NOT_CONVERGED); break;
        case kCgKeepGoing: break;
      }
    }
    g.refreshing.clear();
  } else if (g.phase == Group::kCopy) {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& [rq, rhs] : g.completing) {
      (void)rhs;
      if (--rq->remaining == 0) complete(rq);
    }
    g.completing.clear();
    g.phase = Group::kReady;
    cv.notify_all();
    return true;
  }
  if (!g.completing.empty()) {
    if (hipEventRecord(g.ev, g.stream) != hipSuccess) fatal = WD_ERR_DEVICE;
    g.phase = Group::kCopy;
  } else {
    g.phase = Group::kReady;
  }
  return true;
}

void wd_server::loop() {
  (void)hipSetDevice(device);
  for (;;) {
    bool did = false;
    bool stopping;
    {
      std::unique_lock<std::mutex> lk(mu);
      while (!submitted.empty()) {
        pending.push_back(submitted.front());
        submitted.pop_front();
      }
      stopping = stop;
      if (stopping) {
        // queued requests are cancelled; running slots are cancelled below
        for (Request* rq : pending) {
          for (int k = 0; k < rq->r.nrhs; ++k) rq->stats[k].status = WD_ERR_CANCELLED;
          rq->remaining = 0;
          complete(rq);
        }
        pending.clear();
      }
    }
    for (auto& g : groups) {
      if (g->phase == Group::kReady) continue;
      const hipError_t q = hipEventQuery(g->ev);
      if (q == hipSuccess) {
        did |= advance(*g);
      } else if (q != hipErrorNotReady) {
        fatal = WD_ERR_DEVICE;
      }
    }
    if (stopping) {
      bool busy = false;
      for (auto& g : groups) {
        if (g->phase != Group::kReady) {
          busy = true;
          continue;
        }
        for (int k = 0; k < g->S; ++k)
          if (g->slots[k].req != nullptr) finish_slot(*g, k, WD_ERR_CANCELLED);
        if (!g->completing.empty()) {
          (void)hipEventRecord(g->ev, g->stream);
          g->phase = Group::kCopy;
          busy = true;
        }
      }
      if (!busy) break;
    } else {
      did |= admit();
      for (auto& g : groups)
        if (g->phase == Group::kReady && g->active() > 0) {
          launch_chunk(*g);
          did = true;
        }
      // free idle groups that no admissible queued request wants, so their
      // arena memory can go to other lattices
      for (size_t i = groups.size(); i-- > 0;) {
        Group& g = *groups[i];
        if (g.phase != Group::kReady || g.active() > 0) continue;
        if (!group_wanted(pending, g.gauge, g.S, kStarveSkips)) destroy_group(i);
      }
      // gauge fields removed by the client go once nothing uses them
      std::lock_guard<std::mutex> lk(mu);
      for (auto it = gauges.begin(); it != gauges.end();) {
        GaugeEntry& ge = *it->second;
        if (ge.removing && ge.requests == 0 && ge.groups == 0) {
          wd_gauge_release(ge.hi);
          wd_gauge_release(ge.lo);
          arena.release(ge.mem);
          it = gauges.erase(it);
        } else {
          ++it;
        }
      }
    }
    if (!did) {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait_for(lk, std::chrono::microseconds(50), [&] { return stop || !submitted.empty(); });
    }
  }
  for (size_t i = groups.size(); i-- > 0;) destroy_group(i);
}

extern "C" {

int wd_server_create(const wd_server_cfg* cfg, wd_server** out) {
  try {
    clear_error();
    if (cfg == nullptr || out == nullptr) return set_error(WD_ERR_INVALID_ARG, "cfg and out must not be NULL");
    *out = nullptr;
    if (cfg->inner != WD_FP64 && cfg->inner != WD_FP32 && cfg->inner != WD_FP16)
      return set_error(WD_ERR_INVALID_ARG, "unknown inner precision %d", cfg->inner);
    if (cfg->check_every < 1 || cfg->max_rhs_per_group < 1 || cfg->max_rhs_per_group > kMaxRhs ||
        cfg->n_streams < 1 || cfg->n_streams > 16)
      return set_error(WD_ERR_INVALID_ARG,
                       "need check_every >= 1, max_rhs_per_group in 1..16, n_streams in 1..16");
    if (cfg->inner != WD_FP64 && !(cfg->delta > 0.0 && cfg->delta < 1.0))
      return set_error(WD_ERR_INVALID_ARG, "delta must lie in (0, 1)");
    int rc = check_device_range(cfg->arena_dev, cfg->arena_bytes, "arena_dev");
    if (rc != WD_OK) return rc;
    auto s = std::make_unique<wd_server>();
    s->cfg = *cfg;
    (void)hipGetDevice(&s->device);
    s->arena.init(static_cast<char*>(cfg->arena_dev), cfg->arena_bytes);
    for (int i = 0; i < cfg->n_streams; ++i) {
      hipStream_t st = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
        return set_error(WD_ERR_DEVICE, "stream creation failed");
      }
      s->streams.push_back(st);
    }
    s->t0 = Clock::now();
    wd_server* raw = s.get();
    s->worker = std::thread([raw] { raw->loop(); });
    *out = s.release();
    return WD_OK;
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in wd_server_create");
  }
}

int wd_server_add_gauge(wd_server* s, const int32_t dims[4], const void* U_canon_dev,
                        uint64_t* gauge_id) {
  try {
    clear_error();
    if (s == nullptr || gauge_id == nullptr) return set_error(WD_ERR_INVALID_ARG, "NULL argument");
    long V = 0;
    int rc = check_dims(dims, &V);
    if (rc != WD_OK) return rc;
    if ((rc = check_device_range(U_canon_dev, static_cast<size_t>(V) * 36 * 16, "U_canon_dev")) != WD_OK)
      return rc;
    const size_t bhi = align256(wd_gauge_bytes(dims, WD_FP64, 0));
    const size_t blo = inner_gauge_bytes(dims, s->cfg.inner);
    auto ge = std::make_unique<GaugeEntry>();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      ge->mem = s->arena.alloc(bhi + blo);
      // with eviction on, idle gauge fields (no request queued or running, no
      // group built on them, so no device work uses them) make room, least
      // recently used first
      while (ge->mem == nullptr && s->cfg.evict_idle_gauges) {
        GaugeEntry* lru = nullptr;
        for (auto& kv : s->gauges) {
          GaugeEntry* g = kv.second.get();
          if (!g->removing && g->requests == 0 && g->groups == 0 &&
              (lru == nullptr || g->last_used < lru->last_used))
            lru = g;
        }
        if (lru == nullptr) break;
        wd_gauge_release(lru->hi);
        wd_gauge_release(lru->lo);
        s->arena.release(lru->mem);
        s->gauges.erase(lru->id);
        s->evictions++;
        ge->mem = s->arena.alloc(bhi + blo);
      }
    }
    if (ge->mem == nullptr) return set_error(WD_ERR_NOMEM, "arena has no room for the gauge field");
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->arena.release(ge->mem);
      return set_error(WD_ERR_DEVICE, "stream creation failed");
    }
    rc = wd_gauge_import(dims, U_canon_dev, WD_FP64, 0, ge->mem, bhi, st, &ge->hi);
    if (rc == WD_OK && blo)
      rc = wd_gauge_import(dims, U_canon_dev, s->cfg.inner, 0, ge->mem + bhi, blo, st, &ge->lo);
    if (rc == WD_OK && hipStreamSynchronize(st) != hipSuccess)
      rc = set_error(WD_ERR_DEVICE, "packing the gauge field failed");
    (void)hipStreamDestroy(st);
    if (rc != WD_OK) {
      wd_gauge_release(ge->hi);
      wd_gauge_release(ge->lo);
      std::lock_guard<std::mutex> lk(s->mu);
      s->arena.release(ge->mem);
      return rc;
    }
    for (int i = 0; i < 4; ++i) ge->dims[i] = dims[i];
    ge->V = V;
    std::lock_guard<std::mutex> lk(s->mu);
    ge->id = s->next_gauge++;
    ge->last_used = s->now();
    *gauge_id = ge->id;
    s->gauges[ge->id] = std::move(ge);
    return WD_OK;
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in wd_server_add_gauge");
  }
}

int wd_server_remove_gauge(wd_server* s, uint64_t gauge_id) {
  clear_error();
  if (s == nullptr) return set_error(WD_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->gauges.find(gauge_id);
  if (it == s->gauges.end() || it->second->removing)
    return set_error(WD_ERR_INVALID_ARG, "unknown gauge id %llu", static_cast<unsigned long long>(gauge_id));
  it->second->removing = true;  // freed by the scheduler once no request or group uses it
  s->cv.notify_all();
  return WD_OK;
}

int cg_submit(wd_server* s, const wd_request* req, uint64_t* ticket) {
  try {
    clear_error();
    if (s == nullptr || req == nullptr || ticket == nullptr)
      return set_error(WD_ERR_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop) return set_error(WD_ERR_CANCELLED, "server is shutting down");
    auto git = s->gauges.find(req->gauge_id);
    if (git == s->gauges.end() || git->second->removing)
      return set_error(WD_ERR_INVALID_ARG, "unknown gauge id %llu",
                       static_cast<unsigned long long>(req->gauge_id));
    GaugeEntry* ge = git->second.get();
    if (req->nrhs < 1 || req->nrhs > s->cfg.max_rhs_per_group)
      return set_error(WD_ERR_UNSUPPORTED, "nrhs %d outside 1..%d", req->nrhs, s->cfg.max_rhs_per_group);
    if (!(req->tol > 0.0) || req->max_iter < 1)
      return set_error(WD_ERR_INVALID_ARG, "need tol > 0 and max_iter >= 1");
    for (int k = 0; k < req->nrhs; ++k)
      if (!std::isfinite(req->masses[k])) return set_error(WD_ERR_INVALID_ARG, "mass %d is not finite", k);
    // Reserve the gauge field before the lock is dropped: with requests > 0 no
    // eviction and no removal frees it. Every error return below gives the
    // reservation back under the lock (a removed field is then freed by the
    // scheduler as usual).
    ge->requests++;
    int32_t gdims[4];
    for (int i = 0; i < 4; ++i) gdims[i] = ge->dims[i];
    const long gV = ge->V;
    lk.unlock();
    auto unreserve = [&](int code) {
      lk.lock();
      ge->requests--;
      s->cv.notify_all();
      return code;
    };
    const size_t vec = static_cast<size_t>(packed_sites(gV)) * req->nrhs * spinor_site_bytes(WD_FP64);
    int rc = check_device_range(req->b_dev, vec, "b_dev");
    if (rc == WD_OK) rc = check_device_range(req->x_dev, vec, "x_dev");
    if (rc != WD_OK) return unreserve(rc);
    if (overlaps(req->b_dev, vec, req->x_dev, vec))
      return unreserve(set_error(WD_ERR_INVALID_ARG, "b_dev and x_dev overlap"));
    {
      // the arena minus the registered gauge fields must hold a group of the
      // request's right-hand sides
      size_t gauges = 0;
      lk.lock();
      for (auto& [id, g] : s->gauges)
        if (!g->removing)
          gauges += align256(wd_gauge_bytes(g->dims, WD_FP64, 0)) + inner_gauge_bytes(g->dims, s->cfg.inner);
      lk.unlock();
      if (group_bytes(gdims, gV, req->nrhs, s->cfg.inner) + gauges > s->cfg.arena_bytes)
        return unreserve(
            set_error(WD_ERR_NOMEM, "a solve group of this lattice cannot fit beside the gauge fields"));
    }
    auto rq = std::make_unique<Request>();
    rq->r = *req;
    rq->gauge = ge;
    rq->remaining = req->nrhs;
    for (int k = 0; k < req->nrhs; ++k) rq->stats[k].status = WD_PENDING;
    lk.lock();
    if (s->stop) {
      ge->requests--;
      return set_error(WD_ERR_CANCELLED, "server is shutting down");
    }
    rq->t_submit = s->now();
    rq->ticket = s->next_ticket++;
    *ticket = rq->ticket;
    ge->last_used = s->now();
    s->running.fetch_add(1);
    s->submitted.push_back(rq.get());
    s->requests[rq->ticket] = std::move(rq);
    s->cv.notify_all();
    return WD_OK;
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in cg_submit");
  }
}

int cg_poll(wd_server* s, uint64_t ticket, wd_result* out) {
  try {
    clear_error();
    if (s == nullptr) return set_error(WD_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != WD_OK) return set_error(s->fatal, "the server hit a device error");
    auto it = s->requests.find(ticket);
    if (it == s->requests.end())
      return set_error(WD_ERR_UNKNOWN_TICKET, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
    Request& rq = *it->second;
    if (out != nullptr) {
      out->status = rq.status;
      out->nrhs = rq.r.nrhs;
      out->t_submit = rq.t_submit;
      out->t_start = rq.t_start;
      out->t_done = rq.t_done;
      for (int k = 0; k < rq.r.nrhs; ++k) out->stats[k] = rq.stats[k];
    }
    if (rq.status == WD_PENDING) return WD_PENDING;
    const int st = rq.status;
    s->requests.erase(it);  // a final status is reported once
    return st;
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in cg_poll");
  }
}

int wd_server_info(wd_server* s, wd_server_state* out) {
  clear_error();
  if (s == nullptr || out == nullptr) return set_error(WD_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out->arena_in_use = s->arena.in_use();
  out->arena_peak = s->arena.peak();
  out->unfinished = s->running.load();
  out->gauges = static_cast<int32_t>(s->gauges.size());
  out->evictions = s->evictions;
  out->reserved = 0;
  return WD_OK;
}

int wd_server_destroy(wd_server* s) {
  try {
    clear_error();
    if (s == nullptr) return WD_OK;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& [id, ge] : s->gauges) {
      wd_gauge_release(ge->hi);
      wd_gauge_release(ge->lo);
    }
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return WD_OK;
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in wd_server_destroy");
  }
}

}  // extern "C"
