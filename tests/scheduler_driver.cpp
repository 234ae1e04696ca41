// Host-only checks of the request server's scheduling policy
// (paper_1901_07294_amd/csrc/server_policy.h) with a fake executor: groups are
// plain structs whose "chunks" finish in one simulated round, and group memory
// comes from the real arena allocator over a fake region. Prints one line per
// scenario and exits nonzero if any fails.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <memory>
#include <string>
#include <vector>

#include "server_policy.h"

namespace {

int failures = 0;

void check(bool ok, const std::string& name, const std::string& what) {
  if (!ok) {
    ++failures;
    std::printf("FAIL %s: %s\n", name.c_str(), what.c_str());
  }
}

// Prints PASS for a scenario that added no failure since `before`.
void report(const std::string& name, int before) {
  if (failures == before) std::printf("PASS %s\n", name.c_str());
}

struct FakeReq {
  int id = 0;
  int gauge = 0;
  int n = 1;          // right-hand sides
  int chunks = 1;     // chunks until it converges
  int skipped = 0;
  int admitted_round = -1;
  int done_round = -1;
  int nrhs() const { return n; }
};

struct FakeGroup {
  int gauge = 0;
  int S = 4;
  char* mem = nullptr;
  bool running = false;  // a chunk is in flight
  std::vector<FakeReq*> slots;  // one entry per occupied slot
  int free_slots() const { return S - static_cast<int>(slots.size()); }
  bool ready() const { return !running; }
};

// The executor: opens groups in an arena (group_bytes per slot) of S slots,
// or of just the slots a request needs when S slots do not fit (as the
// server does), and records placements.
struct FakeOps {
  wd::Arena* arena;
  size_t group_bytes;  // of a group of S slots
  int S;
  int round = 0;
  std::vector<std::unique_ptr<FakeGroup>>* groups;
  FakeGroup* make_group(int gauge, int need) {
    int slots = S;
    char* m = arena->alloc(group_bytes);
    if (m == nullptr && need < S) {
      slots = need;
      m = arena->alloc(group_bytes / S * need);
    }
    if (m == nullptr) return nullptr;
    groups->push_back(std::make_unique<FakeGroup>());
    FakeGroup* g = groups->back().get();
    g->gauge = gauge;
    g->S = slots;
    g->mem = m;
    return g;
  }
  void place(FakeGroup* g, FakeReq* r) {
    for (int k = 0; k < r->n; ++k) g->slots.push_back(r);
    r->admitted_round = round;
  }
};

std::vector<FakeGroup*> view(std::vector<std::unique_ptr<FakeGroup>>& gs) {
  std::vector<FakeGroup*> v;
  for (auto& g : gs) v.push_back(g.get());
  return v;
}

void arena_scenarios() {
  const std::string name = "arena";
  const int before = failures;
  static char region[1 << 20];
  wd::Arena a;
  a.init(region, sizeof(region));
  char* p1 = a.alloc(1000);       // rounds to 1024
  char* p2 = a.alloc(256);
  char* p3 = a.alloc(300000);
  check(p1 == region && p2 == region + 1024 && p3 == region + 1280, name, "first fit, 256-B aligned");
  check(a.in_use() == 1024 + 256 + 300032, name, "in_use counts aligned sizes");
  a.release(p2);
  char* p4 = a.alloc(200);
  check(p4 == p2, name, "a freed hole is reused first");
  a.release(p1);
  a.release(p4);
  check(a.free_blocks() == 2, name, "neighbouring holes coalesce");
  a.release(p3);
  check(a.free_blocks() == 1 && a.in_use() == 0, name, "everything coalesces back");
  check(a.peak() == 1024 + 256 + 300032, name, "peak");
  check(a.alloc(sizeof(region) + 1) == nullptr, name, "oversize fails");
  a.release(nullptr);
  a.release(region + 12345);  // not an allocation: ignored
  check(a.in_use() == 0, name, "foreign pointers are ignored");
  report(name, before);
}

void fifo_and_join() {
  const std::string name = "fifo_join";
  const int before = failures;
  static char region[1 << 16];
  wd::Arena a;
  a.init(region, sizeof(region));
  std::vector<std::unique_ptr<FakeGroup>> groups;
  FakeOps ops{&a, 4096, 4, 0, &groups};
  FakeReq r[4];
  r[0] = {0, 7, 2};
  r[1] = {1, 7, 2};
  r[2] = {2, 8, 3};
  r[3] = {3, 7, 1};  // group of gauge 7 is full after r0, r1: a second group opens
  std::deque<FakeReq*> pending = {&r[0], &r[1], &r[2], &r[3]};
  const bool did = wd::admit_requests(pending, view(groups), ops, 64);
  check(did && pending.empty(), name, "all admitted");
  check(groups.size() == 3, name, "groups: 7 (full), 8, 7 again");
  check(groups[0]->gauge == 7 && groups[0]->slots.size() == 4, name, "r0 and r1 share a group");
  check(groups[1]->gauge == 8 && groups[2]->gauge == 7, name, "arrival order of new groups");
  report(name, before);
}

void busy_group_waits() {
  const std::string name = "busy_group";
  const int before = failures;
  static char region[1 << 16];
  wd::Arena a;
  a.init(region, sizeof(region));
  std::vector<std::unique_ptr<FakeGroup>> groups;
  FakeOps ops{&a, 4096, 4, 0, &groups};
  FakeReq r0{0, 7, 1};
  std::deque<FakeReq*> pending = {&r0};
  wd::admit_requests(pending, view(groups), ops, 64);
  groups[0]->running = true;  // a chunk in flight: it takes newcomers at the boundary
  FakeReq r1{1, 7, 2};
  pending = {&r1};
  const bool did = wd::admit_requests(pending, view(groups), ops, 64);
  check(!did && pending.size() == 1 && groups.size() == 1, name,
        "a request waits for a running group with room instead of opening another");
  groups[0]->running = false;
  check(wd::admit_requests(pending, view(groups), ops, 64) && groups[0]->slots.size() == 3, name,
        "it joins at the boundary");
  report(name, before);
}

void arena_limits_and_starvation() {
  const std::string name = "starvation";
  const int before = failures;
  // room for exactly two groups
  static char region[2 * 4096];
  wd::Arena a;
  a.init(region, sizeof(region));
  std::vector<std::unique_ptr<FakeGroup>> groups;
  FakeOps ops{&a, 4096, 2, 0, &groups};
  FakeReq fill[2] = {{0, 1, 2}, {1, 2, 2}};   // gauges 1 and 2 fill both groups
  std::deque<FakeReq*> pending = {&fill[0], &fill[1]};
  wd::admit_requests(pending, view(groups), ops, 3);
  FakeReq big{2, 3, 1};                        // gauge 3 needs a third group: no room
  pending = {&big};
  std::vector<std::unique_ptr<FakeReq>> smalls;
  int admitted_behind = 0;
  for (int round = 0; round < 10; ++round) {
    // gauge-1 group frees its slots every round; a new gauge-1 request arrives
    groups[0]->slots.clear();
    smalls.push_back(std::make_unique<FakeReq>(FakeReq{100 + round, 1, 2}));
    pending.push_back(smalls.back().get());
    const size_t before = pending.size();
    wd::admit_requests(pending, view(groups), ops, 3);
    admitted_behind += static_cast<int>(before - pending.size());
  }
  check(big.skipped == 4, name, "passed over until the limit, then no more");
  check(admitted_behind == 4, name, "only starve_skips + 1 requests overtake a starving one");
  check(pending.front() == &big, name, "the starving request stays first");
  // room appears: the starving request goes first
  a.release(groups[1]->mem);
  groups.erase(groups.begin() + 1);
  wd::admit_requests(pending, view(groups), ops, 3);
  check(big.admitted_round >= 0, name, "admitted once its group fits");
  report(name, before);
}

// Memory for less than a second full group: a request gets a group of just
// its own right-hand sides instead of waiting.
void small_groups() {
  const std::string name = "small_groups";
  const int before = failures;
  static char region[4096 + 2048];  // one group of 4 slots (1024 B each) + 2 slots
  wd::Arena a;
  a.init(region, sizeof(region));
  std::vector<std::unique_ptr<FakeGroup>> groups;
  FakeOps ops{&a, 4096, 4, 0, &groups};
  FakeReq r[4];
  r[0] = {0, 1, 4};
  r[1] = {1, 2, 1};  // no room for 4 slots: a group of 1
  r[2] = {2, 2, 2};  // r1's group is full and 1 slot of memory is left: waits
  r[3] = {3, 2, 1};  // fits in that last slot
  std::deque<FakeReq*> pending = {&r[0], &r[1], &r[2], &r[3]};
  wd::admit_requests(pending, view(groups), ops, 64);
  check(groups.size() == 3 && groups[0]->S == 4 && groups[1]->S == 1 && groups[2]->S == 1, name,
        "one full group, then groups of the requests' own size");
  check(pending.size() == 1 && pending.front() == &r[2] && r[2].skipped == 1, name,
        "the request that does not fit waits and is passed over once");
  check(a.in_use() == sizeof(region), name, "the arena is used up exactly");
  a.release(groups[1]->mem);  // r1 done: its slot frees 1 KiB, still not 2
  groups.erase(groups.begin() + 1);
  check(!wd::admit_requests(pending, view(groups), ops, 64), name, "2 slots do not fit in 1");
  a.release(groups[1]->mem);  // r3 done: 2 KiB free
  groups.erase(groups.begin() + 1);
  check(wd::admit_requests(pending, view(groups), ops, 64) && groups.back()->S == 2, name,
        "then a group of 2");
  report(name, before);
}

// Idle groups too small for the queued requests of their gauge must not be
// kept for them: here two such groups hold the whole arena.
void small_idle_groups_released() {
  const std::string name = "small_idle_groups";
  const int before = failures;
  static char region[2 * 1024];  // room for two 1-slot groups (or one of 2 slots)
  wd::Arena a;
  a.init(region, sizeof(region));
  std::vector<std::unique_ptr<FakeGroup>> groups;
  FakeOps ops{&a, 4096, 4, 0, &groups};
  FakeReq r[4];
  r[0] = {0, 1, 1};
  r[1] = {1, 2, 1};
  std::deque<FakeReq*> pending = {&r[0], &r[1]};
  wd::admit_requests(pending, view(groups), ops, 64);
  check(groups.size() == 2 && groups[0]->S == 1 && groups[1]->S == 1, name, "two 1-slot groups");
  for (auto& g : groups) g->slots.clear();  // both requests finished: the groups are idle
  r[2] = {2, 1, 2};  // 2 right-hand sides on each gauge: neither idle group can take them
  r[3] = {3, 2, 2};
  pending = {&r[2], &r[3]};
  int rounds = 0;
  for (; rounds < 10 && !pending.empty(); ++rounds) {
    wd::admit_requests(pending, view(groups), ops, 64);
    for (size_t i = groups.size(); i-- > 0;) {
      if (groups[i]->slots.empty() &&
          !wd::group_wanted(pending, groups[i]->gauge, groups[i]->S, 64)) {
        a.release(groups[i]->mem);
        groups.erase(groups.begin() + static_cast<long>(i));
      }
    }
    for (auto& g : groups) g->slots.clear();  // admitted requests finish within the round
  }
  check(pending.empty(), name, "the queued requests are admitted once the small groups go");
  report(name, before);
}

// Rounds of admit / run one chunk per group / retire: every request finishes,
// memory never exceeds the arena, idle groups return their memory.
void simulated_serving() {
  const std::string name = "serving";
  const int before = failures;
  static char region[3 * 8192];
  wd::Arena a;
  a.init(region, sizeof(region));
  std::vector<std::unique_ptr<FakeGroup>> groups;
  FakeOps ops{&a, 8192, 4, 0, &groups};
  std::vector<FakeReq> reqs(60);
  unsigned seed = 12345;
  auto rnd = [&](int m) { seed = seed * 1103515245u + 12345u; return static_cast<int>((seed >> 8) % m); };
  for (int i = 0; i < 60; ++i) reqs[i] = {i, rnd(5), 1 + rnd(4), 1 + rnd(6)};
  std::deque<FakeReq*> pending;
  int next = 0, done = 0;
  for (int round = 0; round < 2000 && done < 60; ++round) {
    ops.round = round;
    for (int k = 0; k < 2 && next < 60; ++k) pending.push_back(&reqs[next++]);
    wd::admit_requests(pending, view(groups), ops, 16);
    check(a.in_use() <= sizeof(region), name, "arena never exceeded");
    for (auto& g : groups) {  // one chunk: every request in the group advances
      std::vector<FakeReq*> keep;
      FakeReq* last = nullptr;
      for (FakeReq* r : g->slots) {
        if (r != last && --r->chunks == 0) r->done_round = round, ++done;
        last = r;
        if (r->chunks > 0) keep.push_back(r);
      }
      g->slots = keep;
    }
    for (size_t i = groups.size(); i-- > 0;) {  // idle groups no admissible request wants go
      if (groups[i]->slots.empty() && !wd::group_wanted(pending, groups[i]->gauge, groups[i]->S, 16)) {
        a.release(groups[i]->mem);
        groups.erase(groups.begin() + static_cast<long>(i));
      }
    }
  }
  check(done == 60, name, "every request finished");
  for (auto& r : reqs) check(r.done_round >= r.admitted_round && r.admitted_round >= 0, name, "order");
  check(a.peak() <= sizeof(region) && groups.empty() && a.in_use() == 0, name, "memory returned");
  report(name, before);
}

// The serving mix: 8 gauge fields in 4 lattice sizes (group memory per slot
// 1, 4, 16 and 32 units), requests of 1..12 right-hand sides arriving in
// bursts, an arena that holds about two full groups of the largest size.
// Every request must finish, and the arena is never exceeded.
struct SizedOps {
  wd::Arena* arena;
  int S;
  int round = 0;
  std::vector<std::unique_ptr<FakeGroup>>* groups;
  static size_t unit(int gauge) { return size_t{256} << (gauge / 2 == 0 ? 0 : gauge / 2 == 1 ? 2 : gauge / 2 == 2 ? 4 : 5); }
  FakeGroup* make_group(int gauge, int need) {
    int slots = S;
    char* m = arena->alloc(unit(gauge) * S);
    if (m == nullptr && need < S) {
      slots = need;
      m = arena->alloc(unit(gauge) * need);
    }
    if (m == nullptr) return nullptr;
    groups->push_back(std::make_unique<FakeGroup>());
    FakeGroup* g = groups->back().get();
    g->gauge = gauge;
    g->S = slots;
    g->mem = m;
    return g;
  }
  void place(FakeGroup* g, FakeReq* r) {
    for (int k = 0; k < r->n; ++k) g->slots.push_back(r);
    r->admitted_round = round;
  }
};

void serving_mix(unsigned seed) {
  const std::string name = "serving_mix_" + std::to_string(seed);
  const int before = failures;
  const int S = 12, nreq = 400;
  static char region[2 * 12 * (256 << 5) + 12 * 256];
  wd::Arena a;
  a.init(region, sizeof(region));
  std::vector<std::unique_ptr<FakeGroup>> groups;
  SizedOps ops{&a, S, 0, &groups};
  std::vector<FakeReq> reqs(nreq);
  auto rnd = [&](int m) { seed = seed * 1103515245u + 12345u; return static_cast<int>((seed >> 8) % m); };
  for (int i = 0; i < nreq; ++i) reqs[i] = {i, rnd(8), 1 + rnd(12), 1 + rnd(8)};
  std::deque<FakeReq*> pending;
  int next = 0, done = 0, round = 0;
  for (; round < 20000 && done < nreq; ++round) {
    ops.round = round;
    const int burst = rnd(4) == 0 ? rnd(6) : 0;  // bursts of arrivals, idle gaps between
    for (int k = 0; k < burst && next < nreq; ++k) pending.push_back(&reqs[next++]);
    wd::admit_requests(pending, view(groups), ops, 64);
    check(a.in_use() <= sizeof(region), name, "arena never exceeded");
    for (auto& g : groups) {  // one chunk: every request in the group advances
      std::vector<FakeReq*> keep;
      FakeReq* last = nullptr;
      for (FakeReq* r : g->slots) {
        if (r != last && --r->chunks == 0) r->done_round = round, ++done;
        last = r;
        if (r->chunks > 0) keep.push_back(r);
      }
      g->slots = keep;
    }
    for (size_t i = groups.size(); i-- > 0;) {
      if (groups[i]->slots.empty() && !wd::group_wanted(pending, groups[i]->gauge, groups[i]->S, 64)) {
        a.release(groups[i]->mem);
        groups.erase(groups.begin() + static_cast<long>(i));
      }
    }
    if (next == nreq && pending.empty() && groups.empty()) break;
  }
  check(done == nreq, name, "every request finished (" + std::to_string(done) + " of " +
                                std::to_string(nreq) + " after " + std::to_string(round) + " rounds)");
  check(a.in_use() == 0, name, "memory returned");
  report(name, before);
}

}  // namespace

int main() {
  arena_scenarios();
  fifo_and_join();
  busy_group_waits();
  arena_limits_and_starvation();
  small_groups();
  small_idle_groups_released();
  simulated_serving();
  for (unsigned seed = 1; seed <= 20; ++seed) serving_mix(seed);
  std::printf("failures %d\n", failures);
  return failures == 0 ? 0 : 1;
}
