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

// The executor: opens groups in an arena (group_bytes each) and records
// placements.
struct FakeOps {
  wd::Arena* arena;
  size_t group_bytes;
  int S;
  int round = 0;
  std::vector<std::unique_ptr<FakeGroup>>* groups;
  FakeGroup* make_group(int gauge) {
    char* m = arena->alloc(group_bytes);
    if (m == nullptr) return nullptr;
    groups->push_back(std::make_unique<FakeGroup>());
    FakeGroup* g = groups->back().get();
    g->gauge = gauge;
    g->S = S;
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
      if (groups[i]->slots.empty() && !wd::group_wanted(pending, groups[i]->gauge, 16)) {
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

}  // namespace

int main() {
  arena_scenarios();
  fifo_and_join();
  busy_group_waits();
  arena_limits_and_starvation();
  simulated_serving();
  std::printf("failures %d\n", failures);
  return failures == 0 ? 0 : 1;
}
