// Scheduling policy of the request server, free of device code so that it can
// be exercised on the host with a fake executor: the arena allocator and the
// admission of queued requests into solve groups.
#pragma once

#include <algorithm>
#include <cstddef>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace wd {

// First-fit allocator over a caller-given region (offsets aligned to 256 B).
class Arena {
 public:
  void init(char* base, size_t bytes) {
    base_ = base;
    free_.clear();
    used_.clear();
    in_use_ = peak_ = 0;
    if (bytes > 0) free_[0] = bytes;
  }
  char* alloc(size_t n) {
    n = (n + 255) & ~static_cast<size_t>(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > n) free_[off + n] = sz - n;
      used_[off] = n;
      in_use_ += n;
      peak_ = std::max(peak_, in_use_);
      return base_ + off;
    }
    return nullptr;
  }
  void release(char* p) {
    if (p == nullptr) return;
    const size_t off = static_cast<size_t>(p - base_);
    auto it = used_.find(off);
    if (it == used_.end()) return;
    size_t start = off, size = it->second;
    in_use_ -= size;
    used_.erase(it);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + size) {
      size += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        size += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = size;
  }
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }
  size_t free_blocks() const { return free_.size(); }

 private:
  char* base_ = nullptr;
  std::map<size_t, size_t> free_, used_;
  size_t in_use_ = 0, peak_ = 0;
};

// Admits queued requests, in arrival order, into groups of their gauge field
// with enough free slots, creating a group when none exists and the arena has
// room (the executor decides its size: at least the request's right-hand
// sides). A group that is running a chunk is not joined now, but a request it
// could take waits for it rather than opening a second group. A request that
// cannot be placed is passed over (its `skipped` count grows each time a later
// request is admitted before it); once passed over more than `starve_skips`
// times, nothing behind it is admitted until it has been. Returns whether any
// request was admitted.
//
// Req needs: gauge, nrhs(), skipped. Group needs: gauge, free_slots(), ready().
// Ops needs: Group* make_group(gauge, need) (a group with at least `need`
// slots, nullptr if none fits) and void place(Group*, Req*) (assign slots and
// start them).
template <class Req, class Group, class Ops>
bool admit_requests(std::deque<Req*>& pending, const std::vector<Group*>& groups, Ops& ops,
                    int starve_skips) {
  bool did = false;
  std::vector<Req*> waiting;  // requests this scan has passed over so far
  std::vector<Group*> made;   // groups opened during this scan
  for (auto it = pending.begin(); it != pending.end();) {
    Req* rq = *it;
    Group* target = nullptr;
    bool busy_group_has_room = false;
    const std::vector<Group*>* lists[2] = {&groups, &made};
    for (const std::vector<Group*>* list : lists)
      for (Group* g : *list) {
        if (target != nullptr || g->gauge != rq->gauge || g->free_slots() < rq->nrhs()) continue;
        if (g->ready()) target = g;
        else busy_group_has_room = true;  // it takes the request at its next chunk boundary
      }
    if (target == nullptr && !busy_group_has_room) {
      target = ops.make_group(rq->gauge, rq->nrhs());
      if (target != nullptr) made.push_back(target);
    }
    if (target == nullptr) {
      if (rq->skipped > starve_skips) break;  // starving: nothing behind it may overtake
      waiting.push_back(rq);
      ++it;
      continue;
    }
    ops.place(target, rq);
    for (Req* w : waiting) w->skipped++;
    it = pending.erase(it);
    did = true;
  }
  return did;
}

// Whether an idle group of `gauge` with `slots` slots should be kept for a
// queued request. Only requests that can be admitted count: those up to and
// including the first starving one (nothing behind a starving request is
// admitted before it), so that idle groups of other gauges give their memory
// to the starving request instead of being held, forever, for requests queued
// behind it; and only requests the group can hold, so that a group opened
// small (for a request that found no room for a full one) gives its memory
// back to the larger requests of its gauge.
template <class Req, class Gauge>
bool group_wanted(const std::deque<Req*>& pending, const Gauge& gauge, int slots, int starve_skips) {
  for (const Req* r : pending) {
    if (r->gauge == gauge && r->nrhs() <= slots) return true;
    if (r->skipped > starve_skips) return false;
  }
  return false;
}

}  // namespace wd
