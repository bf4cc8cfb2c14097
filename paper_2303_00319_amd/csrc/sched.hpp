// Host-side admission of the serving engine: the arena allocator and the
// choice of the requests admitted together.  Plain C++ with no device calls,
// so the same code the engine runs is unit-tested on the CPU.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

#include "rift2.h"

namespace rift2 {

// First-fit allocator over [0, size) with coalescing of freed ranges.
class ArenaAlloc {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  // The lowest free range that holds `bytes`; false (and nothing taken) when
  // none does.
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  // Returns a range taken by alloc; it merges with free neighbours.
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  const std::map<size_t, size_t>& free_ranges() const { return free_; }

 private:
  std::map<size_t, size_t> free_;
};

// One queued or admitted request.
struct EngineReq {
  rift2_request req;
  int H, W, K;
  size_t off = 0, bytes = 0;
  int slot = -1;
  int32_t status = RIFT2_OK;
  int32_t batch = 1;  // requests admitted together with this one
};

// Requests whose filter banks can share launches: same size, type and
// keypoint count (so the same buffer layout).
inline bool engine_same_shape(const EngineReq& a, const EngineReq& b) {
  return a.H == b.H && a.W == b.W && a.K == b.K && a.req.dtype == b.req.dtype;
}

constexpr int kLookahead = 64;  // queued requests looked at for a group

// Admits the head of `pending` (which needs `bytes` of arena) and, with it,
// queued requests of its shape that also fit, in queue order, up to `cap`
// requests and looking at most kLookahead entries ahead; each gets an arena
// range and a slot from `free_slots`, and its `batch` is set to the group
// size.  Returns the members' indices in `pending`, head first, ascending; an
// empty result means the head must wait for memory (nothing is taken).  The
// caller has checked that a slot is free.
inline std::vector<size_t> admit_group(std::deque<EngineReq>& pending, std::vector<int>& free_slots,
                                       ArenaAlloc& alloc, size_t bytes, int cap) {
  std::vector<size_t> members;
  if (pending.empty() || free_slots.empty()) return members;
  size_t off = 0;
  if (!alloc.alloc(bytes, &off)) return members;
  EngineReq& q = pending.front();
  q.off = off;
  q.bytes = bytes;
  q.slot = free_slots.back();
  free_slots.pop_back();
  members.push_back(0);
  for (size_t i = 1; i < pending.size() && (int)i <= kLookahead && (int)members.size() < cap && !free_slots.empty();
       ++i) {
    EngineReq& o = pending[i];
    if (!engine_same_shape(o, q) || !alloc.alloc(bytes, &off)) continue;
    o.off = off;
    o.bytes = bytes;
    o.slot = free_slots.back();
    free_slots.pop_back();
    members.push_back(i);
  }
  for (size_t k : members) pending[k].batch = (int32_t)members.size();
  return members;
}

}  // namespace rift2
