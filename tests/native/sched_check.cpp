// CPU checks of the serving engine's host-side admission (sched.hpp): the
// arena allocator against a brute-force model of the live ranges, and the
// grouping of queued same-shape requests.  Exit status 0 when every check
// holds; the first failure is printed.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "sched.hpp"

using rift2::ArenaAlloc;
using rift2::EngineReq;

#define CHECK(c, ...)                                  \
  do {                                                 \
    if (!(c)) {                                        \
      std::printf("FAIL line %d: ", __LINE__);         \
      std::printf(__VA_ARGS__);                        \
      std::printf("\n");                               \
      std::exit(1);                                    \
    }                                                  \
  } while (0)

// Free gaps of [0, size) around the live ranges (sorted, maximal).
static std::vector<std::pair<size_t, size_t>> gaps(const std::set<std::pair<size_t, size_t>>& live, size_t size) {
  std::vector<std::pair<size_t, size_t>> g;
  size_t at = 0;
  for (const auto& r : live) {
    if (r.first > at) g.push_back({at, r.first - at});
    at = r.first + r.second;
  }
  if (at < size) g.push_back({at, size - at});
  return g;
}

static void check_allocator(std::mt19937_64& rng) {
  const size_t unit = 256, size = 4096 * unit;
  ArenaAlloc a;
  a.reset(size);
  std::set<std::pair<size_t, size_t>> live;  // (offset, bytes)
  std::vector<std::pair<size_t, size_t>> order;
  for (int op = 0; op < 200000; ++op) {
    const bool take = live.empty() || (rng() % 100) < 55;
    if (take) {
      const size_t bytes = unit * (1 + rng() % 600);
      const auto g = gaps(live, size);
      size_t want = size;  // the first-fit offset of the model, size = none
      for (const auto& x : g)
        if (x.second >= bytes) {
          want = x.first;
          break;
        }
      size_t off = 0;
      const bool ok = a.alloc(bytes, &off);
      CHECK(ok == (want != size), "op %d: alloc(%zu) returned %d, model %d", op, bytes, (int)ok, (int)(want != size));
      if (ok) {
        CHECK(off == want, "op %d: first fit at %zu, model %zu", op, off, want);
        live.insert({off, bytes});
        order.push_back({off, bytes});
      }
    } else {
      const size_t k = rng() % order.size();
      const auto r = order[k];
      order[k] = order.back();
      order.pop_back();
      live.erase(r);
      a.release(r.first, r.second);
    }
    // the allocator's free map is exactly the model's gaps, fully coalesced
    const auto g = gaps(live, size);
    const auto& f = a.free_ranges();
    CHECK(f.size() == g.size(), "op %d: %zu free ranges, model %zu", op, f.size(), g.size());
    size_t i = 0;
    for (const auto& x : f) {
      CHECK(x.first == g[i].first && x.second == g[i].second, "op %d: free range %zu differs", op, i);
      ++i;
    }
  }
  for (const auto& r : order) a.release(r.first, r.second);
  CHECK(a.free_ranges().size() == 1 && a.free_ranges().begin()->first == 0 &&
            a.free_ranges().begin()->second == size,
        "released arena is not one range");
}

// Shapes 0, 3 and 4 share H and W: 3 differs in K, 4 in pixel type.
static EngineReq make_req(int64_t id, int shape) {
  static const int hw[5][3] = {{512, 512, 524}, {768, 768, 1179}, {1024, 1024, 2097}, {512, 512, 100}, {512, 512, 524}};
  EngineReq q{};
  q.req.id = id;
  q.req.dtype = shape == 4 ? RIFT2_U16 : RIFT2_U8;
  q.H = hw[shape][0];
  q.W = hw[shape][1];
  q.K = hw[shape][2];
  q.req.H = q.H;
  q.req.W = q.W;
  return q;
}

static void check_groups(std::mt19937_64& rng) {
  const size_t unit = 1 << 20, size = 64 * unit;
  for (int trial = 0; trial < 20000; ++trial) {
    ArenaAlloc a;
    a.reset(size);
    // some of the arena already taken by earlier requests
    std::vector<std::pair<size_t, size_t>> held;
    for (int k = (int)(rng() % 6); k-- > 0;) {
      size_t off;
      const size_t b = unit * (1 + rng() % 16);
      if (a.alloc(b, &off)) held.push_back({off, b});
    }
    for (size_t k = 0; k < held.size(); ++k)
      if (rng() % 3 == 0) a.release(held[k].first, held[k].second), held[k].second = 0;
    std::deque<EngineReq> pending;
    const int nq = 1 + (int)(rng() % 90);
    for (int i = 0; i < nq; ++i) pending.push_back(make_req(i, (int)(rng() % 5)));
    std::vector<int> slots;
    const int ns = 1 + (int)(rng() % 8);
    for (int s = 0; s < ns; ++s) slots.push_back(100 + s);
    const size_t bytes = unit * (1 + rng() % 12);
    const int cap = 1 + (int)(rng() % 4);
    const ArenaAlloc before = a;
    const std::deque<EngineReq> pend0 = pending;
    const std::vector<int> slots0 = slots;
    const std::vector<size_t> m = rift2::admit_group(pending, slots, a, bytes, cap);
    if (m.empty()) {
      size_t off;
      ArenaAlloc probe = before;
      CHECK(!probe.alloc(bytes, &off), "trial %d: head not admitted although it fits", trial);
      CHECK(slots == slots0 && a.free_ranges() == before.free_ranges(), "trial %d: state changed", trial);
      continue;
    }
    CHECK(m[0] == 0 && (int)m.size() <= cap && m.size() <= slots0.size(), "trial %d: group shape", trial);
    CHECK(slots.size() == slots0.size() - m.size(), "trial %d: slots taken %zu", trial, slots0.size() - slots.size());
    std::set<int> used;
    std::set<std::pair<size_t, size_t>> ranges;
    for (size_t k = 0; k < m.size(); ++k) {
      const EngineReq& q = pending[m[k]];
      CHECK(k == 0 || (m[k] > m[k - 1] && m[k] <= (size_t)rift2::kLookahead), "trial %d: member order", trial);
      const EngineReq& h = pending[0];
      CHECK(q.H == h.H && q.W == h.W && q.K == h.K && q.req.dtype == h.req.dtype,
            "trial %d: member %zu of another shape or pixel type", trial, m[k]);
      CHECK(q.batch == (int32_t)m.size() && q.bytes == bytes, "trial %d: member fields", trial);
      CHECK(used.insert(q.slot).second, "trial %d: slot %d given twice", trial, q.slot);
      ranges.insert({q.off, q.bytes});
    }
    // the members' ranges were free before and do not overlap each other
    size_t prev_end = 0;
    for (const auto& r : ranges) {
      CHECK(r.first >= prev_end, "trial %d: member ranges overlap", trial);
      prev_end = r.first + r.second;
      bool inside = false;
      for (const auto& f : before.free_ranges())
        inside = inside || (r.first >= f.first && r.first + r.second <= f.first + f.second);
      CHECK(inside, "trial %d: member range was not free", trial);
    }
    // requests left out: other shapes, beyond the look-ahead, or no room / slot / cap left
    for (size_t i = 1; i < pending.size(); ++i) {
      bool member = false;
      for (size_t k : m) member = member || k == i;
      if (member) {
        continue;
      }
      CHECK(pending[i].batch == 1 && pending[i].slot == -1, "trial %d: non-member %zu changed", trial, i);
      const EngineReq& h = pending[0];
      const bool same = pending[i].H == h.H && pending[i].W == h.W && pending[i].K == h.K &&
                        pending[i].req.dtype == h.req.dtype;
      if (same && i <= (size_t)rift2::kLookahead &&
          (int)m.size() < cap && !slots.empty()) {
        size_t off;
        ArenaAlloc probe = a;
        CHECK(!probe.alloc(bytes, &off), "trial %d: same-shape request %zu left out although it fits", trial, i);
      }
    }
    (void)pend0;
  }
}

int main() {
  std::mt19937_64 rng(20230301);
  check_allocator(rng);
  check_groups(rng);
  std::printf("sched checks passed\n");
  return 0;
}
