// Request scheduling for the sampling server: the HBM arena, admission and
// the per-tick work split.  No device calls here; the server (server.hip)
// drives it and the C++ unit test drives it with a fake clock.
//
// Lifecycle of a request: QUEUED (waiting for a slot and arena space) ->
// ACTIVE (its output lives in the arena; its 64-shot words are sampled in
// chunks, a fair share per launch tick) -> DONE (every word written; the
// slot is free again) -> released by the caller (the arena space is free
// again).  Admission is FIFO: a request that does not fit yet blocks the
// ones behind it, so large requests are never starved by small ones.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

namespace sp {
namespace serve {

enum State : int { QUEUED = 0, ACTIVE = 1, DONE = 2, FAILED = 3 };

// First-fit allocator over [0, capacity) with 256-byte granularity.
class Arena {
 public:
  explicit Arena(size_t capacity) : cap_(capacity & ~(size_t)255) {
    if (cap_) free_[0] = cap_;
  }
  static size_t round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round(bytes ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t capacity() const { return cap_; }
  size_t in_use() const { return used_; }
  size_t free_blocks() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;
  size_t cap_, used_ = 0;
};

struct Request {
  uint64_t ticket = 0;
  const void* model = nullptr;   // opaque to the scheduler
  uint32_t n_meas = 0, nb = 0;   // output rows and Philox blocks per shot, over all row tiles
  uint32_t tiles = 1;            // row tiles: each word costs one group per tile
  int path = 0;
  uint64_t seed = 0, first_shot = 0, shots = 0;
  uint64_t words = 0;            // ceil(shots / 64) = ld of the output
  size_t bytes = 0, off = 0;     // arena footprint and offset
  uint64_t next_word = 0, words_done = 0;
  int state = QUEUED;
  uint64_t t_submit = 0, t_admit = 0, t_done = 0;
  std::string error;
};

// Words [w0, w1) of one request, sampled in one tick.
struct Chunk {
  uint64_t ticket, w0, w1;
};

class Scheduler {
 public:
  // tick_cost: Philox block-words (model blocks x 64-shot words) per tick;
  // max_groups: cap on word groups per tick; words_per_group: launch shape.
  Scheduler(size_t arena_bytes, uint32_t max_active, uint32_t max_queued, uint64_t tick_cost, uint32_t max_groups,
            uint32_t words_per_group)
      : arena_(arena_bytes),
        max_active_(std::max<uint32_t>(1, max_active)),
        max_queued_(max_queued),
        tick_cost_(std::max<uint64_t>(1, tick_cost)),
        max_groups_(std::max<uint32_t>(1, max_groups)),
        wpg_(std::max<uint32_t>(1, words_per_group)) {}

  // 0: queued (or done at once for zero shots); 1: refused because the
  // output can never fit in the arena; 2: refused because the queue is full;
  // 3: refused because one word of every row tile exceeds a tick's groups.
  int submit(Request r, uint64_t now, uint64_t* ticket) {
    r.words = (r.shots + 63) / 64;
    r.bytes = Arena::round((size_t)r.n_meas * r.words * 8);
    if (r.bytes > arena_.capacity()) return 1;
    if (std::max<uint32_t>(1, r.tiles) > max_groups_) return 3;
    if (queue_.size() >= max_queued_) return 2;
    r.ticket = ++last_ticket_;
    r.t_submit = now;
    r.state = QUEUED;
    *ticket = r.ticket;
    if (r.words == 0 || r.n_meas == 0) {
      r.state = DONE;
      r.t_admit = r.t_done = now;
      r.bytes = 0;
      reqs_[r.ticket] = r;
      return 0;
    }
    reqs_[r.ticket] = r;
    queue_.push_back(r.ticket);
    return 0;
  }

  // FIFO admission while slots and arena space allow.  Returns admitted tickets.
  std::vector<uint64_t> admit(uint64_t now) {
    std::vector<uint64_t> out;
    while (!queue_.empty() && active_.size() < max_active_) {
      Request& r = reqs_[queue_.front()];
      size_t off = 0;
      if (!arena_.alloc(r.bytes, &off)) break;
      r.off = off;
      r.state = ACTIVE;
      r.t_admit = now;
      active_.push_back(r.ticket);
      out.push_back(r.ticket);
      queue_.pop_front();
    }
    return out;
  }

  // The next tick: every active request with words left gets a share of
  // the tick's cost budget (at least one group per row tile), visiting
  // requests in a rotating order so that no request waits for another to
  // finish.  A request whose tiles no longer fit the tick's groups waits for
  // the next tick (the first request visited always fits).
  std::vector<Chunk> next_tick() {
    std::vector<Chunk> tick;
    std::vector<uint64_t> open;
    for (uint64_t t : active_)
      if (reqs_[t].next_word < reqs_[t].words) open.push_back(t);
    if (open.empty()) return tick;
    const size_t n = open.size();
    const size_t start = rr_ % n;
    rr_ = start + 1;
    uint64_t cost_left = tick_cost_;
    uint64_t groups_left = max_groups_;
    const uint64_t share = std::max<uint64_t>(1, tick_cost_ / n);
    for (size_t i = 0; i < n && groups_left > 0; ++i) {
      Request& r = reqs_[open[(start + i) % n]];
      const uint64_t nb = std::max<uint32_t>(1, r.nb);
      const uint64_t tiles = std::max<uint32_t>(1, r.tiles);
      uint64_t words = std::max<uint64_t>(wpg_, (std::min(share, cost_left) / nb) / wpg_ * wpg_);
      words = std::min<uint64_t>(words, groups_left / tiles * wpg_);
      words = std::min<uint64_t>(words, r.words - r.next_word);
      if (words == 0) continue;
      tick.push_back({r.ticket, r.next_word, r.next_word + words});
      r.next_word += words;
      groups_left -= tiles * ((words + wpg_ - 1) / wpg_);
      const uint64_t cost = words * nb;
      cost_left = cost_left > cost ? cost_left - cost : 0;
      if (cost_left == 0 && i + 1 < n) {
        rr_ = start + i + 1;   // the budget is spent; the requests not visited go first next tick
        break;
      }
    }
    return tick;
  }

  // The tick's words are written (ok) or its launch failed.
  std::vector<uint64_t> complete(const std::vector<Chunk>& tick, uint64_t now, bool ok, const std::string& err = "") {
    std::vector<uint64_t> finished;
    for (const Chunk& c : tick) {
      Request& r = reqs_[c.ticket];
      if (r.state != ACTIVE) continue;
      if (!ok) {
        r.state = FAILED;
        r.error = err;
      } else {
        r.words_done += c.w1 - c.w0;
        if (r.words_done < r.words) continue;
        r.state = DONE;
      }
      r.t_done = now;
      active_.erase(std::find(active_.begin(), active_.end(), r.ticket));
      finished.push_back(r.ticket);
    }
    return finished;
  }

  // Frees a finished request's arena space and forgets it.  -1: unknown
  // ticket, -2: not finished yet.
  int release(uint64_t ticket) {
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return -1;
    if (it->second.state != DONE && it->second.state != FAILED) return -2;
    if (it->second.bytes) arena_.release(it->second.off, it->second.bytes);
    reqs_.erase(it);
    return 0;
  }

  // Marks every queued or active request failed (server shutdown).
  void fail_all(uint64_t now, const std::string& why) {
    for (auto& kv : reqs_) {
      Request& r = kv.second;
      if (r.state == QUEUED || r.state == ACTIVE) {
        if (r.state == QUEUED) r.bytes = 0;   // never got arena space
        r.state = FAILED;
        r.error = why;
        r.t_done = now;
      }
    }
    queue_.clear();
    active_.clear();
  }

  const Request* find(uint64_t ticket) const {
    auto it = reqs_.find(ticket);
    return it == reqs_.end() ? nullptr : &it->second;
  }
  size_t queued() const { return queue_.size(); }
  size_t active() const { return active_.size(); }
  const Arena& arena() const { return arena_; }
  bool idle() const { return queue_.empty() && active_.empty(); }

 private:
  Arena arena_;
  uint32_t max_active_, max_queued_;
  uint64_t tick_cost_;
  uint32_t max_groups_, wpg_;
  std::unordered_map<uint64_t, Request> reqs_;
  std::deque<uint64_t> queue_;
  std::vector<uint64_t> active_;
  uint64_t last_ticket_ = 0;
  size_t rr_ = 0;
};

}  // namespace serve
}  // namespace sp
