// Unit test of the serving scheduler (admission, arena, tick split) with a
// fake clock and a fake device: ticks "complete" when the test says so.
// Exit status 0 = all checks passed.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>

#include "../../paper_2311_03906_amd/csrc/server_core.hpp"

using namespace sp::serve;

static int failures = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);       \
      ++failures;                                                    \
    }                                                                \
  } while (0)

static Request req(uint32_t n_meas, uint32_t nb, uint64_t shots) {
  Request r;
  r.n_meas = n_meas;
  r.nb = nb;
  r.shots = shots;
  return r;
}

static void test_arena() {
  Arena a(4096);
  size_t o1, o2, o3, o4;
  CHECK(a.alloc(1000, &o1) && o1 == 0);
  CHECK(a.alloc(1000, &o2) && o2 == 1024);
  CHECK(a.alloc(2048, &o3) && o3 == 2048);
  CHECK(!a.alloc(1, &o4));
  CHECK(a.in_use() == 4096);
  a.release(o2, 1000);
  CHECK(a.alloc(256, &o4) && o4 == 1024);   // first fit
  a.release(o4, 256);
  a.release(o1, 1000);
  CHECK(a.free_blocks() == 1);              // [0, 2048) coalesced
  a.release(o3, 2048);
  CHECK(a.free_blocks() == 1 && a.in_use() == 0);
  CHECK(a.alloc(4096, &o1) && o1 == 0);
}

static void test_refusal_and_zero_shots() {
  Scheduler s(1 << 20, 4, 2, 1000, 1024, 1);
  uint64_t t;
  CHECK(s.submit(req(1000, 10, 64 * 200), 0, &t) == 1);   // 1.6 MB > 1 MiB arena
  CHECK(s.submit(req(10, 10, 0), 0, &t) == 0);
  CHECK(s.find(t)->state == DONE);
  CHECK(s.release(t) == 0);
  CHECK(s.submit(req(10, 10, 64), 0, &t) == 0);
  CHECK(s.submit(req(10, 10, 64), 0, &t) == 0);
  CHECK(s.submit(req(10, 10, 64), 0, &t) == 2);           // queue of 2 is full
}

static void test_fifo_admission_and_slots() {
  // arena of 100 KiB; request sizes 8 * n_meas * words bytes
  Scheduler s(100 << 10, 2, 100, 1 << 20, 1 << 16, 1);
  uint64_t a, b, c, d;
  s.submit(req(100, 10, 64 * 64), 0, &a);    // 51200 B
  s.submit(req(100, 10, 64 * 65), 1, &b);    // 52000 B: does not fit beside a in 102400 B
  s.submit(req(10, 10, 64), 2, &c);          // tiny
  s.submit(req(10, 10, 64), 3, &d);
  auto adm = s.admit(10);
  CHECK(adm.size() == 1 && adm[0] == a);     // b does not fit next to a (FIFO: c, d wait behind b)
  CHECK(s.find(c)->state == QUEUED);
  auto tick = s.next_tick();
  CHECK(tick.size() == 1 && tick[0].ticket == a);
  CHECK(tick[0].w1 - tick[0].w0 == 64);      // whole request fits the budget
  auto fin = s.complete(tick, 20, true);
  CHECK(fin.size() == 1 && s.find(a)->state == DONE && s.find(a)->t_done == 20);
  CHECK(s.admit(21).empty());                // a still holds its arena space
  CHECK(s.release(a) == 0);
  adm = s.admit(22);
  CHECK(adm.size() == 2 && adm[0] == b && adm[1] == c);   // two slots
  CHECK(s.find(d)->state == QUEUED);
}

static void test_fair_ticks() {
  // budget 10000 block-words; two requests with nb = 100 => 50 words each per tick
  Scheduler s(1 << 30, 8, 100, 10000, 1 << 16, 2);
  uint64_t a, b;
  s.submit(req(10, 100, 64 * 1000), 0, &a);
  s.submit(req(10, 100, 64 * 30), 0, &b);
  s.admit(0);
  auto t1 = s.next_tick();
  CHECK(t1.size() == 2);
  uint64_t wa = 0, wb = 0;
  for (auto& c : t1) (c.ticket == a ? wa : wb) += c.w1 - c.w0;
  CHECK(wa == 50 && wb == 30);               // b finishes in its first tick
  s.complete(t1, 1, true);
  CHECK(s.find(b)->state == DONE);
  auto t2 = s.next_tick();
  CHECK(t2.size() == 1 && t2[0].ticket == a && t2[0].w0 == 50 && t2[0].w1 == 150);   // a alone: whole budget
  // a failed tick fails its requests
  s.complete(t2, 2, false, "device error");
  CHECK(s.find(a)->state == FAILED && s.find(a)->error == "device error");
}

static void test_small_budget_keeps_everyone_moving() {
  // budget smaller than one group of a heavy request: every request still
  // gets at least one group per tick
  Scheduler s(1 << 30, 8, 100, 10, 1 << 16, 1);
  uint64_t a, b;
  s.submit(req(10, 10000, 64 * 5), 0, &a);
  s.submit(req(10, 10000, 64 * 5), 0, &b);
  s.admit(0);
  std::set<uint64_t> seen;
  for (int i = 0; i < 4; ++i) {
    auto t = s.next_tick();
    CHECK(!t.empty());
    for (auto& c : t) seen.insert(c.ticket);
    s.complete(t, i, true);
  }
  CHECK(seen.size() == 2);
}

static void test_random_backpressure() {
  // random arrivals against a tiny arena: capacity is never exceeded, every
  // request finishes, words are written exactly once
  std::mt19937_64 rng(7);
  const size_t cap = 64 << 10;
  Scheduler s(cap, 3, 1000, 5000, 64, 2);
  std::vector<uint64_t> tickets;
  std::map<uint64_t, uint64_t> written;
  uint64_t now = 0;
  for (int i = 0; i < 300; ++i) {
    uint64_t t;
    const uint64_t shots = 1 + rng() % (64 * 100);
    const uint32_t n_meas = 1 + rng() % 60;
    if (s.submit(req(n_meas, 1 + rng() % 500, shots), now, &t) == 0) tickets.push_back(t);
    for (int k = 0; k < 3; ++k) {
      s.admit(++now);
      CHECK(s.arena().in_use() <= cap);
      auto tick = s.next_tick();
      for (auto& c : tick) {
        CHECK(c.w1 > c.w0);
        CHECK(c.w0 == written[c.ticket]);   // contiguous, no overlap, no gap
        written[c.ticket] = c.w1;
      }
      for (uint64_t f : s.complete(tick, ++now, true)) {
        CHECK(written[f] == s.find(f)->words);
        CHECK(s.release(f) == 0);
      }
    }
  }
  for (int k = 0; k < 100000 && !s.idle(); ++k) {
    s.admit(++now);
    auto tick = s.next_tick();
    for (auto& c : tick) written[c.ticket] = c.w1;
    for (uint64_t f : s.complete(tick, ++now, true)) s.release(f);
  }
  CHECK(s.idle());
  CHECK(s.arena().in_use() == 0);
  CHECK(written.size() <= tickets.size());
}

// Row-tiled requests: a word costs one group per tile, a tick never exceeds
// its groups, a request whose tiles do not fit waits for a later tick, and
// a request with more tiles than a tick's groups is refused.
static void test_row_tiles() {
  Scheduler s(1 << 30, 4, 100, 1 << 20, 16, 1);
  uint64_t t;
  Request big = req(100, 10, 64 * 40);
  big.tiles = 17;
  CHECK(s.submit(big, 0, &t) == 3);
  Request a = req(100, 10, 64 * 40), b = req(10, 10, 64 * 40);
  a.tiles = 5;
  uint64_t ta, tb;
  CHECK(s.submit(a, 0, &ta) == 0);
  CHECK(s.submit(b, 0, &tb) == 0);
  s.admit(0);
  uint64_t now = 0, words_a = 0, words_b = 0;
  int ticks = 0;
  while (!s.idle() && ticks < 1000) {
    auto tick = s.next_tick();
    CHECK(!tick.empty());
    uint64_t groups = 0;
    for (const Chunk& c : tick) {
      const uint64_t w = c.w1 - c.w0;
      groups += (c.ticket == ta ? 5 : 1) * w;
      (c.ticket == ta ? words_a : words_b) += w;
    }
    CHECK(groups <= 16);
    for (uint64_t f : s.complete(tick, ++now, true)) s.release(f);
    ++ticks;
  }
  CHECK(words_a == 40 && words_b == 40);
  CHECK(s.idle() && s.arena().in_use() == 0);
}

static void test_fail_all() {
  Scheduler s(1 << 20, 1, 10, 100, 16, 1);
  uint64_t a, b;
  s.submit(req(10, 10, 640), 0, &a);
  s.submit(req(10, 10, 640), 0, &b);
  s.admit(0);
  s.fail_all(5, "stopped");
  CHECK(s.find(a)->state == FAILED && s.find(b)->state == FAILED);
  CHECK(s.release(a) == 0 && s.release(b) == 0);
  CHECK(s.arena().in_use() == 0);
}

int main() {
  test_arena();
  test_refusal_and_zero_shots();
  test_fifo_admission_and_slots();
  test_fair_ticks();
  test_small_budget_keeps_everyone_moving();
  test_random_backpressure();
  test_row_tiles();
  test_fail_all();
  if (failures) {
    std::printf("%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("server core: all checks passed\n");
  return 0;
}
