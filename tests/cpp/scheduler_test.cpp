// CPU unit test of the render server's request bookkeeping (scheduler.h),
// driven with fake ticks instead of GPU events.  Built with g++ by
// tests/test_scheduler_host.py; prints "ok" and exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <utility>
#include <vector>

#include "scheduler.h"

using mnr::Scheduler;
using mnr::TileRef;

struct P {
  int tag = 0;
};
using S = Scheduler<P>;

static int g_fail = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);     \
      ++g_fail;                                                    \
    }                                                              \
  } while (0)

// Runs the scheduler like the server's loop: retire the oldest in-flight
// tick, admit, compose the next; records which tiles each ticket got.
struct Driver {
  S& s;
  int next_buf = 0;
  int64_t clock = 0;
  std::map<uint64_t, std::vector<int>> tiles;  // ticket -> tiles in emission order
  std::map<int, uint64_t> slot_owner;
  std::vector<TileRef> items;
  std::vector<S::Request*> starting;
  explicit Driver(S& sc) : s(sc) {}
  void admit() {
    for (S::Request* r : s.admit(++clock)) {
      CHECK(!slot_owner.count(r->slot));  // a slot holds one request at a time
      slot_owner[r->slot] = r->ticket;
    }
  }
  bool launch() {
    const int buf = next_buf;
    if (s.tick_busy(buf)) return false;
    const int n = s.compose(buf, ++clock, items, starting);
    if (!n) return false;
    for (const TileRef& t : items) {
      CHECK(slot_owner.count(t.slot));
      tiles[slot_owner[t.slot]].push_back(t.tile);
    }
    next_buf ^= 1;
    return true;
  }
  bool retire_oldest() {
    for (int k = 0; k < 2; ++k) {
      const int buf = (next_buf + k) & 1;
      if (!s.tick_busy(buf)) continue;
      // free the slots of requests this tick finishes
      std::vector<uint64_t> before;
      s.for_each([&](const S::Request& r) { if (!r.done && r.slot >= 0) before.push_back(r.ticket); });
      s.retire(buf, ++clock);
      for (uint64_t id : before) {
        const S::Request* r = s.find(id);
        if (r && r->done) slot_owner.erase(r->slot);
      }
      return true;
    }
    return false;
  }
  void run() {
    for (int guard = 0; guard < 100000 && !s.idle(); ++guard) {
      retire_oldest();
      admit();
      launch();
      launch();
    }
    CHECK(s.idle());
  }
};

static void test_every_tile_once_and_in_order() {
  S s(1 << 20, 3, 16);
  const int n_tiles[] = {5, 40, 3, 16, 1, 7, 33};
  std::vector<uint64_t> ids;
  for (int k = 0; k < 7; ++k) {
    uint64_t t = 0;
    CHECK(s.submit(P{k}, n_tiles[k], 1000, 0, &t) == S::SUBMIT_OK);
    ids.push_back(t);
  }
  Driver d(s);
  d.run();
  for (int k = 0; k < 7; ++k) {
    const std::vector<int>& got = d.tiles[ids[k]];
    CHECK((int)got.size() == n_tiles[k]);
    for (int i = 0; i < (int)got.size(); ++i) CHECK(got[i] == i);
    int64_t t[4];
    CHECK(s.poll(ids[k], t, true) == S::POLL_DONE);
    CHECK(t[0] <= t[1] && t[1] <= t[2] && t[2] <= t[3]);
    CHECK(s.poll(ids[k], t, true) == S::POLL_UNKNOWN);  // released
  }
  CHECK(s.free_slots() == 3 && s.inflight_bytes() == 0 && s.queued_bytes() == 0);
  CHECK(s.completed() == 7 && s.failed() == 0 && s.tracked() == 0);
}

static void test_oldest_request_always_progresses() {
  // a large request keeps getting at least a quarter of each tick while
  // many small ones arrive
  S s(1 << 30, 8, 16);
  uint64_t big = 0;
  CHECK(s.submit(P{}, 64, 10, 0, &big) == S::SUBMIT_OK);
  Driver d(s);
  d.admit();
  for (int round = 0; round < 12; ++round) {
    uint64_t t = 0;
    for (int j = 0; j < 4; ++j) CHECK(s.submit(P{}, 2, 10, 0, &t) == S::SUBMIT_OK);
    d.admit();
    const size_t before = d.tiles[big].size();
    if (d.launch()) CHECK(d.tiles[big].size() >= std::min<size_t>(before + 4, 64));
    d.retire_oldest();
  }
  d.run();
  CHECK(d.tiles[big].size() == 64);
}

static void test_memory_admission_waits_then_proceeds() {
  // budget fits the resident field and one 600-byte output at a time
  S s(1000, 4, 16);
  CHECK(s.reserve_resident(300));
  uint64_t a = 0, b = 0;
  CHECK(s.submit(P{}, 4, 600, 0, &a) == S::SUBMIT_OK);
  CHECK(s.submit(P{}, 4, 600, 0, &b) == S::SUBMIT_OK);
  Driver d(s);
  d.admit();
  CHECK(s.admitted() == 1 && s.queued() == 1);     // b waits for memory
  d.run();
  CHECK(s.poll(a, nullptr, true) == S::POLL_DONE);
  CHECK(s.poll(b, nullptr, true) == S::POLL_DONE);
  uint64_t c = 0;
  CHECK(s.submit(P{}, 1, 800, 0, &c) == S::SUBMIT_TOO_BIG);  // 300 + 800 > 1000
  CHECK(s.rejected() == 1);
}

static void test_new_user_cannot_strand_a_queued_request() {
  // a queued 500-byte output must still fit once the request ahead drains:
  // a user that would push resident + queued + in-flight over the budget
  // is refused, one that leaves room is accepted
  S s(1000, 1, 16);
  uint64_t a = 0, b = 0;
  CHECK(s.submit(P{}, 2, 400, 0, &a) == S::SUBMIT_OK);
  CHECK(s.submit(P{}, 2, 500, 0, &b) == S::SUBMIT_OK);
  Driver d(s);
  d.admit();                                        // a admitted, b queued (one slot)
  CHECK(!s.reserve_resident(200));                  // 400 + 500 + 200 > 1000
  CHECK(s.reserve_resident(100));
  s.release_resident(100);                          // a registration that failed later gives it back
  CHECK(s.resident_bytes() == 0);
  CHECK(s.reserve_resident(100));
  d.run();
  CHECK(s.poll(a, nullptr, true) == S::POLL_DONE);
  CHECK(s.poll(b, nullptr, true) == S::POLL_DONE);
}

static void test_gpu_error_with_ticks_in_flight() {
  // The failure path: requests queued, admitted and in flight on both
  // ticks when the error arrives; every one finishes failed exactly once,
  // slots and bytes are all returned, and retiring the (cleared) ticks
  // afterwards changes nothing.
  S s(1 << 20, 4, 8);
  std::vector<uint64_t> ids;
  for (int k = 0; k < 6; ++k) {
    uint64_t t = 0;
    CHECK(s.submit(P{}, 6, 100, 0, &t) == S::SUBMIT_OK);
    ids.push_back(t);
  }
  Driver d(s);
  d.admit();
  CHECK(d.launch() && d.launch());
  CHECK(s.tick_busy(0) && s.tick_busy(1));
  s.fail_all(99);
  CHECK(!s.tick_busy(0) && !s.tick_busy(1));
  s.retire(0, 100);
  s.retire(1, 100);
  CHECK(s.idle());
  CHECK(s.free_slots() == 4 && s.inflight_bytes() == 0 && s.queued_bytes() == 0);
  CHECK(s.failed() == 6 && s.completed() == 0);
  for (uint64_t id : ids) CHECK(s.poll(id, nullptr, true) == S::POLL_FAILED);
  CHECK(s.tracked() == 0);
}

static void test_retire_after_partial_failure_does_not_double_free() {
  // a tick retires after the error path already finished its requests
  S s(1 << 20, 2, 8);
  uint64_t a = 0;
  CHECK(s.submit(P{}, 3, 100, 0, &a) == S::SUBMIT_OK);
  Driver d(s);
  d.admit();
  CHECK(d.launch());
  s.fail_all(5);
  s.retire(0, 6);
  s.retire(1, 6);
  CHECK(s.free_slots() == 2 && s.inflight_bytes() == 0 && s.failed() == 1 && s.completed() == 0);
  CHECK(s.poll(a, nullptr, false) == S::POLL_FAILED);
  CHECK(s.poll(12345, nullptr, true) == S::POLL_UNKNOWN);
}

int main() {
  test_every_tile_once_and_in_order();
  test_oldest_request_always_progresses();
  test_memory_admission_waits_then_proceeds();
  test_new_user_cannot_strand_a_queued_request();
  test_gpu_error_with_ticks_in_flight();
  test_retire_after_partial_failure_does_not_double_free();
  if (g_fail) {
    std::printf("%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
