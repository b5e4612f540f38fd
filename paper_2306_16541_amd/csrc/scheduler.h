// Request bookkeeping of the render server (host only, no HIP): admission by
// slot and memory budget, tick composition, retirement and failure.  The
// server (server.cpp) owns one Scheduler under its mutex and drives it from
// its scheduler thread; a CPU unit test drives it directly with fake ticks.
//
// Life of a request: submit -> queued -> admitted (slot + output bytes
// reserved) -> its tiles go out over one or more ticks -> the tick that
// carries its last tile retires -> done -> released by the caller's
// poll/wait, which erases it.  A GPU error fails every pending request.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace mnr {

struct TileRef {
  int32_t slot, tile;
};

template <class Payload>
class Scheduler {
 public:
  struct Request {
    uint64_t ticket = 0;
    Payload payload{};
    int n_tiles = 0, next_tile = 0;
    int slot = -1;
    uint64_t out_bytes = 0;
    int64_t t[4] = {0, 0, 0, 0};  // arrival, admission, first tick, completion
    bool done = false, failed = false;
  };
  enum Submit { SUBMIT_OK = 0, SUBMIT_TOO_BIG = 1 };
  enum Poll { POLL_UNKNOWN = 0, POLL_PENDING = 1, POLL_DONE = 2, POLL_FAILED = 3 };
  static constexpr int N_TICKS = 2;

  Scheduler(uint64_t budget, int max_slots, int tick_cap) : budget_(budget), tick_cap_(tick_cap) {
    for (int i = max_slots - 1; i >= 0; --i) free_slots_.push_back(i);
  }

  // Resident bytes of a new user.  Counted against what is queued and in
  // flight too, so that every queued request still fits once the requests
  // ahead of it drain (no admission stall).
  bool reserve_resident(uint64_t bytes) {
    if (resident_ + inflight_bytes_ + queued_bytes_ + bytes > budget_) return false;
    resident_ += bytes;
    return true;
  }
  void release_resident(uint64_t bytes) { resident_ = bytes < resident_ ? resident_ - bytes : 0; }

  Submit submit(const Payload& p, int n_tiles, uint64_t out_bytes, int64_t t_arrive, uint64_t* ticket) {
    if (resident_ + out_bytes > budget_) {
      ++rejected_;
      return SUBMIT_TOO_BIG;
    }
    Request r;
    r.ticket = next_ticket_++;
    r.payload = p;
    r.n_tiles = n_tiles;
    r.out_bytes = out_bytes;
    r.t[0] = t_arrive;
    *ticket = r.ticket;
    reqs_.emplace(r.ticket, r);
    queue_.push_back(r.ticket);
    queued_bytes_ += out_bytes;
    ++submitted_;
    return SUBMIT_OK;
  }

  void count_rejected() { ++rejected_; }

  // Admit queued requests in arrival order while a slot is free and the
  // budget allows; returns the admitted requests (their slots need their
  // arguments uploaded).  A front request that can never fit fails.
  std::vector<Request*> admit(int64_t now) {
    std::vector<Request*> out;
    while (!queue_.empty() && !free_slots_.empty()) {
      Request& r = reqs_.at(queue_.front());
      if (resident_ + r.out_bytes > budget_) {  // cannot fit even with nothing in flight
        queue_.pop_front();
        queued_bytes_ -= r.out_bytes;
        r.done = r.failed = true;
        r.t[3] = now;
        ++failed_;
        continue;
      }
      if (resident_ + inflight_bytes_ + r.out_bytes > budget_) break;  // wait for memory
      r.slot = free_slots_.back();
      free_slots_.pop_back();
      queued_bytes_ -= r.out_bytes;
      inflight_bytes_ += r.out_bytes;
      r.t[1] = now;
      active_.push_back(r.ticket);
      queue_.pop_front();
      out.push_back(&r);
    }
    return out;
  }

  bool tick_busy(int buf) const { return ticks_[buf].inflight; }

  // Fill tick `buf` with up to tick_cap tiles: the oldest unfinished request
  // first takes up to a quarter of the budget (no request starves), then the
  // rest goes to requests with the fewest remaining tiles, so small frames
  // overtake large ones.  `starting` receives the requests whose first tile
  // is in this tick.  Returns the tile count; a non-empty tick is marked in
  // flight until retire(buf).
  int compose(int buf, int64_t now, std::vector<TileRef>& items, std::vector<Request*>& starting) {
    Tick& t = ticks_[buf];
    items.clear();
    starting.clear();
    if (t.inflight) return 0;
    std::vector<Request*> cand;
    for (uint64_t id : active_) {
      Request& r = reqs_.at(id);
      if (r.next_tile < r.n_tiles) cand.push_back(&r);  // else: launched, awaiting completion
    }
    auto take_from = [&](Request& r, int room) {
      const int take = std::min(r.n_tiles - r.next_tile, room);
      if (take <= 0) return;
      if (r.next_tile == 0) {
        r.t[2] = now;
        starting.push_back(&r);
      }
      for (int k = 0; k < take; ++k) items.push_back(TileRef{r.slot, r.next_tile + k});
      r.next_tile += take;
      if (r.next_tile == r.n_tiles) t.finishing.push_back(r.ticket);
    };
    if (!cand.empty()) {
      take_from(*cand.front(), std::max(tick_cap_ / 4, 1));
      std::stable_sort(cand.begin(), cand.end(), [](const Request* a, const Request* b) {
        return a->n_tiles - a->next_tile < b->n_tiles - b->next_tile;
      });
      for (Request* r : cand) {
        if ((int)items.size() >= tick_cap_) break;
        take_from(*r, tick_cap_ - (int)items.size());
      }
    }
    if (!items.empty()) {
      t.inflight = true;
      ++ticks_launched_;
      tiles_ += items.size();
    }
    return (int)items.size();
  }

  // Tick `buf` finished: its finishing requests are done; their slots and
  // output bytes are free again.
  void retire(int buf, int64_t now) {
    Tick& t = ticks_[buf];
    for (uint64_t id : t.finishing) complete(id, now, false);
    t.finishing.clear();
    t.inflight = false;
  }

  // A GPU error: every queued, admitted or in-flight request is done and
  // failed; nothing is in flight any more.
  void fail_all(int64_t now) {
    for (uint64_t id : queue_) {
      Request& r = reqs_.at(id);
      r.done = r.failed = true;
      r.t[3] = now;
      ++failed_;
    }
    queue_.clear();
    queued_bytes_ = 0;
    const std::vector<uint64_t> act = active_;
    for (uint64_t id : act) complete(id, now, true);
    for (Tick& t : ticks_) {
      t.finishing.clear();
      t.inflight = false;
    }
  }

  // State of a ticket; a finished ticket is erased when `release` is set.
  Poll poll(uint64_t ticket, int64_t* t_ns, bool release) {
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return POLL_UNKNOWN;
    const Request& r = it->second;
    if (t_ns)
      for (int k = 0; k < 4; ++k) t_ns[k] = r.t[k];
    if (!r.done) return POLL_PENDING;
    const Poll p = r.failed ? POLL_FAILED : POLL_DONE;
    if (release) reqs_.erase(it);
    return p;
  }

  const Request* find(uint64_t ticket) const {
    auto it = reqs_.find(ticket);
    return it == reqs_.end() ? nullptr : &it->second;
  }

  template <class F>
  void for_each(F f) const {
    for (const auto& kv : reqs_) f(kv.second);
  }

  bool idle() const {
    return queue_.empty() && active_.empty() && !ticks_[0].inflight && !ticks_[1].inflight;
  }
  bool has_queue() const { return !queue_.empty(); }

  // counters
  uint64_t submitted() const { return submitted_; }
  uint64_t completed() const { return completed_; }
  uint64_t rejected() const { return rejected_; }
  uint64_t failed() const { return failed_; }
  uint64_t ticks() const { return ticks_launched_; }
  uint64_t tiles() const { return tiles_; }
  int queued() const { return (int)queue_.size(); }
  int admitted() const { return (int)active_.size(); }
  int free_slots() const { return (int)free_slots_.size(); }
  size_t tracked() const { return reqs_.size(); }
  uint64_t budget() const { return budget_; }
  uint64_t resident_bytes() const { return resident_; }
  uint64_t inflight_bytes() const { return inflight_bytes_; }
  uint64_t queued_bytes() const { return queued_bytes_; }

 private:
  struct Tick {
    bool inflight = false;
    std::vector<uint64_t> finishing;
  };

  // Finish an admitted request once; a ticket that is unknown, already done
  // or not admitted is left alone.
  void complete(uint64_t ticket, int64_t now, bool failed) {
    auto it = reqs_.find(ticket);
    if (it == reqs_.end() || it->second.done) return;
    auto a = std::find(active_.begin(), active_.end(), ticket);
    if (a == active_.end()) return;
    Request& r = it->second;
    active_.erase(a);
    r.done = true;
    r.failed = failed;
    r.t[3] = now;
    free_slots_.push_back(r.slot);
    inflight_bytes_ -= r.out_bytes;
    if (failed)
      ++failed_;
    else
      ++completed_;
  }

  uint64_t budget_ = 0, resident_ = 0, inflight_bytes_ = 0, queued_bytes_ = 0;
  int tick_cap_ = 1;
  std::map<uint64_t, Request> reqs_;
  std::deque<uint64_t> queue_;    // waiting for admission, arrival order
  std::vector<uint64_t> active_;  // admitted, oldest first
  std::vector<int> free_slots_;
  Tick ticks_[N_TICKS];
  uint64_t next_ticket_ = 1;
  uint64_t submitted_ = 0, completed_ = 0, rejected_ = 0, failed_ = 0, ticks_launched_ = 0, tiles_ = 0;
};

}  // namespace mnr
