// Multi-user continuous-batching render server (host side).  See
// include/metanerf_server.h for the contract.
//
// One scheduler thread owns the GPU side: it retires finished ticks,
// admits queued requests (free slot + memory budget), and launches the next
// tick whenever fewer than two are in flight.  A tick renders up to
// tiles_per_tick 16x16 tiles taken from admitted requests; a request
// completes with the tick that renders its last tile (tick composition: see
// launch_locked).  Ticks are replayed from two captured hipGraphs (tile-table
// upload + tick kernel), alternating between two tile tables so the host can
// fill one while the GPU reads the other.  Each table has its own stream, so
// the next tick's blocks take over compute units as the previous tick's
// last blocks drain instead of waiting for the whole grid; ticks still
// retire in launch order.  Per-request arguments go up on a third stream
// that every tick waits on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/metanerf_server.h"
#include "host_common.h"
#include "kernels.h"

namespace mnr {

static int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket = 0;
  int user = 0;
  RenderArgs args;
  int n_tiles = 0, next_tile = 0;
  int slot = -1;
  uint64_t out_bytes = 0;
  int64_t t[4] = {0, 0, 0, 0};  // arrival, admission, first tick, completion
  bool done = false;
};

struct User {
  mnr_field field;
  mnr_motion motion;
  uint64_t bytes;
};

struct Tick {
  hipEvent_t ev = nullptr;
  bool inflight = false;
  std::vector<uint64_t> finishing;
};

static uint64_t field_bytes(const mnr_field& f, const mnr_motion& m) {
  const uint64_t el = f.table_dtype == MNR_F32 ? 4 : 2, wl = f.mlp_dtype == MNR_F32 ? 4 : 2;
  uint64_t b = (uint64_t)f.n_levels * ((uint64_t)1 << f.log2_T) * f.n_feat * el;
  for (int k = 0; k < f.n_layers; ++k) b += (uint64_t)f.width[k] * f.width[k + 1] * wl;
  b += (uint64_t)(m.n_bones + 1) * m.res * m.res * m.res * 4;
  if (m.packed) b += mnr_motion_packed_bytes(m.res, m.n_bones);
  if (f.dense_packed) b += mnr_field_packed_bytes(&f);
  return b;
}

}  // namespace mnr

using namespace mnr;

struct mnr_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stop = false;
  hipError_t gpu_err = hipSuccess;
  int device = 0;
  uint64_t budget = 0, resident = 0, inflight_bytes = 0;
  int max_slots = 0, tick_cap = 0;
  bool have_format = false;
  mnr_dtype table_dt = MNR_F32, mlp_dt = MNR_F32;
  int nhh = 0;
  std::map<int, User> users;
  std::map<uint64_t, Request> reqs;
  std::deque<uint64_t> queue;    // waiting for admission
  std::vector<uint64_t> active;  // admitted, oldest first
  std::vector<int> free_slots;
  uint64_t next_ticket = 1;
  mnr_server_stats st{};
  // device side
  hipStream_t stream[2] = {nullptr, nullptr};  // one per tick buffer
  hipStream_t copy_stream = nullptr;            // request arguments
  hipEvent_t copy_ev = nullptr;                 // after the latest argument upload
  bool copy_wait[2] = {false, false};           // tick stream must wait on copy_ev
  RenderArgs* d_slots = nullptr;
  RenderArgs* h_slots = nullptr;  // pinned staging, one per slot
  WorkTable* d_wt[2] = {nullptr, nullptr};
  WorkTable* h_wt[2] = {nullptr, nullptr};
  size_t wt_bytes = 0;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  Tick ticks[2];
  int next_buf = 0;

  void loop();
  bool retire_locked();
  bool admit_locked();
  bool launch_locked();
};

static void complete_locked(mnr_server* s, uint64_t ticket, int64_t t_done) {
  Request& r = s->reqs[ticket];
  r.done = true;
  r.t[3] = t_done;
  s->free_slots.push_back(r.slot);
  s->inflight_bytes -= r.out_bytes;
  s->active.erase(std::find(s->active.begin(), s->active.end(), ticket));
  s->st.completed++;
}

bool mnr_server::retire_locked() {
  bool any = false;
  for (int k = 0; k < 2; ++k) {
    Tick& t = ticks[(next_buf + k) & 1];  // oldest first
    if (!t.inflight) continue;
    const hipError_t q = hipEventQuery(t.ev);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess && gpu_err == hipSuccess) gpu_err = q;
    const int64_t tn = now_ns();
    for (uint64_t id : t.finishing) complete_locked(this, id, tn);
    t.finishing.clear();
    t.inflight = false;
    any = true;
  }
  if (any) cv_done.notify_all();
  return any;
}

bool mnr_server::admit_locked() {
  bool any = false;
  while (!queue.empty() && !free_slots.empty()) {
    Request& r = reqs[queue.front()];
    if (resident + inflight_bytes + r.out_bytes > budget) break;  // wait for memory
    r.slot = free_slots.back();
    free_slots.pop_back();
    inflight_bytes += r.out_bytes;
    r.t[1] = now_ns();
    h_slots[r.slot] = r.args;
    const hipError_t e = hipMemcpyAsync(d_slots + r.slot, h_slots + r.slot, sizeof(RenderArgs),
                                        hipMemcpyHostToDevice, copy_stream);
    if (e != hipSuccess && gpu_err == hipSuccess) gpu_err = e;
    active.push_back(r.ticket);
    queue.pop_front();
    any = true;
  }
  if (any) {  // a slot is rewritten only after every tick that read it retired
    const hipError_t e = hipEventRecord(copy_ev, copy_stream);
    if (e != hipSuccess && gpu_err == hipSuccess) gpu_err = e;
    copy_wait[0] = copy_wait[1] = true;
  }
  return any;
}

bool mnr_server::launch_locked() {
  const int buf = next_buf;
  Tick& t = ticks[buf];
  if (t.inflight) return false;
  WorkTable* w = h_wt[buf];
  int n = 0;
  const int64_t tn = now_ns();
  // Tick composition: the oldest unfinished request first takes up to a
  // quarter of the tile budget (no request starves), then the rest of the
  // budget goes to requests with the fewest remaining tiles, so small
  // frames overtake large ones instead of queueing behind them.
  std::vector<Request*> cand;
  for (uint64_t id : active) {
    Request& r = reqs[id];
    if (r.next_tile < r.n_tiles) cand.push_back(&r);  // else: launched, awaiting completion
  }
  auto take_from = [&](Request& r, int budget) {
    const int take = std::min(r.n_tiles - r.next_tile, budget);
    if (take <= 0) return;
    if (r.next_tile == 0) r.t[2] = tn;
    for (int k = 0; k < take; ++k) w->items[n + k] = WorkItem{r.slot, r.next_tile + k};
    n += take;
    r.next_tile += take;
    if (r.next_tile == r.n_tiles) t.finishing.push_back(r.ticket);
  };
  if (!cand.empty()) {
    take_from(*cand.front(), std::max(tick_cap / 4, 1));
    std::stable_sort(cand.begin(), cand.end(), [](const Request* a, const Request* b) {
      return a->n_tiles - a->next_tile < b->n_tiles - b->next_tile;
    });
    for (Request* r : cand) {
      if (n >= tick_cap) break;
      take_from(*r, tick_cap - n);
    }
  }
  if (n == 0) return false;
  w->counter = 0;
  w->n_items = n;
  hipStream_t sb = stream[buf];
  if (!graph[buf]) {  // capture this buffer's tick once: table upload + tick kernel
    hipGraph_t g = nullptr;
    hipError_t e = launch_serve(nullptr, nullptr, table_dt, mlp_dt, nhh, sb);  // kernel set-up, no launch
    if (e == hipSuccess) e = hipStreamBeginCapture(sb, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = hipMemcpyAsync(d_wt[buf], h_wt[buf], wt_bytes, hipMemcpyHostToDevice, sb);
    if (e == hipSuccess) e = launch_serve(d_slots, d_wt[buf], table_dt, mlp_dt, nhh, sb);
    const hipError_t e2 = hipStreamEndCapture(sb, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&graph[buf], g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) {
      if (gpu_err == hipSuccess) gpu_err = e;
      return false;
    }
  }
  hipError_t e = hipSuccess;
  if (copy_wait[buf]) {
    e = hipStreamWaitEvent(sb, copy_ev, 0);
    copy_wait[buf] = false;
  }
  if (e == hipSuccess) e = hipGraphLaunch(graph[buf], sb);
  if (e == hipSuccess) e = hipEventRecord(t.ev, sb);
  if (e != hipSuccess && gpu_err == hipSuccess) gpu_err = e;
  t.inflight = true;
  next_buf ^= 1;
  st.ticks++;
  st.tiles += n;
  return true;
}

void mnr_server::loop() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progress = retire_locked();
    progress |= admit_locked();
    progress |= launch_locked();
    const bool idle = queue.empty() && active.empty() && !ticks[0].inflight && !ticks[1].inflight;
    if (stop && idle) break;
    if (gpu_err != hipSuccess) {  // fail every pending request rather than hang
      for (auto& kv : reqs) kv.second.done = true;
      queue.clear();
      active.clear();
      cv_done.notify_all();
      if (stop) break;
    }
    if (!progress) {
      if (idle)
        cv_work.wait(lk);
      else
        cv_work.wait_for(lk, std::chrono::microseconds(50));  // poll in-flight ticks
    }
  }
}

extern "C" {

mnr_status mnr_server_create(uint64_t mem_budget, int32_t max_slots, int32_t tiles_per_tick, mnr_server** out) {
  clear_error();
  if (!out) return fail(MNR_E_INVALID, "server: null output");
  if (max_slots < 1 || max_slots > 256) return fail(MNR_E_SHAPE, "server: max_slots must be in [1, 256]");
  if (tiles_per_tick == 0) tiles_per_tick = 1024;
  if (tiles_per_tick < 16 || tiles_per_tick > 16384) return fail(MNR_E_SHAPE, "server: tiles_per_tick out of range");
  mnr_server* s = new mnr_server();
  s->budget = mem_budget;
  s->max_slots = max_slots;
  s->tick_cap = tiles_per_tick;
  for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->wt_bytes = sizeof(WorkTable) + sizeof(WorkItem) * (size_t)tiles_per_tick;
  hipError_t e = hipGetDevice(&s->device);
  for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipStreamCreateWithFlags(&s->stream[b], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->copy_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc((void**)&s->d_slots, sizeof(RenderArgs) * max_slots);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_slots, sizeof(RenderArgs) * max_slots, hipHostMallocDefault);
  for (int b = 0; b < 2 && e == hipSuccess; ++b) {
    e = hipMalloc((void**)&s->d_wt[b], s->wt_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_wt[b], s->wt_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ticks[b].ev, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    mnr_server_destroy(s);
    return fail(MNR_E_HIP, "server: %s", hipGetErrorString(e));
  }
  s->th = std::thread([s] { s->loop(); });
  *out = s;
  return MNR_OK;
}

mnr_status mnr_server_add_user(mnr_server* s, int32_t user, const mnr_field* field, const mnr_motion* motion) {
  clear_error();
  if (!s || !field || !motion || !motion->weights) return fail(MNR_E_INVALID, "server: null argument");
  if (motion->res_w[0]) return fail(MNR_E_UNSUPPORTED, "server: users with a residual motion network");
  if (field->encoding != MNR_ENC_GRID) return fail(MNR_E_UNSUPPORTED, "server: users with a frequency-encoded field");
  if (user < 0 || user > 1023) return fail(MNR_E_INVALID, "server: user id out of range");
  if (mnr_status st = validate_field(field)) return st;
  const uint64_t bytes = field_bytes(*field, *motion);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->users.count(user)) return fail(MNR_E_INVALID, "server: user %d already registered", user);
  if (s->have_format && (field->table_dtype != s->table_dt || field->mlp_dtype != s->mlp_dt ||
                         field->n_layers - 2 != s->nhh))
    return fail(MNR_E_DTYPE, "server: every user must share the field format");
  if (s->resident + bytes > s->budget)
    return fail(MNR_E_OOM, "server: user needs %llu bytes, %llu of %llu in use", (unsigned long long)bytes,
                (unsigned long long)s->resident, (unsigned long long)s->budget);
  s->users[user] = User{*field, *motion, bytes};
  s->resident += bytes;
  s->have_format = true;
  s->table_dt = field->table_dtype;
  s->mlp_dt = field->mlp_dtype;
  s->nhh = field->n_layers - 2;
  return MNR_OK;
}

mnr_status mnr_server_submit(mnr_server* s, int32_t user, const mnr_pose* pose, const mnr_camera* cam, int32_t H,
                             int32_t W, int32_t spp, const mnr_opts* opts, float* out_rgba, uint64_t* ticket) {
  clear_error();
  if (!s || !ticket) return fail(MNR_E_INVALID, "server: null argument");
  const int64_t arrive = now_ns();
  User u;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->users.find(user);
    if (it == s->users.end()) {
      s->st.rejected++;
      return fail(MNR_E_INVALID, "server: unknown user %d", user);
    }
    u = it->second;
  }
  if (mnr_status st = validate_common(&u.field, &u.motion, pose, cam, H, W, spp, opts, nullptr, H * W, out_rgba)) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.rejected++;
    return st;
  }
  Request r;
  pack_args(r.args, &u.field, &u.motion, pose, cam, H, W, spp, opts, nullptr, H * W);  // FK here
  r.args.out = out_rgba;
  r.user = user;
  r.n_tiles = slot_count(H, W, nullptr, H * W) / 256;
  r.out_bytes = (uint64_t)H * W * 16;
  r.t[0] = arrive;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->resident + r.out_bytes > s->budget) {
    s->st.rejected++;
    return fail(MNR_E_OOM, "server: a %dx%d frame does not fit the memory budget", H, W);
  }
  r.ticket = s->next_ticket++;
  *ticket = r.ticket;
  s->reqs.emplace(r.ticket, r);
  s->queue.push_back(r.ticket);
  s->st.submitted++;
  s->cv_work.notify_one();
  return MNR_OK;
}

mnr_status mnr_server_poll(mnr_server* s, uint64_t ticket, int32_t* done, int64_t* t_ns) {
  clear_error();
  if (!s || !done) return fail(MNR_E_INVALID, "server: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MNR_E_INVALID, "server: unknown ticket");
  if (s->gpu_err != hipSuccess) return fail(MNR_E_HIP, "server: %s", hipGetErrorString(s->gpu_err));
  *done = it->second.done ? 1 : 0;
  if (t_ns) std::memcpy(t_ns, it->second.t, sizeof(it->second.t));
  return MNR_OK;
}

mnr_status mnr_server_wait(mnr_server* s, uint64_t ticket, int32_t timeout_ms, int64_t* t_ns) {
  clear_error();
  if (!s) return fail(MNR_E_INVALID, "server: null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MNR_E_INVALID, "server: unknown ticket");
  const bool ok = s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms),
                                      [&] { return it->second.done || s->gpu_err != hipSuccess; });
  if (s->gpu_err != hipSuccess) return fail(MNR_E_HIP, "server: %s", hipGetErrorString(s->gpu_err));
  if (!ok) return fail(MNR_E_BUSY, "server: ticket not done after %d ms", timeout_ms);
  if (t_ns) std::memcpy(t_ns, it->second.t, sizeof(it->second.t));
  return MNR_OK;
}

mnr_status mnr_server_get_stats(mnr_server* s, mnr_server_stats* out) {
  clear_error();
  if (!s || !out) return fail(MNR_E_INVALID, "server: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->queued = (int32_t)s->queue.size();
  out->admitted = (int32_t)s->active.size();
  out->resident_bytes = s->resident;
  out->inflight_bytes = s->inflight_bytes;
  return MNR_OK;
}

mnr_status mnr_server_destroy(mnr_server* s) {
  clear_error();
  if (!s) return MNR_OK;
  if (s->th.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->th.join();
  }
  for (int b = 0; b < 2; ++b)
    if (s->stream[b]) hipStreamSynchronize(s->stream[b]);
  if (s->copy_stream) hipStreamSynchronize(s->copy_stream);
  for (int b = 0; b < 2; ++b) {
    if (s->graph[b]) hipGraphExecDestroy(s->graph[b]);
    if (s->ticks[b].ev) hipEventDestroy(s->ticks[b].ev);
    if (s->d_wt[b]) hipFree(s->d_wt[b]);
    if (s->h_wt[b]) hipHostFree(s->h_wt[b]);
  }
  if (s->d_slots) hipFree(s->d_slots);
  if (s->h_slots) hipHostFree(s->h_slots);
  if (s->copy_ev) hipEventDestroy(s->copy_ev);
  for (int b = 0; b < 2; ++b)
    if (s->stream[b]) hipStreamDestroy(s->stream[b]);
  if (s->copy_stream) hipStreamDestroy(s->copy_stream);
  delete s;
  return MNR_OK;
}

}  // extern "C"
