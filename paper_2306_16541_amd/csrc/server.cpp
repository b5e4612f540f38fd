// Multi-user continuous-batching render server (host side).  See
// include/metanerf_server.h for the contract.
//
// One scheduler thread owns the GPU side: it retires finished ticks,
// admits queued requests (free slot + memory budget), and launches the next
// tick whenever fewer than two are in flight.  A tick renders up to
// tiles_per_tick 16x16 tiles taken from admitted requests; a request
// completes with the tick that renders its last tile (request bookkeeping
// and tick composition: scheduler.h).  Ticks are replayed from two captured hipGraphs (tile-table
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
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/metanerf_server.h"
#include "host_common.h"
#include "kernels.h"
#include "scheduler.h"

namespace mnr {

static int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// What the scheduler carries per request: the kernel's arguments and an
// event on the caller's stream that the request's first tick waits on.
struct Payload {
  RenderArgs args;
  hipEvent_t ready = nullptr;
};
using Sched = Scheduler<Payload>;

struct User {
  mnr_field field;
  mnr_motion motion;
  uint64_t bytes;
};

static uint64_t field_bytes(const mnr_field& f, const mnr_motion& m) {
  const uint64_t el = f.table_dtype == MNR_F32 ? 4 : 2, wl = f.mlp_dtype == MNR_F32 ? 4 : 2;
  const bool freq = f.encoding == MNR_ENC_FREQ;
  uint64_t b = freq ? 0 : (uint64_t)f.n_levels * ((uint64_t)1 << f.log2_T) * f.n_feat * el;
  for (int k = 0; k < f.n_layers; ++k)  // the frequency field's W4 takes [h3; gamma]: 64 x 128
    b += (uint64_t)f.width[k] * f.width[k + 1] * (freq && k == 3 ? 2 : 1) * wl;
  if (m.res_w[0])  // residual network, BF16: W1..W5 and W_omega
    b += (uint64_t)(64 * 32 + 2 * 64 * 64 + 64 * 96 + 3 * 64 + 64 * 3 * m.n_bones) * 2;
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
  int tick_cap = 0;
  bool have_format = false;
  mnr_dtype table_dt = MNR_F32, mlp_dt = MNR_F32;
  int nhh = 0;
  bool res = false, freq = false;  // residual motion network; frequency-encoded field
  std::map<int, User> users;
  Sched* sched = nullptr;
  std::vector<TileRef> items;           // composition scratch of the next tick
  std::vector<Sched::Request*> starting;
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
  hipEvent_t tick_ev[2] = {nullptr, nullptr};
  int next_buf = 0;

  void loop();
  hipError_t prepare_ticks();
  void drop_ticks();
  bool retire_locked();
  bool admit_locked();
  bool launch_locked();
  void set_error(hipError_t e) {
    if (e != hipSuccess && gpu_err == hipSuccess) gpu_err = e;
  }
};

bool mnr_server::retire_locked() {
  bool any = false;
  for (int k = 0; k < 2; ++k) {
    const int buf = (next_buf + k) & 1;  // oldest first
    if (!sched->tick_busy(buf)) continue;
    const hipError_t q = hipEventQuery(tick_ev[buf]);
    if (q == hipErrorNotReady) break;
    set_error(q);
    sched->retire(buf, now_ns());
    any = true;
  }
  if (any) cv_done.notify_all();
  return any;
}

bool mnr_server::admit_locked() {
  const std::vector<Sched::Request*> adm = sched->admit(now_ns());
  for (Sched::Request* r : adm) {
    h_slots[r->slot] = r->payload.args;
    set_error(hipMemcpyAsync(d_slots + r->slot, h_slots + r->slot, sizeof(RenderArgs), hipMemcpyHostToDevice,
                             copy_stream));
  }
  if (!adm.empty()) {  // a slot is rewritten only after every tick that read it retired
    set_error(hipEventRecord(copy_ev, copy_stream));
    copy_wait[0] = copy_wait[1] = true;
  }
  return !adm.empty();
}

// The two tick graphs (tile-table upload + tick kernel, one per tick
// buffer) for the field format, captured when the first user fixes it, on
// the thread that registers that user: the scheduler thread then only
// replays them, and a stream capture never runs while other threads of the
// application synchronise their own work.
hipError_t mnr_server::prepare_ticks() {
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e == hipSuccess) e = hipSetDevice(device);
  for (int buf = 0; buf < 2 && e == hipSuccess; ++buf) {
    hipStream_t sb = stream[buf];
    hipGraph_t g = nullptr;
    e = launch_serve(nullptr, nullptr, table_dt, mlp_dt, nhh, res, freq, sb);  // kernel set-up, no launch
    if (e == hipSuccess) e = hipStreamBeginCapture(sb, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      e = hipMemcpyAsync(d_wt[buf], h_wt[buf], wt_bytes, hipMemcpyHostToDevice, sb);
      if (e == hipSuccess) e = launch_serve(d_slots, d_wt[buf], table_dt, mlp_dt, nhh, res, freq, sb);
      const hipError_t e2 = hipStreamEndCapture(sb, &g);
      if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&graph[buf], g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
  }
  if (e != hipSuccess) drop_ticks();
  (void)hipSetDevice(prev);
  return e;
}

void mnr_server::drop_ticks() {
  for (int buf = 0; buf < 2; ++buf)
    if (graph[buf]) {
      (void)hipGraphExecDestroy(graph[buf]);
      graph[buf] = nullptr;
    }
}

// Tick composition is the scheduler's (Scheduler::compose); this uploads
// the tile table and replays the buffer's captured graph.
bool mnr_server::launch_locked() {
  const int buf = next_buf;
  if (sched->tick_busy(buf)) return false;
  const int n = sched->compose(buf, now_ns(), items, starting);
  if (n == 0) return false;
  WorkTable* w = h_wt[buf];
  for (int k = 0; k < n; ++k) w->items[k] = WorkItem{items[k].slot, items[k].tile};
  w->counter = 0;
  w->n_items = n;
  hipStream_t sb = stream[buf];
  hipError_t e = graph[buf] ? hipSuccess : hipErrorNotReady;  // captured by the first add_user
  if (e == hipSuccess && copy_wait[buf]) {
    e = hipStreamWaitEvent(sb, copy_ev, 0);
    copy_wait[buf] = false;
  }
  for (Sched::Request* r : starting)  // work the caller queued on the output first
    if (e == hipSuccess && r->payload.ready) e = hipStreamWaitEvent(sb, r->payload.ready, 0);
  if (e == hipSuccess) e = hipGraphLaunch(graph[buf], sb);
  if (e == hipSuccess) e = hipEventRecord(tick_ev[buf], sb);
  set_error(e);
  next_buf ^= 1;
  return true;
}

void mnr_server::loop() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progress = false;
    if (gpu_err == hipSuccess) {
      progress = retire_locked();
      if (gpu_err == hipSuccess) progress |= admit_locked();
      if (gpu_err == hipSuccess) progress |= launch_locked();
    }
    if (gpu_err != hipSuccess && !sched->idle()) {  // fail every pending request rather than hang
      sched->fail_all(now_ns());
      cv_done.notify_all();
    }
    const bool idle = sched->idle();
    if (stop && idle) break;
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
  s->sched = new Sched(mem_budget, max_slots, tiles_per_tick);
  s->tick_cap = tiles_per_tick;
  s->items.reserve(tiles_per_tick);
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
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->tick_ev[b], hipEventDisableTiming);
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
  if (user < 0 || user > 1023) return fail(MNR_E_INVALID, "server: user id out of range");
  if (mnr_status st = validate_field(field)) return st;
  const uint64_t bytes = field_bytes(*field, *motion);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->users.count(user)) return fail(MNR_E_INVALID, "server: user %d already registered", user);
  const bool res = motion->res_w[0] != nullptr, freq = field->encoding == MNR_ENC_FREQ;
  if (res && field->mlp_dtype != MNR_BF16)
    return fail(MNR_E_UNSUPPORTED, "server: the residual motion network needs the BF16 MLP path");
  if (s->have_format && (field->table_dtype != s->table_dt || field->mlp_dtype != s->mlp_dt ||
                         field->n_layers - 2 != s->nhh || res != s->res || freq != s->freq))
    return fail(MNR_E_DTYPE, "server: every user must share the field format (dtypes, layers, encoding, residual network)");
  if (!s->sched->reserve_resident(bytes))
    return fail(MNR_E_OOM, "server: user needs %llu bytes; %llu resident and %llu queued or in flight of %llu",
                (unsigned long long)bytes, (unsigned long long)s->sched->resident_bytes(),
                (unsigned long long)(s->sched->inflight_bytes() + s->sched->queued_bytes()),
                (unsigned long long)s->sched->budget());
  if (!s->have_format) {  // the first user fixes the format: capture the tick graphs for it
    s->table_dt = field->table_dtype;
    s->mlp_dt = field->mlp_dtype;
    s->nhh = field->n_layers - 2;
    s->res = res;
    s->freq = freq;
    if (const hipError_t e = s->prepare_ticks()) {
      s->sched->release_resident(bytes);
      return fail(MNR_E_HIP, "server: preparing the tick kernel: %s", hipGetErrorString(e));
    }
    s->have_format = true;
  }
  s->users[user] = User{*field, *motion, bytes};
  return MNR_OK;
}

mnr_status mnr_server_submit(mnr_server* s, int32_t user, const mnr_pose* pose, const mnr_camera* cam, int32_t H,
                             int32_t W, int32_t spp, const mnr_opts* opts, float* out_rgba, void* after_stream,
                             uint64_t* ticket) {
  clear_error();
  if (!s || !ticket) return fail(MNR_E_INVALID, "server: null argument");
  const int64_t arrive = now_ns();
  User u;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->users.find(user);
    if (it == s->users.end()) {
      s->sched->count_rejected();
      return fail(MNR_E_INVALID, "server: unknown user %d", user);
    }
    u = it->second;
  }
  if (mnr_status st = validate_common(&u.field, &u.motion, pose, cam, H, W, spp, opts, nullptr, H * W, out_rgba)) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->sched->count_rejected();
    return st;
  }
  Payload p;
  pack_args(p.args, &u.field, &u.motion, pose, cam, H, W, spp, opts, nullptr, H * W);  // FK here
  p.args.out = out_rgba;
  if (after_stream) {  // the first tick of this request waits for what is queued there now
    hipError_t e = hipEventCreateWithFlags(&p.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(p.ready, (hipStream_t)after_stream);
    if (e != hipSuccess) {
      if (p.ready) hipEventDestroy(p.ready);
      return fail(MNR_E_HIP, "server: ordering event: %s", hipGetErrorString(e));
    }
  }
  const int n_tiles = slot_count(H, W, nullptr, H * W) / 256;
  const uint64_t out_bytes = (uint64_t)H * W * 16;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->gpu_err != hipSuccess) {
    if (p.ready) hipEventDestroy(p.ready);
    return fail(MNR_E_HIP, "server: %s", hipGetErrorString(s->gpu_err));
  }
  if (s->sched->submit(p, n_tiles, out_bytes, arrive, ticket) != Sched::SUBMIT_OK) {
    if (p.ready) hipEventDestroy(p.ready);
    return fail(MNR_E_OOM, "server: a %dx%d frame does not fit the memory budget", H, W);
  }
  s->cv_work.notify_one();
  return MNR_OK;
}

// A finished ticket is released (forgotten) by the poll or wait that
// reports it finished.
static mnr_status report_locked(mnr_server* s, uint64_t ticket, int32_t* done, int64_t* t_ns) {
  const Sched::Request* r = s->sched->find(ticket);
  if (!r) return fail(MNR_E_INVALID, "server: unknown ticket %llu", (unsigned long long)ticket);
  const hipEvent_t ready = r->payload.ready;
  const Sched::Poll p = s->sched->poll(ticket, t_ns, true);
  if (p == Sched::POLL_PENDING) {
    if (done) *done = 0;
    return MNR_OK;
  }
  if (ready) hipEventDestroy(ready);
  if (done) *done = 1;
  if (p == Sched::POLL_FAILED) {
    if (s->gpu_err != hipSuccess) return fail(MNR_E_HIP, "server: %s", hipGetErrorString(s->gpu_err));
    return fail(MNR_E_OOM, "server: request can no longer fit the memory budget");
  }
  return MNR_OK;
}

mnr_status mnr_server_poll(mnr_server* s, uint64_t ticket, int32_t* done, int64_t* t_ns) {
  clear_error();
  if (!s || !done) return fail(MNR_E_INVALID, "server: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  return report_locked(s, ticket, done, t_ns);
}

mnr_status mnr_server_wait(mnr_server* s, uint64_t ticket, int32_t timeout_ms, int64_t* t_ns) {
  clear_error();
  if (!s) return fail(MNR_E_INVALID, "server: null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->sched->find(ticket)) return fail(MNR_E_INVALID, "server: unknown ticket %llu", (unsigned long long)ticket);
  const bool ok = s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms), [&] {
    const Sched::Request* r = s->sched->find(ticket);
    return !r || r->done;
  });
  if (!ok) return fail(MNR_E_BUSY, "server: ticket not done after %d ms", timeout_ms);
  return report_locked(s, ticket, nullptr, t_ns);
}

mnr_status mnr_server_get_stats(mnr_server* s, mnr_server_stats* out) {
  clear_error();
  if (!s || !out) return fail(MNR_E_INVALID, "server: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  const Sched& q = *s->sched;
  *out = mnr_server_stats{};
  out->submitted = q.submitted();
  out->completed = q.completed();
  out->rejected = q.rejected();
  out->failed = q.failed();
  out->ticks = q.ticks();
  out->tiles = q.tiles();
  out->queued = q.queued();
  out->admitted = q.admitted();
  out->tracked = (int32_t)q.tracked();
  out->resident_bytes = q.resident_bytes();
  out->inflight_bytes = q.inflight_bytes();
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
  if (s->sched) {
    s->sched->for_each([](const Sched::Request& r) {
      if (r.payload.ready) hipEventDestroy(r.payload.ready);
    });
    delete s->sched;
  }
  for (int b = 0; b < 2; ++b) {
    if (s->graph[b]) hipGraphExecDestroy(s->graph[b]);
    if (s->tick_ev[b]) hipEventDestroy(s->tick_ev[b]);
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
