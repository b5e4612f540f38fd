/*
 * metanerf_server.h -- multi-user continuous-batching render server.
 *
 * The paper envisions many conference participants rendered by one
 * renderer (Sec. 3, Fig. 1: multi-user conferencing; real time needs about
 * 30 frames/s, Sec. 5.3).  A server keeps every user's canonical field and
 * blend-weight volume resident on the GPU and renders pose/camera requests
 * as they arrive:
 *   - admission: a queued request is admitted when a slot is free and the
 *     memory budget (resident users + outputs of admitted requests) allows;
 *   - continuous batching: each GPU tick renders 16x16-pixel tiles of the
 *     admitted requests up to a tile budget -- a quarter of it for the
 *     oldest unfinished request, the rest shortest-remaining-first -- so
 *     requests that arrive while a tick runs join the next one and small
 *     frames overtake large ones; large frames span several ticks;
 *   - one persistent kernel per tick pulls tiles from a device-side table;
 *     the per-tick work (table upload + kernel) is replayed from captured
 *     hipGraphs (two, double-buffered, so the host prepares tick k+1 while
 *     tick k runs), each on its own stream so that tick k+1 starts on the
 *     compute units that tick k's last blocks leave idle;
 *   - per-request timestamps (arrival, admission, first tick, completion)
 *     give p50/p99 latency.
 * A request's pixels are computed with a fixed ray-to-lane mapping and no
 * atomics, so its image is bitwise identical whether it is rendered alone
 * or in a mix; it is the same device code as mnr_render's full-frame path
 * (inlined into another kernel) and matches it to within 1e-6.
 *
 * All calls are thread-safe.  Device memory: the server allocates its
 * request slots and tile tables; users' fields and request outputs are
 * caller-owned and must stay valid while in use.  The server works on its
 * own streams.  A field must have no pending work on other streams when it
 * is registered.  An output buffer is ordered after the work queued on the
 * stream passed to mnr_server_submit (if any) at the time of the call; it
 * must stay allocated, and must not be read or reused, until poll or wait
 * has reported the request finished.
 * Request records live from submit until the poll or wait that reports
 * them finished, which releases them: a ticket is reported finished once.
 * After a GPU error every pending request finishes as failed (MNR_E_HIP);
 * kernels already running may still write their outputs, and the server
 * takes no new work.
 */
#ifndef METANERF_SERVER_H
#define METANERF_SERVER_H

#include "metanerf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mnr_server mnr_server;

typedef struct {
  uint64_t submitted, completed, rejected;
  uint64_t failed;                 /* finished without a frame (GPU error, budget) */
  uint64_t ticks, tiles;
  int32_t queued, admitted;        /* right now */
  int32_t tracked;                 /* request records not yet released */
  uint64_t resident_bytes;         /* registered users */
  uint64_t inflight_bytes;         /* outputs of admitted requests */
} mnr_server_stats;

/* mem_budget: bytes for resident users plus admitted outputs.  max_slots:
 * admitted requests at once (1..256).  tiles_per_tick: tile budget of one
 * GPU tick (16..16384; 0 = 1024).  Creates the server's streams and
 * scheduler thread on the current device. */
mnr_status mnr_server_create(uint64_t mem_budget, int32_t max_slots, int32_t tiles_per_tick, mnr_server** out);

/* Register user `user` (0..1023) with a resident field and blend-weight
 * volume (dev pointers, caller-owned).  Every user of a server must share
 * the field format: dtypes, layer count, encoding (grid or the
 * frequency-encoded field) and whether the residual motion network is on
 * (MNR_E_DTYPE otherwise; the residual network needs the BF16 MLP path,
 * MNR_E_UNSUPPORTED).  The first user fixes the format, and this call then
 * captures the server's two tick graphs on its streams (stream capture on
 * the calling thread: no thread may synchronise the whole device while it
 * runs).  MNR_E_OOM when the resident
 * bytes plus the outputs of queued and admitted requests would exceed the
 * budget (so that every queued request still fits once the ones ahead of
 * it finish); MNR_E_INVALID if the id is taken. */
mnr_status mnr_server_add_user(mnr_server* srv, int32_t user, const mnr_field* field, const mnr_motion* motion);

/* Queue a frame: pose and camera are read during the call (FK runs here);
 * out_rgba: dev float [H*W][4], written when the request completes.
 * after_stream (a hipStream_t, or NULL): the request's first tick waits for
 * the work queued on that stream at the time of this call (e.g. the last
 * reader of out_rgba).  MNR_E_OOM when the output alone exceeds the
 * budget, MNR_E_INVALID for a bad pose/camera or unknown user. */
mnr_status mnr_server_submit(mnr_server* srv, int32_t user, const mnr_pose* pose, const mnr_camera* cam,
                             int32_t H, int32_t W, int32_t spp, const mnr_opts* opts, float* out_rgba,
                             void* after_stream, uint64_t* ticket);

/* done = 1 once the request has finished (the frame is in out_rgba, or it
 * failed: then the call returns MNR_E_HIP after a GPU error, or MNR_E_OOM
 * for a request that can no longer fit the budget); reporting it releases
 * the ticket.  t_ns (optional, 4 entries): arrival, admission, first tick
 * launch, completion (steady clock, ns). */
mnr_status mnr_server_poll(mnr_server* srv, uint64_t ticket, int32_t* done, int64_t* t_ns);
/* Block until the ticket finishes (or timeout_ms elapses: MNR_E_BUSY), then
 * report it as poll does (and release it). */
mnr_status mnr_server_wait(mnr_server* srv, uint64_t ticket, int32_t timeout_ms, int64_t* t_ns);
mnr_status mnr_server_get_stats(mnr_server* srv, mnr_server_stats* stats);
/* Finish admitted and queued work, stop the scheduler, free device memory. */
mnr_status mnr_server_destroy(mnr_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* METANERF_SERVER_H */
