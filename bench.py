"""Benchmark of the posed-body renderer on one MI355X.

One step = one full render of the 512x512 seeded-body frame, 128 samples per
ray, FP32 path (inverse LBS over 24 bones with a 64^3 x 25 weight volume,
16-level grid with 2^19 entries per level, MLP 32-64-64-64-4), inputs
resident in HBM.  Printed as ONE JSON line:
  value      nominal Msamples/s (H*W*S per frame / frame time)
  roofline   the fused render kernel against the chip's peak (HIP-event
             timed launches, algorithmic bytes and FLOPs per evaluated sample)
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same frame
Extra fields: the same frame in mixed precision (FP16 table, BF16 MLP), the
1024x1024 / 192-sample mixed frame, the 8192-ray training step, and PSNR /
max-abs of each against the oracle on the sampled pixels.
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2306_16541_amd as m  # noqa: E402
import scenes  # noqa: E402

METRIC = "Msamples/s & 512² frames/s, BF16 vs FP32 at stated PSNR; serving p99 latency"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK = {"f32": 157.3, "bf16": 2500.0}     # dense TFLOP/s
BYTES_WARP = 24 * 8 * 4                        # per evaluated sample: 24 bones x 8 corners x fp32
BYTES_ENC = {"f32": 16 * 8 * 2 * 4, "f16": 16 * 8 * 2 * 2}   # 16 levels x 8 corners x 2 features


# The files that define the frame kernels (and the arguments they are
# launched with): a change to any of them invalidates the recorded counters.
FRAME_KERNEL_SOURCES = ("paper_2306_16541_amd/csrc/render.hip", "paper_2306_16541_amd/csrc/field_device.h",
                        "paper_2306_16541_amd/csrc/device_common.h", "paper_2306_16541_amd/csrc/kernels.h",
                        "paper_2306_16541_amd/csrc/api.cpp", "include/metanerf.h")


def sources_digest():
    """SHA-256 over the frame kernels' sources (identifies the build the
    counter-based traffic figures were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for rel in FRAME_KERNEL_SOURCES:
        h.update(rel.encode())
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()


def measured_traffic(key):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, scaled by the copy calibration; None if the kernel sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("sources_sha256") != sources_digest() or key not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][key]
    return (k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]) * 1024.0


def add_traffic_rate(roof, kernel_ms):
    """Beside the algorithmic rate (achieved / frac: every gather counted,
    L1 and L2 hits included), the rate of the measured traffic beyond the
    L2: traffic bytes per launch / kernel time, and its fraction of the HBM
    peak (when the counters match the current sources)."""
    if roof.get("traffic") and roof.get("bound") == "hbm":
        rate = roof["traffic"] / (kernel_ms * 1e-3) / 1e9
        roof["traffic_GB_per_s"] = rate
        roof["traffic_frac"] = rate / HBM_PEAK_GBS
    return roof


def mlp_flops(widths):
    return 2 * sum(a * b for a, b in zip(widths[:-1], widths[1:]))


def timed_launches(fn, steps, warmup):
    """Run fn warmup times, then `steps` times with a HIP event pair around each
    launch on the current stream.  Returns (wall ms/step, mean kernel ms)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ks = [a.elapsed_time(b) for a, b in evs]
    timed_launches.last_median = float(np.median(ks))
    return wall, float(np.mean(ks))


def psnr(a, b):
    mse = float(np.mean((a.astype(np.float64) - b) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)


def render_bench(sc, table_dt, mlp_dt, steps, warmup, residual=None):
    fld, _ = m.upload_scene(sc, "cuda", table_dt, mlp_dt)
    if residual is not None:
        fld.set_residual(*residual)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=1e-6)
    out = torch.empty(sc.H * sc.W, 4, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, out=out, counter=cnt)
    torch.cuda.synchronize()
    n_eval = int(cnt.item())
    wall, kern = timed_launches(lambda: m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, out=out), steps, warmup)
    img = out.cpu().numpy()
    return {"wall_ms": wall, "kernel_ms": kern, "kernel_ms_median": timed_launches.last_median, "n_eval": n_eval,
            "img": img}


def roofline(res, sc, enc_key, mlp_key, widths):
    """Both candidate bounds of the fused render kernel; the binding one
    (larger fraction of its peak) is reported."""
    k_s = res["kernel_ms"] * 1e-3
    gbytes = res["n_eval"] * (BYTES_WARP + BYTES_ENC[enc_key]) / 1e9
    tflop = res["n_eval"] * mlp_flops(widths) / 1e12
    hbm = {"bound": "hbm", "achieved": gbytes / k_s, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    mf = {"bound": "mfma", "achieved": tflop / k_s, "peak": MFMA_PEAK[mlp_key], "unit": "TFLOP/s"}
    for r in (hbm, mf):
        r["frac"] = r["achieved"] / r["peak"]
        r["traffic"] = None
    return (hbm, mf) if hbm["frac"] >= mf["frac"] else (mf, hbm)


def cpu_model() -> str:
    """The host CPU's model name, from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample(sc, img_fp32, img_mixed, budget_s):
    """FP64 oracle on a bounded random sample of the frame's pixels."""
    import oracle
    g = np.random.default_rng(0)
    order = g.permutation(sc.H * sc.W)
    done, refs, t0 = 0, [], time.perf_counter()
    chunk = 1024
    while time.perf_counter() - t0 < budget_s and done < order.size:
        pid = order[done:done + chunk]
        refs.append(oracle.render_image(sc, pixel_ids=pid).numpy())
        done += pid.size
    el = time.perf_counter() - t0
    pid = order[:done]
    ref = np.concatenate(refs)
    hit = ref[:, 3] > 0
    out = {"value": done * sc.spp / el / 1e6, "unit": "Msamples/s (nominal)", "cores": torch.get_num_threads(),
           "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": cpu_model(),
           "sample": f"{done} random pixels of the {sc.H}x{sc.W}x{sc.spp} frame ({done * sc.spp} nominal samples, "
                     f"{el:.1f} s, float64 torch CPU)"}
    par = {}
    for name, img in (("fp32", img_fp32), ("mixed", img_mixed)):
        if img is None:
            continue
        d = img[pid]
        par[name] = {"max_abs": float(np.abs(d - ref).max()), "psnr_all": psnr(d[:, :3], ref[:, :3]),
                     "psnr_hit": psnr(d[hit, :3], ref[hit, :3]), "pixels": int(done)}
    return out, par


def oracle_one_thread(sc, budget_s):
    """The same oracle restricted to one CPU thread, on a short sample."""
    import oracle
    n0 = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        order = np.random.default_rng(1).permutation(sc.H * sc.W)
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget_s and done < order.size:
            oracle.render_image(sc, pixel_ids=order[done:done + 256])
            done += 256
        el = time.perf_counter() - t0
    finally:
        torch.set_num_threads(n0)
    return {"value": done * sc.spp / el / 1e6, "unit": "Msamples/s (nominal)", "cores": 1,
            "sample": f"{done} random pixels, {el:.1f} s"}


def ceilings(reps=5):
    """Measured machine ceilings: random small gathers from tables of the
    grid's sizes (uniform, and within a 4 KiB window per wave as neighbouring
    rays do), scattered float atomics (alone, and 8 lanes per address) and
    dense MFMA loops, each the median of `reps` launches."""
    out = {}
    n_lanes, per_lane = 1 << 20, 64
    for rb, mib, name in ((4, 32, "fp16_table_rows"), (8, 64, "fp32_table_rows"), (16, 104, "packed_weight_cells")):
        table = torch.zeros((mib << 20) // 4, dtype=torch.float32, device="cuda")
        res = {}
        for win, key in ((0, "uniform"), (4096, "window_4KiB")):
            buf = torch.empty(n_lanes, dtype=torch.float32, device="cuda")
            timed_launches(lambda: m.probe_gather(table, rb, win, per_lane, n_lanes, out=buf), reps, 2)
            ms = timed_launches.last_median
            g = n_lanes * per_lane / (ms * 1e-3)
            res[key] = {"Ggathers_per_s": g / 1e9, "useful_GB_per_s": g * rb / 1e9}
        out[f"gather_{rb}B_{name}_{mib}MiB"] = res
        del table
    acc = torch.zeros(16 << 20, dtype=torch.float32, device="cuda")   # 64 MiB, the FP32 table's size
    for run in (1, 8):
        timed_launches(lambda: m.probe_atomic(acc, 128, 1 << 20, run), reps, 1)
        ms = timed_launches.last_median
        out[f"float_atomics_64MiB_run{run}"] = {"G_atomics_per_s": (1 << 20) * 128 / (ms * 1e-3) / 1e9}
    del acc
    # LDS operations (the adjoint's block sums): cycles per wave instruction per CU at 2.4 GHz
    lb, li = 512, 2000
    lbuf = torch.empty(lb * 1024, dtype=torch.float32, device="cuda")
    lds = {}
    for op, name in enumerate(m.PROBE_LDS_OPS):
        timed_launches(lambda: m.probe_lds(op, li, lb, out=lbuf), reps, 1)
        ms = timed_launches.last_median
        lane_ops = lb * 1024 * li
        lds[name] = {"G_lane_ops_per_s": lane_ops / (ms * 1e-3) / 1e9,
                     "cycles_per_wave_op_per_CU": ms * 1e-3 * 2.4e9 / (lane_ops / 64 / 256)}
    out["lds_ops"] = lds
    del lbuf
    n_blocks, iters = 2048, 4000
    buf = torch.empty(n_blocks * 256, dtype=torch.float32, device="cuda")
    for dt, name, flop in ((m.F32, "mfma_f32_16x16x4", 2048), (m.BF16, "mfma_bf16_16x16x32", 16384)):
        timed_launches(lambda: m.probe_mfma(dt, iters, n_blocks, out=buf), reps, 2)
        ms = timed_launches.last_median
        out[name] = {"TFLOP_per_s": n_blocks * 4 * iters * 4 * flop / (ms * 1e-3) / 1e12}
    return out


def mlp_unfused_bench(sc, n, fused_ms, reps=10):
    """The field MLP alone (mnr_probe_mlp: the renderer's MLP device code)
    over n stored feature rows, n = the frame's evaluated samples, against
    the MFMA peak of its type; `share` = its time / the fused frame kernel's."""
    out = {}
    widths = [32] + [w.shape[0] for w in sc.mlp]
    g = torch.Generator(device="cuda")
    g.manual_seed(16541)
    for dt, key, tname, row in ((m.F32, "f32", "fp32", 128), (m.BF16, "bf16", "mixed", 64)):
        fld, _ = m.upload_scene(sc, "cuda", m.F32, dt)
        feat = torch.rand(n, 32, generator=g, device="cuda").mul_(2.0).sub_(1.0)
        if dt == m.BF16:
            feat = feat.to(torch.bfloat16)
        o = torch.empty(n, 4, device="cuda")
        timed_launches(lambda: m.probe_mlp(fld, feat, out=o), reps, 2)
        ms = timed_launches.last_median
        tf = n * mlp_flops(widths) / (ms * 1e-3) / 1e12
        out[key] = {"samples": n, "kernel_ms_median": ms, "Gsamples_per_s": n / (ms * 1e-3) / 1e9,
                    "TFLOP_per_s": tf, "frac_of_mfma_peak": tf / MFMA_PEAK[key],
                    "GB_per_s": n * (row + 16) / (ms * 1e-3) / 1e9,
                    "share_of_fused_frame": ms / fused_ms[tname] if fused_ms.get(tname) else None}
        del feat, o, fld
    return out


def train_bench(steps, warmup):
    sc = scenes.scene_body()
    dev = "cuda"
    tr = m.Trainer(torch.as_tensor(sc.table, device=dev), [torch.as_tensor(w, device=dev) for w in sc.mlp],
                   torch.as_tensor(sc.logits, device=dev), sc.level_res, m.F32, m.BF16, max_rays=8192, spp=sc.spp)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    pid, tgt = scenes.train_batch(7, sc.H, sc.W, 8192)
    pid, tgt = torch.as_tensor(pid, device=dev), torch.as_tensor(tgt, device=dev)
    k = [0]

    def step():
        k[0] += 1
        tr.step(pose, cam, sc.H, sc.W, sc.spp, pid, tgt, seed=k[0])
    wall, _ = timed_launches(step, steps, warmup)
    res = {"ms_per_step": wall, "steps_per_s": 1e3 / wall, "rays": 8192, "spp": sc.spp,
           "Msamples_per_s": 8192 * sc.spp / wall / 1e3, "loss": tr.loss(),
           "dtype": "fp32 table/adam, bf16 MLP"}
    # Time split: the same kernels called one at a time (forward with saved
    # state, adjoint into zeroed gradients); the rest of a step is the loss,
    # softmax adjoint/forward, Adam and the gradient fills.
    opts = m.make_opts(stratified=True, seed=1)
    rgba, g_rgba = tr.buf["rgba"], tr.buf["grad_rgba"]
    tch = tr.buf["t_chunks"][: 8192 * m.saved_size(sc.spp)].view(8192, -1)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    m.render(tr.field, pose, cam, sc.H, sc.W, sc.spp, opts, pid, out=rgba, counter=cnt, t_chunks=tch)
    torch.cuda.synchronize()
    n_eval = int(cnt.item())
    _, fwd_ms = timed_launches(lambda: m.render(tr.field, pose, cam, sc.H, sc.W, sc.spp, opts, pid, out=rgba,
                                                t_chunks=tch), steps, 1)
    m.mse_loss(rgba, tgt, g_rgba)
    b = tr.buf

    def bwd(ws, gG=None):
        m.render_backward(tr.field, pose, cam, sc.H, sc.W, sc.spp, opts, pid, tch, g_rgba, b["table_grad"],
                          b["w_grad"], b["weights_grad"], grad_bones=gG, adjoint_ws=ws)
    for t in [b["table_grad"], b["weights_grad"]] + b["w_grad"]:
        t.zero_()
    # the adjoint as the training step runs it (table and blend-weight
    # gradients through the binned scatter), and with every gradient added by
    # global atomics
    _, bwd_ms = timed_launches(lambda: bwd(tr.adjoint_ws), steps, 1)
    torch.cuda.synchronize()
    n_records = int(tr.adjoint_ws[:4].view(torch.int32).item())  # the workspace's first word: records written
    _, bwd_atomic_ms = timed_launches(lambda: bwd(None), steps, 1)
    gG = torch.zeros(24, 3, 4, device=dev)
    _, bwd_pose_ms = timed_launches(lambda: bwd(tr.adjoint_ws, gG), steps, 1)
    res["adjoint_with_bone_grads_ms"] = bwd_pose_ms
    res["adjoint_atomic_scatter_ms"] = bwd_atomic_ms
    res["binned_scatter"] = tr.adjoint_ws is not None
    # skeleton-motion CNN (32^3 x 25 logits from the 256-d latent): forward and adjoint per step
    cnn = m.SkeletonCNN(*scenes.skel_cnn_weights(5))
    glog = torch.ones(25, 32, 32, 32, device=dev)
    _, cnn_f = timed_launches(lambda: cnn.forward(), steps, 1)
    _, cnn_b = timed_launches(lambda: cnn.backward(glog), steps, 1)
    res["skel_cnn_ms"] = {"forward": cnn_f, "adjoint": cnn_b}
    atomics = n_eval * (16 * 8 * 2 + 24 * 8)
    res["split_ms"] = {"forward": fwd_ms, "adjoint": bwd_ms, "rest": wall - fwd_ms - bwd_ms}
    res.update(train_variants(sc, pose, cam, pid, tgt, steps))
    res["binned_records"] = n_records
    res["evaluated_samples"] = n_eval
    res["adjoint_atomics_per_s_upper"] = atomics / (bwd_atomic_ms * 1e-3)
    return res


def train_variants(sc, pose, cam, pid, tgt, steps):
    """The same 8192-ray batch with the residual motion network on (grid
    field), with the paper's frequency-encoded field, with an FP32 MLP on the
    grid field, and with the renderer reading an FP16 copy of the table (FP32
    masters and Adam state): step time and the adjoint alone (through the
    adjoint workspace)."""
    dev = "cuda"
    out = {}
    rw, w_omega = scenes.residual_weights(21)
    trainers = {
        "residual_network": m.Trainer(torch.as_tensor(sc.table, device=dev),
                                      [torch.as_tensor(w, device=dev) for w in sc.mlp],
                                      torch.as_tensor(sc.logits, device=dev), sc.level_res, m.F32, m.BF16,
                                      max_rays=8192, spp=sc.spp, residual=(rw, w_omega, 4.0)),
        "frequency_field": m.Trainer.frequency([torch.as_tensor(w, device=dev) for w in scenes.freq_field_weights(31)],
                                               torch.as_tensor(sc.logits, device=dev), max_rays=8192, spp=sc.spp),
        "fp32_mlp": m.Trainer(torch.as_tensor(sc.table, device=dev), [torch.as_tensor(w, device=dev) for w in sc.mlp],
                              torch.as_tensor(sc.logits, device=dev), sc.level_res, m.F32, m.F32,
                              max_rays=8192, spp=sc.spp),
        "fp16_table": m.Trainer(torch.as_tensor(sc.table, device=dev), [torch.as_tensor(w, device=dev) for w in sc.mlp],
                                torch.as_tensor(sc.logits, device=dev), sc.level_res, m.F16, m.BF16,
                                max_rays=8192, spp=sc.spp),
    }
    opts = m.make_opts(stratified=True, seed=1)
    for name, tr in trainers.items():
        k = [0]

        def step():
            k[0] += 1
            tr.step(pose, cam, sc.H, sc.W, sc.spp, pid, tgt, seed=k[0])
        wall, _ = timed_launches(step, steps, 2)
        b = tr.buf
        tch = b["t_chunks"][: 8192 * m.saved_size(sc.spp)].view(8192, -1)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        m.render(tr.field, pose, cam, sc.H, sc.W, sc.spp, opts, pid, out=b["rgba"], counter=cnt, t_chunks=tch)
        m.mse_loss(b["rgba"], tgt, b["grad_rgba"])
        gres = b.get("res_grad")
        _, bwd_ms = timed_launches(
            lambda: m.render_backward(tr.field, pose, cam, sc.H, sc.W, sc.spp, opts, pid, tch, b["grad_rgba"],
                                      b.get("table_grad"), b["w_grad"], b["weights_grad"], adjoint_ws=tr.adjoint_ws,
                                      grad_res=gres), steps, 1)
        torch.cuda.synchronize()
        out[name] = {"ms_per_step": wall, "adjoint_ms": bwd_ms, "evaluated_samples": int(cnt.item()),
                     "loss": tr.loss()}
    return out


def serve_bench(user_counts=(1, 2, 4, 8), spp=128, rate_hz=30.0, warmup_s=1.0, window_s=(10.0, 10.0, 10.0, 10.0),
                tiles_per_tick=1024):
    """Poisson arrivals from U users at rate_hz each; resolutions uniform over
    {256^2, 512^2, 1024^2}; per-user fields resident (FP16 table, BF16 MLP);
    per-frame pose ~ N(0, 0.3).  Latency = completion - arrival."""
    import threading
    sizes = (256, 512, 1024)
    fields = []
    for u in range(max(user_counts)):
        sc = scenes.scene_body(H=512, W=512, spp=spp, seed=16541 + 5 + 1000 * u)
        fld, _ = m.upload_scene(sc, "cuda", m.F16, m.BF16)
        fields.append((sc, fld))
    pool = {n: [torch.empty(n * n, 4, device="cuda") for _ in range(48)] for n in sizes}
    results = []
    for U, window in zip(user_counts, window_s):
        srv = m.Server(mem_budget=8 << 30, max_slots=32, tiles_per_tick=tiles_per_tick)
        for u in range(U):
            srv.add_user(u, fields[u][1])
        g = np.random.default_rng(U)
        arrivals = []
        for u in range(U):
            t = g.exponential(1.0 / rate_hz)
            while t < warmup_s + window:
                arrivals.append((t, u))
                t += g.exponential(1.0 / rate_hz)
        arrivals.sort()
        reqs = []
        for k, (t, u) in enumerate(arrivals):
            n = sizes[g.integers(3)]
            sc = fields[u][0]
            pose = m.PoseHost(sc.parents, sc.rest_joints, scenes.pose(7 * k + u, 0.3))
            cam = m.make_camera(scenes.camera(n, n, yaw=float(g.uniform(0, 2 * np.pi))))
            reqs.append((t, u, n, pose, cam, pool[n][k % len(pool[n])]))
        tickets = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()

        def producer():
            for t, u, n, pose, cam, out in reqs:
                dt = t0 + t - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                tickets.append((t, n, srv.submit(u, pose, cam, n, n, spp, out)))
        th = threading.Thread(target=producer)
        th.start()
        th.join()
        lat = {n: [] for n in sizes}
        done_times = []
        for t, n, tk in tickets:
            ts = srv.wait(tk, 600000)
            if t >= warmup_s:
                lat[n].append((ts[3] - ts[0]) / 1e6)
                done_times.append(ts[3])
        st = srv.stats()
        srv.close()
        every = [v for n in sizes for v in lat[n]]
        span = (max(done_times) - min(done_times)) / 1e9 if len(done_times) > 1 else float("nan")
        q = lambda v, p: float(np.percentile(v, p)) if v else None
        results.append({"users": U, "offered_frames_per_s": U * rate_hz, "window_s": window,
                        "frames": len(every), "completed_frames_per_s": len(every) / span,
                        "p50_ms": q(every, 50), "p99_ms": q(every, 99),
                        "p50_ms_512": q(lat[512], 50), "p99_ms_512": q(lat[512], 99),
                        "p99_ms_256": q(lat[256], 99), "p99_ms_1024": q(lat[1024], 99),
                        "ticks": st["ticks"], "tiles": st["tiles"]})
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--quick", action="store_true", help="headline FP32 frame only (for profiling)")
    ap.add_argument("--ceilings-only", action="store_true", help="the machine-ceiling probes only")
    ap.add_argument("--mixed-only", action="store_true", help="the mixed-precision 512x512 frame only (profiling)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--train-only", action="store_true", help="the 8192-ray training step only (profiling)")
    ap.add_argument("--digest", action="store_true", help="print the kernel-source digest and exit")
    ap.add_argument("--serve-only", action="store_true", help="only the serving measurement")
    ap.add_argument("--copy-calib", action="store_true",
                    help="plain 1 GiB device-to-device copy, for scaling FETCH_SIZE/WRITE_SIZE counters")
    args = ap.parse_args()
    if args.digest:
        print(sources_digest())
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every ray is independent and the whole frame fits one MI355X; "
              "multi-GPU sharding is described in DESIGN.md but not run.", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_per_launch": src.numel() * 4, "launches": args.steps}))
        return
    if args.train_only:
        print(json.dumps({"train_step_8192x128": train_bench(args.steps, args.warmup)}))
        return
    if args.ceilings_only:
        print(json.dumps({"ceilings": ceilings()}))
        return
    if args.serve_only:
        print(json.dumps({"serving": serve_bench()}))
        return
    sc = scenes.scene_body()                              # 512x512, 128 spp
    if args.mixed_only:
        res = render_bench(sc, m.F16, m.BF16, args.steps, args.warmup)
        print(json.dumps({"mixed_512_kernel_ms": res["kernel_ms"], "evaluated_samples": res["n_eval"]}))
        return
    fp32 = render_bench(sc, m.F32, m.F32, args.steps, args.warmup)
    widths = [32] + [w.shape[0] for w in sc.mlp]
    roof, roof2 = roofline(fp32, sc, "f32", "f32", widths)
    roof["traffic"] = measured_traffic("render_fwd_fp32_512x512x128")
    add_traffic_rate(roof, fp32["kernel_ms"])
    nominal = sc.H * sc.W * sc.spp
    line = {
        "metric": METRIC,
        "value": nominal / (fp32["wall_ms"] * 1e-3) / 1e6,
        "unit": "Msamples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": fp32["wall_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "posed-body render 512x512, 128 samples/ray, fp32 (24 bones, 64^3x25 weights, "
                               "16-level grid 2^19/level, MLP 32-64-64-64-4, ~30% of rays opaque)",
                   "H": sc.H, "W": sc.W, "spp": sc.spp},
        "frames_per_s": 1e3 / fp32["wall_ms"],
        "kernel_ms": fp32["kernel_ms"],
        "kernel_ms_median": fp32["kernel_ms_median"],
        "evaluated_Msamples_per_s": fp32["n_eval"] / (fp32["kernel_ms"] * 1e-3) / 1e6,
        "evaluated_samples": fp32["n_eval"],
        "roofline": roof,
        "roofline_other_bound": roof2,
    }
    mixed = None
    if not args.quick:
        mixed = render_bench(sc, m.F16, m.BF16, args.steps, args.warmup)
        line["mixed_512"] = {
            "Msamples_per_s": nominal / (mixed["kernel_ms"] * 1e-3) / 1e6, "frames_per_s": 1e3 / mixed["kernel_ms"],
            "speedup_vs_fp32": fp32["kernel_ms"] / mixed["kernel_ms"], "dtype": "fp16 table, bf16 MLP (fp32 acc)",
            "roofline": add_traffic_rate(dict(roofline(mixed, sc, "f16", "bf16", widths)[0],
                                              traffic=measured_traffic("render_fwd_mixed_512x512x128")),
                                         mixed["kernel_ms"])}
        # Residual non-rigid motion network on (all four bands open).
        rb = render_bench(sc, m.F16, m.BF16, args.steps, args.warmup, residual=(*scenes.residual_weights(21), 4.0))
        res_flop = 2 * (64 * 32 + 2 * 64 * 64 + 64 * 96 + 3 * 64)
        k_s = rb["kernel_ms"] * 1e-3
        line["mixed_512_residual"] = {
            "Msamples_per_s": nominal / k_s / 1e6, "frames_per_s": 1e3 / rb["kernel_ms"],
            "cost_vs_mixed": rb["kernel_ms"] / mixed["kernel_ms"], "evaluated_samples": rb["n_eval"],
            "roofline_mfma": {"bound": "mfma", "achieved": rb["n_eval"] * (mlp_flops(widths) + res_flop) / k_s / 1e12,
                              "peak": MFMA_PEAK["bf16"], "unit": "TFLOP/s"}}
        line["mixed_512_residual"]["roofline_mfma"]["frac"] = (line["mixed_512_residual"]["roofline_mfma"]["achieved"]
                                                               / MFMA_PEAK["bf16"])
        # the same gathers as the mixed frame (warp + FP16 grid): its binding bound
        rb_gbs = rb["n_eval"] * (BYTES_WARP + BYTES_ENC["f16"]) / k_s / 1e9
        line["mixed_512_residual"]["roofline"] = {"bound": "hbm", "achieved": rb_gbs, "peak": HBM_PEAK_GBS,
                                                  "unit": "GB/s", "frac": rb_gbs / HBM_PEAK_GBS, "traffic": None}
        del rb
        # The paper's own field: 10-band positional encoding and the skip MLP (BF16), no grid.
        lg = torch.as_tensor(sc.logits, device="cuda")
        ffield = m.DeviceField.frequency([m.convert(torch.as_tensor(w, device="cuda"), m.BF16)
                                          for w in scenes.freq_field_weights(31)], m.softmax_fwd(lg))
        fpose, fcam = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle), m.make_camera(sc.cam)
        fout = torch.empty(sc.H * sc.W, 4, device="cuda")
        fcnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        m.render(ffield, fpose, fcam, sc.H, sc.W, sc.spp, m.make_opts(), out=fout, counter=fcnt)
        torch.cuda.synchronize()
        f_eval = int(fcnt.item())
        _, f_ms = timed_launches(lambda: m.render(ffield, fpose, fcam, sc.H, sc.W, sc.spp, m.make_opts(), out=fout),
                                 args.steps, args.warmup)
        f_flop = 2 * (64 * 64 * 3 + 64 * 128 + 4 * 64)
        line["freq_field_512"] = {
            "Msamples_per_s": nominal / (f_ms * 1e-3) / 1e6, "frames_per_s": 1e3 / f_ms, "evaluated_samples": f_eval,
            "roofline_mfma": {"bound": "mfma", "achieved": f_eval * f_flop / (f_ms * 1e-3) / 1e12,
                              "peak": MFMA_PEAK["bf16"], "unit": "TFLOP/s"}}
        line["freq_field_512"]["roofline_mfma"]["frac"] = line["freq_field_512"]["roofline_mfma"]["achieved"] / \
            MFMA_PEAK["bf16"]
        # no grid: the warp's gathers are the only table traffic, and they bind
        f_gbs = f_eval * BYTES_WARP / (f_ms * 1e-3) / 1e9
        line["freq_field_512"]["roofline"] = {"bound": "hbm", "achieved": f_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                              "frac": f_gbs / HBM_PEAK_GBS, "traffic": None}
        del ffield
        line["mlp_unfused"] = mlp_unfused_bench(sc, fp32["n_eval"],
                                                {"fp32": fp32["kernel_ms_median"], "mixed": mixed["kernel_ms_median"]})
        sc3 = scenes.scene_body(H=1024, W=1024, spp=192)
        big = render_bench(sc3, m.F16, m.BF16, max(3, args.steps // 4), 1)
        big32 = render_bench(sc3, m.F32, m.F32, max(3, args.steps // 4), 1)
        for key, r in (("mixed_1024_192spp", big), ("fp32_1024_192spp", big32)):
            line[key] = {
                "Msamples_per_s": 1024 * 1024 * 192 / (r["kernel_ms"] * 1e-3) / 1e6,
                "frames_per_s": 1e3 / r["kernel_ms"],
                "evaluated_Msamples_per_s": r["n_eval"] / (r["kernel_ms"] * 1e-3) / 1e6}
        line["mixed_1024_192spp"]["speedup_vs_fp32"] = big32["kernel_ms"] / big["kernel_ms"]
        del big, big32
        line["train_step_8192x128"] = train_bench(max(3, args.steps // 2), 2)
        line["ceilings"] = ceilings()
        if not args.no_serve:
            line["serving"] = serve_bench()
    cpu, par = oracle_sample(sc, fp32["img"], None if mixed is None else mixed["img"], args.cpu_budget)
    line["cpu_baseline"] = cpu
    if not args.quick:
        line["cpu_baseline_1thread"] = oracle_one_thread(sc, min(5.0, args.cpu_budget))
    line["parity_vs_oracle"] = par
    print(json.dumps(line))


if __name__ == "__main__":
    main()
