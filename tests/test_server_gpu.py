"""Render server on the GPU: continuous batching of mixed-resolution,
multi-user requests; a request's image is bitwise identical alone and in
the mix (same tick kernel, fixed ray-to-lane mapping, no atomics) and
matches mnr_render within 1e-6 (same device code inlined into another
kernel may contract floating-point operations differently); memory
admission; rejection of invalid requests."""
import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu


def _user(seed, table_dt=1, mlp_dt=2):
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=64, W=64, spp=64, res=32, log2_T=16, seed=seed)
    fld, _ = m.upload_scene(sc, "cuda", table_dt, mlp_dt)
    return sc, fld


def _req(sc, seed, H, W):
    import paper_2306_16541_amd as m
    aa = scenes.pose(seed, 0.3)
    return m.PoseHost(sc.parents, sc.rest_joints, aa), m.make_camera(scenes.camera(H, W, yaw=0.3 * seed)), H, W


def test_alone_equals_mix_equals_render():
    import paper_2306_16541_amd as m
    users = [_user(16541 + 50 + u) for u in range(3)]
    srv = m.Server(mem_budget=4 << 30, max_slots=8, tiles_per_tick=64)   # small ticks: frames span ticks
    for u, (_, fld) in enumerate(users):
        srv.add_user(u, fld)
    spp = 64
    sc0, fld0 = users[0]
    pose, cam, H, W = _req(sc0, 1, 160, 128)
    alone = torch.full((H * W, 4), -1.0, device="cuda")
    # The server renders on its own stream: buffers handed to it must have no
    # pending work on torch's stream, and torch must not recycle memory the
    # server may still write (synchronise before submitting).
    torch.cuda.synchronize()
    srv.wait(srv.submit(0, pose, cam, H, W, spp, alone))
    ref = m.render(fld0, pose, cam, H, W, spp, m.make_opts()).clone()
    torch.cuda.synchronize()
    # the same request inside a mix of other users and sizes, several ticks deep
    outs, tickets = [], []
    sizes = [(64, 64), (256, 192), (96, 96), (32, 200), (128, 128)]
    for k, (h, w) in enumerate(sizes):
        u = (k + 1) % 3
        p, c, hh, ww = _req(users[u][0], 10 + k, h, w)
        o = torch.zeros(hh * ww, 4, device="cuda")
        torch.cuda.synchronize()
        tickets.append(srv.submit(u, p, c, hh, ww, spp, o))
        outs.append((u, p, c, hh, ww, o))
        if k == 2:
            mixed = torch.full((H * W, 4), -2.0, device="cuda")
            torch.cuda.synchronize()
            t_mix = srv.submit(0, pose, cam, H, W, spp, mixed)
    srv.wait(t_mix)
    for t in tickets:
        srv.wait(t)
    torch.cuda.synchronize()
    assert torch.equal(mixed, alone)
    diff = (alone - ref).abs().amax(1)
    d = float(diff.max())
    bad = torch.nonzero(diff > 1e-6)[:5, 0].tolist()
    print(f"server vs mnr_render max-abs {d:.3e}; first differing pixels {bad}: "
          f"server {alone[bad].tolist()} render {ref[bad].tolist()}")
    assert d <= 1e-6
    # the request from the mix against the FP64 oracle on the FP32 master
    # parameters (FP16 table, BF16 MLP on the GPU): PSNR >= 45 dB on a
    # sample of its pixels
    import dataclasses
    from helpers import oracle_render, psnr
    sc_req = dataclasses.replace(sc0, H=H, W=W, spp=spp)
    pid = np.arange(0, H * W, 7)
    want = oracle_render(sc_req, pixel_ids=pid, axis_angle=scenes.pose(1, 0.3), cam=scenes.camera(H, W, yaw=0.3))
    got = mixed.cpu().numpy()[pid]
    q = psnr(got[:, :3], want[:, :3])
    print(f"server request in the mix vs oracle: PSNR {q:.1f} dB, max-abs {np.abs(got - want).max():.2e} "
          f"({pid.size} pixels, opacity > 0.5 on {(want[:, 3] > 0.5).mean():.0%})", flush=True)
    assert q >= 45.0
    for u, p, c, hh, ww, o in outs:     # every mixed request matches its own plain render
        r = m.render(users[u][1], p, c, hh, ww, spp, m.make_opts())
        assert float((o - r).abs().max()) <= 1e-6
    st = srv.stats()
    print("server stats", st)
    assert st["completed"] == 7 and st["ticks"] >= 7
    srv.close()


def test_memory_admission_and_rejections():
    import math
    import paper_2306_16541_amd as m
    sc, fld = _user(16541 + 60)
    dense = sum((n + 1) * n * n * 16 for n in sc.level_res if (n + 1) ** 3 <= 1 << 16)
    resident = (16 * (1 << 16) * 2 * 2 + sum(w.size for w in sc.mlp) * 2 + 25 * 32 ** 3 * 4
                + 24 * 32 * 33 * 33 * 16 + dense)   # + the packed copies of the bone channels and dense levels
    frame = 64 * 64 * 16
    srv = m.Server(mem_budget=resident + frame + 100, max_slots=4)      # room for one 64x64 output
    srv.add_user(0, fld)
    with pytest.raises(m.MnrError, match="already"):
        srv.add_user(0, fld)
    _, fld2 = _user(16541 + 61)
    with pytest.raises(m.MnrError, match="over memory budget"):
        srv.add_user(1, fld2)
    pose, cam, H, W = _req(sc, 3, 64, 64)
    big = torch.zeros(128 * 128, 4, device="cuda")
    with pytest.raises(m.MnrError, match="over memory budget"):
        srv.submit(0, *_req(sc, 3, 128, 128)[:2], 128, 128, 64, big)
    bad = sc.axis_angle.copy(); bad[5, 0] = math.nan
    with pytest.raises(m.MnrError, match="invalid"):
        srv.submit(0, m.PoseHost(sc.parents, sc.rest_joints, bad), cam, H, W, 64, big)
    with pytest.raises(m.MnrError, match="invalid"):
        srv.submit(7, pose, cam, H, W, 64, big)
    outs = [torch.zeros(H * W, 4, device="cuda") for _ in range(5)]
    torch.cuda.synchronize()
    tickets = [srv.submit(0, pose, cam, H, W, 64, o) for o in outs]
    ts = [srv.wait(t) for t in tickets]
    # only one output fits: each request is admitted after the previous one completed
    for a, b in zip(ts[:-1], ts[1:]):
        assert b[1] >= a[3]
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    st = srv.stats()
    assert st["rejected"] >= 3 and st["completed"] == 5
    srv.close()


@pytest.mark.parametrize("kind", ["frequency", "residual"])
def test_frequency_and_residual_users(kind):
    # Users of the paper's own field (Sec. 4.4) or with the residual motion
    # network (Sec. 4.3, conditioned on each request's pose): two users,
    # requests interleaved over several ticks; each image equals the same
    # request alone (bitwise) and mnr_render within 1e-6, and the first is
    # within 45 dB of the FP64 oracle.
    import dataclasses
    import paper_2306_16541_amd as m
    from helpers import oracle_render, psnr
    users = []
    for u in range(2):
        sc = scenes.scene_body(H=64, W=64, spp=64, res=32, log2_T=16, seed=16541 + 70 + u)
        if kind == "frequency":
            ws = scenes.freq_field_weights(40 + u)
            fld = m.DeviceField.frequency([m.convert(torch.as_tensor(w, device="cuda"), m.BF16) for w in ws],
                                          m.softmax_fwd(torch.as_tensor(sc.logits, device="cuda")))
            extra = {"freq": ws}
        else:
            fld, _ = m.upload_scene(sc, "cuda", 1, 2)
            rw, w_omega = scenes.residual_weights(45 + u)
            fld.set_residual(rw, w_omega, 4.0)
            extra = {"residual": (rw, w_omega)}
        users.append((sc, fld, extra))
    srv = m.Server(mem_budget=4 << 30, max_slots=8, tiles_per_tick=64)
    for u, (_, fld, _) in enumerate(users):
        srv.add_user(u, fld)
    spp = 64
    reqs = []
    for k, (h, w) in enumerate([(96, 80), (64, 64), (128, 96), (48, 112)]):
        u = k % 2
        p, c, hh, ww = _req(users[u][0], 20 + k, h, w)
        o = torch.zeros(hh * ww, 4, device="cuda")
        torch.cuda.synchronize()
        reqs.append((u, k, p, c, hh, ww, o, srv.submit(u, p, c, hh, ww, spp, o)))
    for r in reqs:
        srv.wait(r[-1])
    torch.cuda.synchronize()
    for u, k, p, c, hh, ww, o, _ in reqs:
        alone = torch.zeros(hh * ww, 4, device="cuda")
        torch.cuda.synchronize()
        srv.wait(srv.submit(u, p, c, hh, ww, spp, alone))
        torch.cuda.synchronize()
        assert torch.equal(alone, o), (kind, k)
        ref = m.render(users[u][1], p, c, hh, ww, spp, m.make_opts())
        torch.cuda.synchronize()
        assert float((o - ref).abs().max()) <= 1e-6, (kind, k)
    # the first request against the oracle
    u, k, p, c, hh, ww, o, _ = reqs[0]
    sc, _, extra = users[u]
    sc_req = dataclasses.replace(sc, H=hh, W=ww, spp=spp)
    pid = np.arange(0, hh * ww, 5)
    want = oracle_render(sc_req, pixel_ids=pid, axis_angle=scenes.pose(20 + k, 0.3),
                         cam=scenes.camera(hh, ww, yaw=0.3 * (20 + k)), **extra)
    got = o.cpu().numpy()[pid]
    q = psnr(got[:, :3], want[:, :3])
    print(f"[server, {kind} users] request vs oracle: PSNR {q:.1f} dB", flush=True)
    assert q >= 45.0
    srv.close()


def test_users_must_share_the_field_format():
    import paper_2306_16541_amd as m
    sc, fld = _user(16541 + 80)
    sc2 = scenes.scene_body(H=64, W=64, spp=64, res=32, log2_T=16, seed=16541 + 81)
    freq = m.DeviceField.frequency([m.convert(torch.as_tensor(w, device="cuda"), m.BF16)
                                    for w in scenes.freq_field_weights(46)],
                                   m.softmax_fwd(torch.as_tensor(sc2.logits, device="cuda")))
    srv = m.Server(mem_budget=4 << 30, max_slots=8, tiles_per_tick=64)
    srv.add_user(0, fld)
    with pytest.raises(m.MnrError, match="format"):
        srv.add_user(1, freq)
    srv.close()
