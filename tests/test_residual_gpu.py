"""GPU parity of the residual non-rigid motion network (Sec. 4.3, Eq. 11-12)
against the FP64 oracle.

The network runs on BF16 MFMA with FP32 accumulation (the mixed-precision
path), so the bar is the mixed path's: PSNR >= 45 dB against the oracle
evaluated on the FP32 master weights.  A zero output layer must leave the
render bitwise unchanged, and the residual must visibly move the image.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from helpers import psnr

pytestmark = pytest.mark.gpu


def _render(sc, tdt, mdt, res=None, pixel_ids=None, alpha=4.0):
    import paper_2306_16541_amd as m
    fld, _ = m.upload_scene(sc, "cuda", tdt, mdt)
    if res is not None:
        fld.set_residual(res[0], res[1], alpha)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    pid = None if pixel_ids is None else torch.as_tensor(np.asarray(pixel_ids, np.int32), device="cuda")
    out = m.render(fld, pose, m.make_camera(sc.cam), sc.H, sc.W, sc.spp, m.make_opts(), pid)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _oracle(sc, res, pixel_ids=None, alpha=4.0):
    return oracle.render_image(sc, pixel_ids=pixel_ids,
                               residual={"weights": res[0], "w_omega": res[1], "alpha": alpha}).numpy()


@pytest.mark.parametrize("tdt,alpha", [(1, 4.0), (0, 2.5), (1, 0.0)])
def test_residual_render_matches_oracle(tdt, alpha):
    sc = scenes.scene_body(H=48, W=64, spp=128)
    res = scenes.residual_weights(21)
    g = _render(sc, tdt, 2, res, alpha=alpha)
    o = _oracle(sc, res, alpha=alpha)
    plain = oracle.render_image(sc).numpy()
    moved = float(np.abs(o - plain).max())
    p = psnr(g[:, :3], o[:, :3])
    print(f"[residual tdt={tdt} alpha={alpha}] PSNR {p:.2f} dB, max-abs {np.abs(g - o).max():.3e}, "
          f"oracle moved by the residual {moved:.3e}", flush=True)
    assert moved > 1e-2
    assert p >= 45.0


def test_residual_ray_list_matches_oracle():
    sc = scenes.scene_body(H=40, W=56, spp=96)
    res = scenes.residual_weights(22)
    pid = np.random.default_rng(4).integers(0, sc.H * sc.W, 500)
    g = _render(sc, 1, 2, res, pixel_ids=pid)
    o = _oracle(sc, res, pixel_ids=pid)
    assert psnr(g[:, :3], o[:, :3]) >= 45.0


def test_zero_output_layer_is_bitwise_plain():
    sc = scenes.scene_body(H=32, W=48, spp=128)
    ws, w_omega = scenes.residual_weights(23)
    ws[4] = np.zeros_like(ws[4])
    a = _render(sc, 1, 2, (ws, w_omega))
    b = _render(sc, 1, 2, None)
    assert np.array_equal(a, b)


def test_residual_on_a_refined_pose_matches_oracle():
    # Eq. 11 conditions the residual network on the observed pose theta^o:
    # with a refiner adjustment its joint angles are those of
    # R(Delta_j) R(omega_j), the rotations the bone transforms use.  The
    # oracle conditioned on the unrefined angles instead must differ
    # visibly, so the test sees which angles the GPU used.
    import paper_2306_16541_amd as m
    from oracle import pose as OP
    from oracle import render as O
    sc = scenes.scene_body(H=40, W=48, spp=96)
    res = scenes.residual_weights(25)
    delta = np.random.default_rng(11).normal(0.0, 0.3, (24, 3)).astype(np.float32)
    fld, _ = m.upload_scene(sc, "cuda", 1, 2)
    fld.set_residual(res[0], res[1], 4.0)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle, delta)
    got = m.render(fld, pose, m.make_camera(sc.cam), sc.H, sc.W, sc.spp, m.make_opts()).cpu().numpy()
    G = OP.refined_bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle, delta)
    o, d = O.camera_rays(sc.cam, sc.H, sc.W, np.arange(sc.H * sc.W))
    field = O.Field.from_scene(sc)

    def orc(omega):
        r = {"weights": res[0], "w_omega": res[1], "alpha": 4.0, "omega": omega}
        return O.render_rays(field, G, o, d, sc.spp, residual=r).numpy()
    want = orc(OP.observed_angles(sc.axis_angle, delta))
    stale = orc(sc.axis_angle)
    p, p_stale = psnr(got[:, :3], want[:, :3]), psnr(got[:, :3], stale[:, :3])
    moved = float(np.abs(want - stale).max())
    print(f"[residual, refined pose] PSNR {p:.2f} dB vs oracle; {p_stale:.2f} dB vs the oracle on the unrefined "
          f"angles (which moves pixels by {moved:.3e})", flush=True)
    assert moved > 1e-2
    assert p >= 45.0 and p > p_stale + 10.0


def test_residual_needs_the_bf16_path():
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=16, W=16, spp=32)
    with pytest.raises(m.MnrError, match="BF16"):
        _render(sc, 0, 0, scenes.residual_weights(24))


# ---------------------------------------------------------------- adjoint --
#
# The residual network trains (Sec. 4.3, Sec. 5.2): its split adjoint
# against the FP64 oracle's autograd, for every learnable tensor, and a
# training run that fits a residual motion.  Tolerances are the BF16 path's
# (the residual network, hence the field's MLP, run in BF16 with FP32
# accumulation): relative L2 5e-2 per group, every entry within 1e-1 of the
# group's largest (8-bit mantissas in every product of two MLPs, forward and
# back).

def _res_grads_gpu(sc, res, pid, tgt, alpha, seed=77, delta=None):
    import paper_2306_16541_amd as m
    fld, _ = m.upload_scene(sc, "cuda", m.F32, m.BF16)
    fld.set_residual(res[0], res[1], alpha)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle, delta)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=0.0, stratified=True, seed=seed)
    n = len(pid)
    pid_t = torch.as_tensor(pid, device="cuda")
    tch = torch.zeros(n, m.saved_size(sc.spp), device="cuda")
    rgba = m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, t_chunks=tch)
    grad_rgba = torch.empty(n, 4, device="cuda")
    loss = torch.zeros(1, device="cuda")
    m.mse_loss(rgba, torch.as_tensor(tgt, device="cuda"), grad_rgba, loss)
    g_table = torch.zeros(sc.table.shape, device="cuda")
    g_w = [torch.zeros(w.shape, device="cuda") for w in sc.mlp]
    g_wc = torch.zeros(sc.logits.shape, device="cuda")
    g_res = [torch.zeros(w.shape, device="cuda") for w in list(res[0]) + [res[1]]]
    gG = torch.zeros(24, 3, 4, device="cuda")
    ws = m.adjoint_workspace(fld, n, sc.spp)
    m.render_backward(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, tch, grad_rgba, g_table, g_w, g_wc,
                      grad_bones=gG, adjoint_ws=ws, grad_res=g_res)
    g_logits = torch.zeros_like(g_wc)
    m.softmax_bwd(fld.weights, g_wc, g_logits)
    torch.cuda.synchronize()
    return (float(loss.item()), [g_table.cpu().numpy(), g_logits.cpu().numpy()] + [w.cpu().numpy() for w in g_w] +
            [w.cpu().numpy() for w in g_res], gG.cpu().numpy())


def _res_grads_oracle(sc, res, pid, tgt, alpha, seed=77, delta=None):
    from oracle import pose as OP
    from oracle import render as O
    from oracle.rng import stratified_xi
    field = O.Field.from_scene(sc, requires_grad=True)
    rw = [torch.tensor(np.asarray(w, np.float64), requires_grad=True) for w in res[0]]
    wo = torch.tensor(np.asarray(res[1], np.float64), requires_grad=True)
    if delta is None:
        G, omega = O.bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle), sc.axis_angle
    else:
        G = OP.refined_bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle, delta)
        omega = OP.observed_angles(sc.axis_angle, delta)
    G = G.detach().requires_grad_(True)
    o, d = O.camera_rays(sc.cam, sc.H, sc.W, pid)
    rgba = O.render_rays(field, G, o, d, sc.spp, xi=stratified_xi(seed, len(pid), sc.spp),
                         residual={"weights": rw, "w_omega": wo, "alpha": alpha, "omega": omega})
    loss = O.mse_loss(rgba, tgt)
    loss.backward()
    return (float(loss.detach()), [field.table.grad.numpy(), field.logits.grad.numpy()] +
            [w.grad.numpy() for w in field.mlp] + [w.grad.numpy() for w in rw] + [wo.grad.numpy()],
            G.grad.numpy())


def test_split_adjoint_with_a_zero_output_layer_equals_the_fused_adjoint():
    # With W5 = 0 the residual offset is exactly zero, so the forward pass is
    # the plain one and the split adjoint (residual forward, field adjoint,
    # residual adjoint, skinning adjoint) must give the fused adjoint's
    # gradients for the field, the blend weights and the bone transforms, up
    # to the order of float additions.  The residual network's own gradients
    # are then dL/dW5 = sum over samples of dL/dx_res h4^T and zero for
    # W1..W4 and W_omega (nothing flows back through W5 = 0).
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=32, W=32, spp=128, res=32, log2_T=16, seed=16541 + 4)
    ws, w_omega = scenes.residual_weights(33)
    ws[4] = np.zeros_like(ws[4])
    g = np.random.default_rng(7)
    pid = g.integers(0, sc.H * sc.W, 64).astype(np.int32)
    tgt = g.random((64, 3)).astype(np.float32)
    _, split, gG_split = _res_grads_gpu(sc, (ws, w_omega), pid, tgt, 4.0)
    # the fused adjoint, same forward (no residual network at all)
    fld, _ = m.upload_scene(sc, "cuda", m.F32, m.BF16)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=0.0, stratified=True, seed=77)
    pid_t = torch.as_tensor(pid, device="cuda")
    tch = torch.zeros(64, m.saved_size(sc.spp), device="cuda")
    rgba = m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, t_chunks=tch)
    grad_rgba = torch.empty(64, 4, device="cuda")
    m.mse_loss(rgba, torch.as_tensor(tgt, device="cuda"), grad_rgba)
    g_table = torch.zeros(sc.table.shape, device="cuda")
    g_w = [torch.zeros(w.shape, device="cuda") for w in sc.mlp]
    g_wc = torch.zeros(sc.logits.shape, device="cuda")
    gG = torch.zeros(24, 3, 4, device="cuda")
    m.render_backward(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, tch, grad_rgba, g_table, g_w, g_wc,
                      grad_bones=gG)
    g_logits = torch.zeros_like(g_wc)
    m.softmax_bwd(fld.weights, g_wc, g_logits)
    torch.cuda.synchronize()
    fused = [g_table.cpu().numpy(), g_logits.cpu().numpy()] + [w.cpu().numpy() for w in g_w]
    names = ["table", "logits"] + [f"w{k}" for k in range(len(sc.mlp))]
    for name, a, b in zip(names, split[:len(fused)], fused):
        err = float(np.abs(a - b).max() / np.abs(b).max())
        print(f"  split vs fused {name:7s} max diff {err:.2e} of max", flush=True)
        assert err <= 1e-5, name
    err = float(np.abs(gG_split - gG.cpu().numpy()).max() / np.abs(gG.cpu().numpy()).max())
    print(f"  split vs fused dL/dG   max diff {err:.2e} of max", flush=True)
    assert err <= 1e-5
    res_g = split[len(fused):]
    for k in (0, 1, 2, 3, 5):
        assert not res_g[k].any(), k
    assert np.abs(res_g[4]).max() > 0


COARSE_RES = np.array([4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 18, 20, 24], np.int32)


def _coarse_body(sigma=20.0):
    """The body scene on a grid whose finest cell is 1/24 of the box (every
    level dense), with its density seeded on all 16 levels."""
    seed = 16541 + 4
    sc = scenes.scene_body(H=32, W=32, spp=128, res=32, log2_T=16, seed=seed)
    sc.level_res = COARSE_RES
    sc.table = scenes.grid_table(seed, 16)
    nd = scenes.seed_density(sc.table, 16, level_res=COARSE_RES, thickness=scenes.BODY_THICKNESS)
    sc.mlp = scenes.mlp_weights(seed, (32, 64, 64, 64, 4))
    scenes.density_mlp(sc.mlp, nd, sigma / nd)
    return sc


def _bf16(a):
    return torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).float().numpy()


@pytest.mark.parametrize("alpha,refined", [(4.0, False), (1.5, False), (4.0, True)])
def test_residual_adjoint_matches_oracle_gradient(alpha, refined):
    # On the fine hashed levels (cells of 1/512) the gradients with respect
    # to the residual network are ill-conditioned: a BF16-sized change of the
    # offset x_res (~1e-4) moves samples across cell faces, where the
    # encoding's spatial derivative jumps, and in the FP64 oracle alone
    # rounding the weights to BF16 changes them by 20-40%.  So the adjoint is
    # checked on a coarse grid (finest cell 1/24).  There the same rounding
    # still moves the oracle's residual-network gradients by 1.5-4% with the
    # window open (alpha = 4) and by up to ~17% with it half closed
    # (alpha = 1.5, small gradients).  The GPU (two BF16 networks in series,
    # operands rounded in every product) must stay within three times that
    # shift of the FP64 oracle, per group in relative L2 and for every entry
    # relative to the largest, and never further than the plain BF16 bounds
    # (1e-1 / 2e-1) where the shift is small.  A wrong term (sign, missing
    # Jacobian, transposed weight) moves the affected groups by O(1).
    import copy
    sc = _coarse_body()
    res = scenes.residual_weights(31, out_scale=0.3)
    g = np.random.default_rng(6)
    pid = np.array([(12 + g.integers(0, 8)) * sc.W + 12 + g.integers(0, 8) for _ in range(12)] +
                   list(g.integers(0, sc.H * sc.W, 4)), dtype=np.int32)
    tgt = g.random((16, 3)).astype(np.float32)
    # refined: a pose-refiner adjustment; the residual network then sees the
    # observed pose's joint angles (R(Delta_j) R(omega_j)), so dL/dW_omega
    # is taken against those
    delta = np.random.default_rng(12).normal(0.0, 0.3, (24, 3)).astype(np.float32) if refined else None
    lg, got, gG = _res_grads_gpu(sc, res, pid, tgt, alpha, delta=delta)
    lo, want, oG = _res_grads_oracle(sc, res, pid, tgt, alpha, delta=delta)
    sc_r = copy.copy(sc)
    sc_r.mlp = [_bf16(w) for w in sc.mlp]
    _, shifted, _ = _res_grads_oracle(sc_r, ([_bf16(w) for w in res[0]], _bf16(res[1])), pid, tgt, alpha,
                                      delta=delta)
    print(f"[residual adjoint alpha={alpha} refined={refined}] loss gpu {lg:.7f} oracle {lo:.7f}", flush=True)
    names = ["table", "logits"] + [f"w{k}" for k in range(len(sc.mlp))] + [f"res W{k + 1}" for k in range(5)] + \
        ["res W_omega"]
    bad = []
    for name, a, b, c in zip(names, got, want, shifted):
        if name == "res W1":
            b = b.copy()
            b[:, 27:] = 0.0          # inputs 27..31 of gamma are zero padding: no gradient
        nb, mb = np.linalg.norm(b), np.abs(b).max()
        rel = float(np.linalg.norm(a - b) / max(nb, 1e-30))
        ew = float(np.abs(a - b).max() / max(mb, 1e-30))
        s_rel = float(np.linalg.norm(c - b) / max(nb, 1e-30))
        s_ew = float(np.abs(c - b).max() / max(mb, 1e-30))
        t_rel, t_ew = max(3 * s_rel, 1e-1), max(3 * s_ew, 2e-1)
        print(f"  {name:11s} rel-L2 {rel:.2e} (bf16 shift {s_rel:.2e})  every entry {ew:.2e} "
              f"(shift {s_ew:.2e})  |g| {nb:.3e}", flush=True)
        if not (nb > 0 and rel <= t_rel and ew <= t_ew):
            bad.append(name)
    relG = float(np.linalg.norm(gG - oG) / np.linalg.norm(oG))
    print(f"  dL/dG       rel-L2 {relG:.2e}", flush=True)
    assert abs(lg - lo) <= 1e-2 * lo
    assert not bad, bad


def test_training_the_residual_network_fits_a_residual_motion():
    # The image of a body whose canonical points are moved by a residual
    # network ("teacher") is the target.  The student has the same field,
    # skinning and residual network except for a zero output layer, so it
    # starts as the plain renderer; mnr_train_step trains only its residual
    # network.  The loss must fall far below the plain renderer's: what the
    # learned residual motion gains over the method without it.
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=48, W=48, spp=96, res=32, log2_T=16, seed=16541 + 4)
    teach = scenes.residual_weights(41, out_scale=0.15)
    target = torch.as_tensor(_render(sc, 0, 2, teach, alpha=4.0)[:, :3], device="cuda").contiguous()
    student = ([w.copy() for w in teach[0]], teach[1].copy())
    student[0][4][:] = 0.0
    tr = m.Trainer(torch.as_tensor(sc.table, device="cuda"), [torch.as_tensor(w, device="cuda") for w in sc.mlp],
                   torch.as_tensor(sc.logits, device="cuda"), sc.level_res, m.F32, m.BF16, max_rays=sc.H * sc.W,
                   spp=sc.spp, lr_field=0.0, train_motion=False, residual=(student[0], student[1], 4.0),
                   lr_res=2e-3)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    pid = torch.arange(0, sc.H * sc.W, dtype=torch.int32, device="cuda")
    losses = []
    for k in range(300):
        tr.step(pose, cam, sc.H, sc.W, sc.spp, pid, target, seed=k, ert_tau=0.0)
        losses.append(tr.loss())
    print(f"[residual training] loss {losses[0]:.5f} (plain renderer) -> {losses[-1]:.5f}; "
          f"every 50: {[round(v, 5) for v in losses[::50]]}", flush=True)
    assert losses[0] > 1e-3                    # the residual motion changes the image
    assert losses[-1] < 0.3 * losses[0]
