"""GPU adjoint vs the FP64 oracle's gradient (autograd over the oracle's
forward, itself pinned to central differences on the CPU), on a 16-ray
subset with stratified jitter.  Also a directional finite-difference check
of the GPU gradient against the oracle loss.

Tolerances (relative L2 error per parameter group): FP32 path 2e-3 (FP32
forward/adjoint and unordered float atomics); BF16-MLP path 5e-2 (BF16
operands, 8-bit mantissa, in every MLP product).
"""
import numpy as np
import pytest
import torch

import scenes
from oracle import render as O
from oracle.rng import stratified_xi

pytestmark = pytest.mark.gpu

SEED = 77


def _scene():
    return scenes.scene_body(H=32, W=32, spp=128, res=32, log2_T=16, seed=16541 + 4)


def _rays(sc, n=16):
    g = np.random.default_rng(5)
    pid = np.array([(12 + g.integers(0, 8)) * sc.W + 12 + g.integers(0, 8) for _ in range(n // 2)] +
                   list(g.integers(0, sc.H * sc.W, n - n // 2)), dtype=np.int32)
    tgt = g.random((n, 3)).astype(np.float32)
    return pid, tgt


def gpu_grads(sc, pid, tgt, mlp_dtype, ert_tau=1e-6):
    import paper_2306_16541_amd as m
    fld, _ = m.upload_scene(sc, "cuda", m.F32, mlp_dtype)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=ert_tau, stratified=True, seed=SEED)
    pid_t = torch.as_tensor(pid, device="cuda")
    tgt_t = torch.as_tensor(tgt, device="cuda")
    n = len(pid)
    tch = torch.zeros(n, m.saved_size(sc.spp), device="cuda")
    rgba = m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, t_chunks=tch)
    grad_rgba = torch.empty(n, 4, device="cuda")
    loss = torch.zeros(1, device="cuda")
    m.mse_loss(rgba, tgt_t, grad_rgba, loss)
    g_table = torch.zeros(sc.table.shape, device="cuda")
    g_w = [torch.zeros(w.shape, device="cuda") for w in sc.mlp]
    g_wc = torch.zeros(sc.logits.shape, device="cuda")
    m.render_backward(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, tch, grad_rgba, g_table, g_w, g_wc)
    g_logits = torch.zeros_like(g_wc)
    m.softmax_bwd(fld.weights, g_wc, g_logits)
    torch.cuda.synchronize()
    return (float(loss.item()), g_table.cpu().numpy(), [w.cpu().numpy() for w in g_w], g_logits.cpu().numpy(),
            rgba.cpu().numpy())


def oracle_grads(sc, pid, tgt):
    field = O.Field.from_scene(sc, requires_grad=True)
    G = O.bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle)
    o, d = O.camera_rays(sc.cam, sc.H, sc.W, pid)
    rgba = O.render_rays(field, G, o, d, sc.spp, xi=stratified_xi(SEED, len(pid), sc.spp))
    loss = O.mse_loss(rgba, tgt)
    loss.backward()
    return (float(loss.detach()), field.table.grad.numpy(), [w.grad.numpy() for w in field.mlp], field.logits.grad.numpy(),
            rgba.detach().numpy())


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-30))


def _cos(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30))


@pytest.mark.parametrize("mlp_dtype,tol", [(0, 2e-3), (2, 5e-2)])
def test_adjoint_matches_oracle_gradient(mlp_dtype, tol):
    sc = _scene()
    pid, tgt = _rays(sc)
    lg, tg, wg, logg, rg = gpu_grads(sc, pid, tgt, mlp_dtype)
    lo, to, wo, logo, ro = oracle_grads(sc, pid, tgt)
    assert (ro[:, 3] > 0.5).sum() >= 4                 # the subset sees the body
    print(f"[dtype {mlp_dtype}] loss gpu {lg:.8f} oracle {lo:.8f}; rgba max-abs {np.abs(rg - ro).max():.2e}")
    assert abs(lg - lo) <= (1e-5 if mlp_dtype == 0 else 1e-2) * abs(lo)
    groups = [("table", tg, to), ("logits", logg, logo)] + [(f"w{k}", a, b) for k, (a, b) in enumerate(zip(wg, wo))]
    for name, a, b in groups:
        r, c = _rel(a, b), _cos(a, b)
        print(f"  {name:7s} rel-L2 {r:.3e} cos {c:.6f} |g| {np.linalg.norm(b):.3e}", flush=True)
        assert np.linalg.norm(b) > 0, name
        assert r <= tol, name
    # partition of unity of the grid scatter: per-level sums agree
    sg, so = tg.reshape(tg.shape[0], -1).sum(1), to.reshape(to.shape[0], -1).sum(1)
    np.testing.assert_allclose(sg, so, rtol=0, atol=max(tol, 1e-4) * np.abs(so).max())
    # softmax adjoint: gradients of each voxel's logits sum to zero
    assert np.abs(logg.sum(0)).max() <= 1e-6 * max(np.abs(logg).max(), 1e-12) + 1e-12


def test_adjoint_directional_derivative_matches_oracle_differences():
    # Move every parameter (table, MLP weights, logits) along the GPU
    # gradient g and take central differences of the FP64 oracle loss: the
    # directional derivative must equal g . g_true / |g| = |g| when the
    # adjoint is right.  The step is small enough that no ReLU or cell-face
    # kink lies inside the stencil (checked with the one-sided slopes).
    sc = _scene()
    pid, tgt = _rays(sc)
    _, tg, wg, logg, _ = gpu_grads(sc, pid, tgt, 0, ert_tau=0.0)
    gnorm = np.sqrt(sum(float((a.astype(np.float64) ** 2).sum()) for a in [tg, logg] + wg))
    G = O.bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle)
    o, d = O.camera_rays(sc.cam, sc.H, sc.W, pid)
    xi = stratified_xi(SEED, len(pid), sc.spp)

    def loss_at(eps):
        f = O.Field(sc.table.astype(np.float64) + eps * tg / gnorm,
                    [w.astype(np.float64) + eps * g / gnorm for w, g in zip(sc.mlp, wg)],
                    sc.logits.astype(np.float64) + eps * logg / gnorm, sc.level_res, sc.box_min, sc.box_max)
        return float(O.mse_loss(O.render_rays(f, G, o, d, sc.spp, xi=xi), tgt))

    eps = 1e-7
    lm, l0, lp = loss_at(-eps), loss_at(0.0), loss_at(eps)
    left, right, fd = (l0 - lm) / eps, (lp - l0) / eps, (lp - lm) / (2 * eps)
    print(f"  |g| {gnorm:.6e}  directional fd {fd:.6e}  one-sided {left:.6e} {right:.6e}", flush=True)
    assert abs(left - right) <= 1e-4 * abs(fd)
    assert abs(fd - gnorm) <= 1e-3 * gnorm


def test_adjoint_after_full_frame_forward():
    # Full-frame forward (ray-packet kernel, per-sample early termination)
    # followed by the adjoint over every pixel, against the oracle.
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=16, W=16, spp=64, res=32, log2_T=16, seed=16541 + 9)
    fld, _ = m.upload_scene(sc, "cuda", m.F32, m.F32)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=1e-6)
    n = sc.H * sc.W
    tgt = np.random.default_rng(1).random((n, 3)).astype(np.float32)
    tch = torch.zeros(n, m.saved_size(sc.spp), device="cuda")
    rgba = m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, None, t_chunks=tch)
    grad_rgba = torch.empty(n, 4, device="cuda")
    m.mse_loss(rgba, torch.as_tensor(tgt, device="cuda"), grad_rgba)
    g_table = torch.zeros(sc.table.shape, device="cuda")
    g_w = [torch.zeros(w.shape, device="cuda") for w in sc.mlp]
    g_wc = torch.zeros(sc.logits.shape, device="cuda")
    m.render_backward(fld, pose, cam, sc.H, sc.W, sc.spp, opts, None, tch, grad_rgba, g_table, g_w, g_wc)
    g_logits = torch.zeros_like(g_wc)
    m.softmax_bwd(fld.weights, g_wc, g_logits)
    torch.cuda.synchronize()
    field = O.Field.from_scene(sc, requires_grad=True)
    G = O.bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle)
    o, d = O.camera_rays(sc.cam, sc.H, sc.W)
    O.mse_loss(O.render_rays(field, G, o, d, sc.spp), tgt).backward()
    pairs = [("table", g_table, field.table.grad), ("logits", g_logits, field.logits.grad)] + \
        [(f"w{k}", a, b.grad) for k, (a, b) in enumerate(zip(g_w, field.mlp))]
    for name, a, b in pairs:
        r = _rel(a.cpu().numpy(), b.numpy())
        print(f"  full-frame {name:7s} rel-L2 {r:.3e}", flush=True)
        assert r <= 2e-3, name


def test_render_fn_autograd_matches_oracle_gradient():
    # The adjoint behind torch.autograd: the loss is built and differentiated
    # by torch on the GPU, while the render and its backward are RenderFn
    # (the library's kernels).  dL/dW^c goes to the logits through the
    # library's softmax adjoint; tolerances as for the FP32 path above.
    import paper_2306_16541_amd as m
    sc = _scene()
    pid, tgt = _rays(sc)
    fld, _ = m.upload_scene(sc, "cuda", m.F32, m.F32)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=1e-6, stratified=True, seed=SEED)
    pid_t = torch.as_tensor(pid, device="cuda")
    tgt_t = torch.as_tensor(tgt, device="cuda")
    table = fld.table.requires_grad_(True)
    weights = fld.weights.requires_grad_(True)
    mlp = [w.requires_grad_(True) for w in fld.mlp]
    rgba = m.RenderFn.apply(table, weights, *mlp, (fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t))
    loss = ((rgba[:, :3] - tgt_t) ** 2).mean()
    loss.backward()
    g_logits = torch.zeros_like(weights)
    m.softmax_bwd(weights.detach(), weights.grad, g_logits)
    torch.cuda.synchronize()
    lo, to, wo, logo, _ = oracle_grads(sc, pid, tgt)
    assert abs(float(loss.detach()) - lo) <= 1e-5 * abs(lo)
    groups = [("table", table.grad, to), ("logits", g_logits, logo)] + \
        [(f"w{k}", w.grad, b) for k, (w, b) in enumerate(zip(mlp, wo))]
    for name, a, b in groups:
        a = a.detach().cpu().numpy()
        r = _rel(a, b)
        print(f"  autograd {name:7s} rel-L2 {r:.3e}", flush=True)
        assert np.linalg.norm(b) > 0, name
        assert r <= 2e-3, name
