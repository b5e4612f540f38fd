"""The learned part, trained on the GPU by the library's own forward and
adjoint kernels (mnr_train_step), and what it gains.

Protocol of the paper's evaluation (Sec. 5.1-5.2): train from ONE camera on
a sequence in which the subject moves (here: turns in place and moves its
joints), evaluate on other cameras (novel views) of the training poses.
Only a correct warp to the shared canonical body lets the views of
different poses combine, so learned skinning should beat fixed skinning.

Targets: analytic images of a rigidly skinned ellipsoid body with one
colour per bone (tests/teacher.py), 24 poses, root yaw uniform in [0, 2pi),
other joints ~ N(0, 0.2^2) rad, 96x96.  Students share one initialisation
(small random grid, Xavier MLP, uniform blend weights):
  untrained - the initialisation itself
  frozen    - grid + MLP trained, blend-weight logits frozen at uniform
              (every bone weighs the same: no learned skinning)
  learned   - grid + MLP + blend-weight logits trained
Hyper-parameters (Adam 0.9/0.99; lr 1e-2 grid/MLP, 3e-2 logits; 2500 steps
of 4096 rays) are the test's own: the free logits stand in for the paper's
weight-volume CNN.
"""
import math

import numpy as np
import pytest
import torch

import scenes
from teacher import render_teacher

pytestmark = pytest.mark.gpu

H = W = 96
SPP = 64
N_RAYS = 4096
STEPS = 2500


def _psnr(a, b):
    return 10 * math.log10(1.0 / max(float(np.mean((a.astype(np.float64) - b) ** 2)), 1e-12))


def _poses(n, seed=5):
    g = np.random.default_rng(seed)
    out = []
    for k in range(n):
        aa = scenes.pose(seed * 100 + k, 0.2).astype(np.float64)
        aa[0] = [0.0, g.uniform(0.0, 2.0 * math.pi), 0.0]     # the subject turns in place
        out.append(aa.astype(np.float32))
    return out


def _student(train_motion):
    import paper_2306_16541_amd as m
    g = np.random.default_rng(123)
    table = torch.as_tensor(g.uniform(-1e-4, 1e-4, (16, 1 << 16, 2)).astype(np.float32), device="cuda")
    mlp = [torch.as_tensor(w, device="cuda") for w in scenes.mlp_weights(123, (32, 64, 64, 4))]
    logits = torch.zeros(25, 32, 32, 32, device="cuda")
    return m.Trainer(table, mlp, logits, scenes.LEVEL_RES, m.F32, m.F32, max_rays=N_RAYS, spp=SPP,
                     lr_field=1e-2, lr_motion=3e-2, train_motion=train_motion)


def _evaluate(tr, held):
    import paper_2306_16541_amd as m
    parents, rest = scenes.skeleton()
    ps = []
    for aa, cam, img in held:
        out = m.render(tr.field, m.PoseHost(parents, rest, aa), m.make_camera(cam), H, W, SPP).cpu().numpy()
        ps.append(_psnr(out[:, :3], img[:, :3]))
    return float(np.mean(ps))


def _train(tr, data):
    g = np.random.default_rng(7)
    losses = []
    for s in range(STEPS):
        pose, cam, img = data[g.integers(len(data))]
        pid = torch.as_tensor(g.integers(0, H * W, N_RAYS).astype(np.int32), device="cuda")
        tr.step(pose, cam, H, W, SPP, pid, img[pid.long()].contiguous(), seed=s)
        if s % 250 == 0 or s == STEPS - 1:
            losses.append(tr.loss())
    return losses


def test_learned_skinning_beats_untrained_and_frozen():
    import paper_2306_16541_amd as m
    parents, rest = scenes.skeleton()
    colors = scenes.bone_colors(2)
    poses = _poses(24)
    train_cam = scenes.camera(H, W, yaw=0.0)
    data = [(m.PoseHost(parents, rest, aa), m.make_camera(train_cam),
             torch.as_tensor(render_teacher(parents, rest, aa, train_cam, H, W, colors)[:, :3], device="cuda"))
            for aa in poses]
    held = []
    for aa in poses[:6]:
        for yaw in (0.5 * math.pi, math.pi):
            cam = scenes.camera(H, W, yaw=yaw)
            held.append((aa, cam, render_teacher(parents, rest, aa, cam, H, W, colors)))
    untrained = _evaluate(_student(True), held)
    frozen_tr = _student(False)
    lf = _train(frozen_tr, data)
    frozen = _evaluate(frozen_tr, held)
    learned_tr = _student(True)
    ll = _train(learned_tr, data)
    learned = _evaluate(learned_tr, held)
    print(f"novel-view PSNR: untrained {untrained:.2f} dB, frozen skinning {frozen:.2f} dB, "
          f"learned {learned:.2f} dB", flush=True)
    print("loss (frozen) ", [round(v, 5) for v in lf])
    print("loss (learned)", [round(v, 5) for v in ll])
    assert ll[-1] < 0.25 * ll[0]
    assert ll[-1] < lf[-1]
    assert learned > untrained + 4.0
    assert learned > frozen + 1.0
