"""The learned part, trained on the GPU by the library's own forward and
adjoint kernels (mnr_train_step), and what it gains.

Targets: analytic images of a rigidly skinned ellipsoid body with one colour
per bone (tests/teacher.py) at 8 training poses x 4 views.  Students share
one initialisation (small random grid, Xavier MLP, uniform blend weights):
  untrained  - the initialisation itself
  frozen     - grid + MLP trained, blend-weight logits frozen at uniform
               (every bone weighs the same: no learned skinning)
  learned    - grid + MLP + blend-weight logits trained
Held-out: 3 new poses x 2 new views.  The learned model must beat both.
Hyper-parameters (Adam 0.9/0.99; lr 1e-2 for grid/MLP and logits) are the
test's own: the free logits stand in for the paper's weight-volume CNN.
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
STEPS = 1500


def _images(poses, yaws, colors):
    parents, rest = scenes.skeleton()
    out = []
    for aa in poses:
        for yaw in yaws:
            cam = scenes.camera(H, W, yaw=yaw)
            out.append((aa, cam, render_teacher(parents, rest, aa, cam, H, W, colors)))
    return out


def _psnr(a, b):
    return 10 * math.log10(1.0 / max(float(np.mean((a.astype(np.float64) - b) ** 2)), 1e-12))


def _student(train_motion):
    import paper_2306_16541_amd as m
    g = np.random.default_rng(123)
    table = torch.as_tensor(g.uniform(-1e-4, 1e-4, (16, 1 << 16, 2)).astype(np.float32), device="cuda")
    mlp = [torch.as_tensor(w, device="cuda") for w in scenes.mlp_weights(123, (32, 64, 64, 4))]
    logits = torch.zeros(25, 32, 32, 32, device="cuda")
    return m.Trainer(table, mlp, logits, scenes.LEVEL_RES, m.F32, m.F32, max_rays=N_RAYS, spp=SPP,
                     lr_field=1e-2, lr_motion=1e-2, train_motion=train_motion)


def _evaluate(tr, held):
    import paper_2306_16541_amd as m
    parents, rest = scenes.skeleton()
    ps = []
    for aa, cam, img in held:
        out = m.render(tr.field, m.PoseHost(parents, rest, aa), m.make_camera(cam), H, W, SPP).cpu().numpy()
        ps.append(_psnr(out[:, :3], img[:, :3]))
    return float(np.mean(ps))


def _train(tr, train):
    import paper_2306_16541_amd as m
    parents, rest = scenes.skeleton()
    g = np.random.default_rng(7)
    data = [(m.PoseHost(parents, rest, aa), m.make_camera(cam), torch.as_tensor(img[:, :3], device="cuda"))
            for aa, cam, img in train]
    losses = []
    for s in range(STEPS):
        pose, cam, img = data[g.integers(len(data))]
        pid = torch.as_tensor(g.integers(0, H * W, N_RAYS).astype(np.int32), device="cuda")
        tr.step(pose, cam, H, W, SPP, pid, img[pid.long()].contiguous(), seed=s)
        if s % 100 == 0 or s == STEPS - 1:
            losses.append(tr.loss())
    return losses


def test_learned_skinning_beats_untrained_and_frozen():
    colors = scenes.bone_colors(2)
    train = _images([scenes.pose(100 + k, 0.2) for k in range(8)], [0.0, 0.5 * math.pi, math.pi, 1.5 * math.pi],
                    colors)
    held = _images([scenes.pose(200 + k, 0.2) for k in range(3)], [0.25 * math.pi, 1.25 * math.pi], colors)
    untrained = _evaluate(_student(True), held)
    frozen_tr = _student(False)
    lf = _train(frozen_tr, train)
    frozen = _evaluate(frozen_tr, held)
    learned_tr = _student(True)
    ll = _train(learned_tr, train)
    learned = _evaluate(learned_tr, held)
    print(f"held-out PSNR: untrained {untrained:.2f} dB, frozen skinning {frozen:.2f} dB, "
          f"learned {learned:.2f} dB", flush=True)
    print("loss (frozen) ", [round(v, 5) for v in lf])
    print("loss (learned)", [round(v, 5) for v in ll])
    assert ll[-1] < 0.5 * ll[0]
    assert learned > untrained + 5.0
    assert learned > frozen + 0.5
