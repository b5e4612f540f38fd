"""mnr_train_step on the GPU: the loss falls, a checkpoint restores the run,
and the full training-step workload (8192 random rays x 128 samples over the
512x512 body scene) runs."""
import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu


def _trainer(sc, mlp_dtype, max_rays=4096, train_motion=True):
    import paper_2306_16541_amd as m
    dev = "cuda"
    return m.Trainer(torch.as_tensor(sc.table, device=dev), [torch.as_tensor(w, device=dev) for w in sc.mlp],
                     torch.as_tensor(sc.logits, device=dev), sc.level_res, m.F32, mlp_dtype, max_rays=max_rays,
                     spp=sc.spp, train_motion=train_motion)


def _batches(sc, n, steps, seed=3):
    out = []
    for s in range(steps):
        pid, tgt = scenes.train_batch(seed + s, sc.H, sc.W, n)
        out.append((torch.as_tensor(pid, device="cuda"), torch.as_tensor(tgt, device="cuda")))
    return out


@pytest.mark.parametrize("mlp_dtype", [0, 2])
def test_loss_decreases(mlp_dtype):
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=64, W=64, spp=64, res=32, log2_T=16)
    tr = _trainer(sc, mlp_dtype)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    pid, tgt = _batches(sc, 2048, 1)[0]        # fit one fixed batch
    losses = []
    for s in range(40):
        tr.step(pose, cam, sc.H, sc.W, sc.spp, pid, tgt, seed=s)
        losses.append(tr.loss())
    print("losses", losses[0], losses[9], losses[-1])
    assert np.all(np.isfinite(losses))
    # random U(0,1) targets: the loss can only fall towards their variance
    assert np.mean(losses[-5:]) < 0.9 * np.mean(losses[:5])
    assert losses[-1] < losses[0]


def test_checkpoint_round_trip():
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=48, W=48, spp=64, res=32, log2_T=16)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    batches = _batches(sc, 1024, 10)
    a = _trainer(sc, 2)
    for s in range(5):
        a.step(pose, cam, sc.H, sc.W, sc.spp, *batches[s], seed=s)
    ckpt = a.state_dict()
    la = []
    for s in range(5, 10):
        a.step(pose, cam, sc.H, sc.W, sc.spp, *batches[s], seed=s)
        la.append(a.loss())
    b = _trainer(sc, 2)
    b.load_state_dict(ckpt)
    lb = []
    for s in range(5, 10):
        b.step(pose, cam, sc.H, sc.W, sc.spp, *batches[s], seed=s)
        lb.append(b.loss())
    print("resumed", la, lb)
    np.testing.assert_allclose(lb, la, rtol=1e-3)


def test_full_size_training_step_runs():
    import paper_2306_16541_amd as m
    sc = scenes.scene_body()               # 512x512 scene, T = 2^19, R = 64
    tr = _trainer(sc, 2, max_rays=8192)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    pid, tgt = _batches(sc, 8192, 1)[0]
    for s in range(3):
        tr.step(pose, cam, sc.H, sc.W, sc.spp, pid, tgt, seed=s)
    torch.cuda.synchronize()
    assert np.isfinite(tr.loss())
    assert float(tr.buf["table_grad"].abs().sum()) > 0
    assert float(tr.buf["logits_grad"].abs().sum()) > 0
