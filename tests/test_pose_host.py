"""The library's host pose path against the oracle (no GPU needed): forward
kinematics with refiner adjustments, its adjoint (dual numbers, FP64), and
the refiner MLP with its adjoint."""
import numpy as np
import torch

import oracle
import scenes
from oracle.pose import refine, refined_bone_transforms


def _m():
    import paper_2306_16541_amd as m
    return m


def test_fk_with_adjustment_matches_oracle():
    m = _m()
    parents, rest = scenes.skeleton()
    for seed in (1, 2):
        aa = scenes.pose(seed, 0.3)
        d = scenes.pose(seed + 50, 0.1)
        G = m.fk_bones(m.PoseHost(parents, rest, aa, d))
        Go = refined_bone_transforms(parents, rest, aa, d).numpy()
        assert np.abs(G - Go).max() < 3e-7


def test_fk_adjoint_matches_oracle_autograd():
    m = _m()
    parents, rest = scenes.skeleton()
    g = np.random.default_rng(4)
    aa = scenes.pose(3, 0.3).astype(np.float32)
    for delta in (None, scenes.pose(60, 0.1).astype(np.float32)):
        gG = g.standard_normal((24, 3, 4)).astype(np.float32)
        gd, ga = m.fk_backward(m.PoseHost(parents, rest, aa, delta), gG)
        w = torch.tensor(aa.astype(np.float64), requires_grad=True)
        dl = torch.tensor(np.zeros((24, 3)) if delta is None else delta.astype(np.float64), requires_grad=True)
        (refined_bone_transforms(parents, rest, w, dl) * torch.as_tensor(gG.astype(np.float64))).sum().backward()
        assert np.allclose(ga, w.grad.numpy(), rtol=1e-5, atol=1e-5)
        assert np.allclose(gd, dl.grad.numpy(), rtol=1e-5, atol=1e-5)


def test_refiner_and_its_adjoint_match_oracle():
    m = _m()
    g = np.random.default_rng(5)
    ws = [(g.standard_normal((48, 72)) * 0.2).astype(np.float32), (g.standard_normal((48, 48)) * 0.2).astype(np.float32),
          (g.standard_normal((72, 48)) * 0.2).astype(np.float32)]
    ref = m.PoseRefiner(ws)
    aa = scenes.pose(6, 0.3).astype(np.float32)
    d = ref.apply(aa)
    tw = [torch.tensor(w.astype(np.float64), requires_grad=True) for w in ws]
    do = refine(tw, aa.astype(np.float64))
    assert np.allclose(d, do.detach().numpy(), rtol=1e-5, atol=1e-6)
    gd = g.standard_normal((24, 3)).astype(np.float32)
    ref.backward(aa, gd)
    (do * torch.as_tensor(gd.astype(np.float64))).sum().backward()
    for k in range(3):
        assert np.allclose(ref.g[k], tw[k].grad.numpy(), rtol=1e-5, atol=1e-6)


def test_refiner_rejects_bad_shapes():
    m = _m()
    ref = m.PoseRefiner([np.zeros((8, 70), np.float32), np.zeros((72, 8), np.float32)])   # input width != 72
    try:
        ref.apply(np.zeros((24, 3), np.float32))
    except m.MnrError as e:
        assert "widths" in str(e)
    else:
        raise AssertionError("accepted a refiner whose input is not 3 n_joints wide")


def test_refiner_adam_step_matches_adam_written_out():
    # Two steps of the library's host Adam against the update written out
    # here (Kingma and Ba 2015, with bias correction; beta = 0.9 / 0.99 as in
    # Sec. 5.2); the gradients are cleared after each step.
    m = _m()
    g = np.random.default_rng(8)
    ws = [(g.standard_normal((16, 72)) * 0.2).astype(np.float32), (g.standard_normal((72, 16)) * 0.2).astype(np.float32)]
    lr, b1, b2, eps = 1e-2, 0.9, 0.99, 1e-8
    ref = m.PoseRefiner(ws, lr=lr, beta1=b1, beta2=b2, eps=eps)
    w = [x.astype(np.float64) for x in ws]
    mm = [np.zeros_like(x) for x in w]
    vv = [np.zeros_like(x) for x in w]
    for t in (1, 2):
        grads = [g.standard_normal(x.shape).astype(np.float32) for x in ws]
        for k in range(2):
            ref.g[k][:] = grads[k]
        ref.step()
        for k in range(2):
            gk = grads[k].astype(np.float64)
            mm[k] = b1 * mm[k] + (1 - b1) * gk
            vv[k] = b2 * vv[k] + (1 - b2) * gk * gk
            w[k] = w[k] - lr * (mm[k] / (1 - b1 ** t)) / (np.sqrt(vv[k] / (1 - b2 ** t)) + eps)
            np.testing.assert_allclose(ref.w[k], w[k], rtol=0, atol=2e-6)
            assert not ref.g[k].any()
        # the refiner reads the updated weights
        aa = scenes.pose(7, 0.3).astype(np.float32)
        np.testing.assert_allclose(ref.apply(aa), refine([torch.as_tensor(x) for x in w], aa.astype(np.float64)).numpy(),
                                   rtol=1e-4, atol=1e-5)
