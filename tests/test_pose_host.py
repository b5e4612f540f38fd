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
