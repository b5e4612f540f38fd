"""Pins of the pose-refiner oracle (oracle/pose.py): the composition and
forward kinematics against closed forms and the unrefined FK, and the
gradient that torch.autograd takes through them against central finite
differences of the FP64 forward."""
import math

import numpy as np
import torch

import oracle
import scenes
from oracle.pose import composed_rotations, refine, refined_bone_transforms


def test_zero_adjustment_is_the_unrefined_pose():
    parents, rest = scenes.skeleton()
    aa = scenes.pose(7, 0.3)
    G0 = oracle.bone_transforms(parents, rest, aa)
    G1 = refined_bone_transforms(parents, rest, aa, np.zeros_like(aa))
    assert torch.allclose(G0, G1, atol=1e-14)


def test_adjustment_that_undoes_the_pose_gives_the_rest_pose():
    # Delta_j = -omega_j: R(-w) R(w) = I, so every bone transform is the identity.
    parents, rest = scenes.skeleton()
    aa = scenes.pose(8, 0.3)
    G = refined_bone_transforms(parents, rest, aa, -aa)
    eye = torch.cat([torch.eye(3, dtype=torch.float64), torch.zeros(3, 1, dtype=torch.float64)], 1)
    assert torch.allclose(G, eye.expand_as(G), atol=1e-12)


def test_composition_about_one_axis_adds_angles():
    # Rotations about the same axis commute and add.
    w = torch.tensor([[0.0, 0.3, 0.0]], dtype=torch.float64)
    d = torch.tensor([[0.0, -0.1, 0.0]], dtype=torch.float64)
    R = composed_rotations(w, d)[0]
    c, s = math.cos(0.2), math.sin(0.2)
    want = torch.tensor([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=torch.float64)
    assert torch.allclose(R, want, atol=1e-15)


def test_refiner_closed_form():
    # One hidden layer: Delta = W2 ReLU(W1 Omega).
    g = np.random.default_rng(2)
    W1, W2 = g.standard_normal((8, 72)), g.standard_normal((72, 8))
    om = g.standard_normal(72)
    want = (W2 @ np.maximum(W1 @ om, 0.0)).reshape(24, 3)
    assert np.allclose(refine([W1, W2], om).numpy(), want, atol=1e-12)


def test_autograd_through_refiner_and_fk_matches_finite_differences():
    parents, rest = scenes.skeleton()
    g = np.random.default_rng(3)
    aa = scenes.pose(9, 0.3).astype(np.float64)
    ws = [torch.tensor(g.standard_normal((16, 72)) * 0.1, requires_grad=True),
          torch.tensor(g.standard_normal((72, 16)) * 0.1, requires_grad=True)]
    probe = torch.as_tensor(g.standard_normal((24, 3, 4)))

    def f(w0, w1):
        return (refined_bone_transforms(parents, rest, aa, refine([w0, w1], aa)) * probe).sum()
    f(*ws).backward()
    h = 1e-6
    for k, W in enumerate(ws):
        for idx in [(0, 0), (3, 17), (10, 5), (15, 71)] if k == 0 else [(0, 0), (17, 3), (40, 9), (71, 15)]:
            wp = [w.detach().clone() for w in ws]
            wm = [w.detach().clone() for w in ws]
            wp[k][idx] += h
            wm[k][idx] -= h
            fd = (f(*wp) - f(*wm)).item() / (2 * h)
            assert abs(fd - W.grad[idx].item()) <= 1e-6 * max(1.0, abs(fd))
