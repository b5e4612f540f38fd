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


# ---- the observed pose's joint angles (what the residual network sees) ----

def _rot(axis, angle):
    a = np.asarray(axis, np.float64)
    return oracle.render.rodrigues(torch.tensor(a / np.linalg.norm(a) * angle)[None])[0]


def test_rotation_log_hand_values():
    # 90 degrees about z, 180 degrees about x (either sign is the same
    # rotation), the identity
    from oracle.pose import rotation_log
    Rz = torch.tensor([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]], dtype=torch.float64)
    assert torch.allclose(rotation_log(Rz[None])[0], torch.tensor([0.0, 0.0, math.pi / 2], dtype=torch.float64),
                          atol=1e-15)
    Rx = torch.diag(torch.tensor([1.0, -1.0, -1.0], dtype=torch.float64))
    w = rotation_log(Rx[None])[0]
    assert abs(abs(float(w[0])) - math.pi) < 1e-15 and float(w[1:].abs().max()) < 1e-15
    assert float(rotation_log(torch.eye(3, dtype=torch.float64)[None]).abs().max()) == 0.0


def test_rotation_log_inverts_rodrigues_on_the_principal_branch():
    # log(R(w)) = w for |w| < pi, and R(log(R)) = R for every rotation,
    # angles from 0 to pi, near pi included (where the axis comes from the
    # symmetric part)
    from oracle.pose import rotation_log
    g = np.random.default_rng(3)
    angles = [0.0, 1e-12, 1e-7, 1e-3, 0.3, 1.0, 2.0, 2.6, 3.0, math.pi - 1e-4, math.pi - 1e-8, math.pi]
    for ang in angles:
        for _ in range(4):
            axis = g.normal(size=3)
            R = _rot(axis, ang)
            w = rotation_log(R[None])[0]
            assert float((oracle.render.rodrigues(w[None])[0] - R).abs().max()) < 1e-12, ang
            if ang < math.pi - 1e-3:
                want = torch.tensor(axis / np.linalg.norm(axis) * ang)
                assert float((w - want).abs().max()) < 1e-12, ang
            assert float(torch.linalg.norm(w)) <= math.pi + 1e-12


def test_observed_angles_compose_about_one_axis_and_reduce_without_adjustment():
    from oracle.pose import observed_angles
    sc = scenes.scene_body(H=8, W=8, spp=8, res=8, log2_T=14)
    om = np.asarray(sc.axis_angle, np.float64).reshape(-1, 3)
    assert float((observed_angles(om, np.zeros_like(om)) - torch.tensor(om)).abs().max()) < 1e-14
    n = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    a = np.array([0.4, -1.1, 2.0])[:, None] * n[None]
    b = np.array([0.7, 0.2, 1.5])[:, None] * n[None]
    got = observed_angles(a, b).numpy()
    want = (np.array([1.1, -0.9, 3.5])[:, None] * n[None])
    want[2] = (3.5 - 2 * math.pi) * n          # beyond pi: the principal branch wraps
    assert np.abs(got - want).max() < 1e-12
