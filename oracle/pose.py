"""FP64 oracle of the pose refiner (test infrastructure).

TEST INFRASTRUCTURE ONLY (same rules as oracle/render.py).

Paper: Sec. 4.1, Eq. 5-6.  A small MLP maps the estimated joint angles
Omega (axis-angle per joint) to adjustments Delta = MLP_theta(Omega); the
refined pose is theta^o = (J, Delta (x) Omega).  Readings (each listed in
the design doc): (x) composes rotations per joint, R(omega^o_j) = R(Delta_j)
R(omega_j); the MLP has ReLU hidden layers, no biases and a linear output
of 3 values per joint.  The bone transforms then follow Eq. 8 with the
composed rotations (oracle/render.py's forward kinematics).  The residual
motion network (Eq. 11) is conditioned on the observed pose's joint angles:
the axis-angle of each composed rotation, angle in [0, pi] (rotation_log).
"""
from __future__ import annotations

from typing import Sequence

import torch

from .render import F64, as64, rodrigues


def refine(weights: Sequence, omega) -> torch.Tensor:
    """Delta [J,3] = MLP_theta(Omega): ReLU hidden layers, linear output."""
    h = as64(omega).reshape(-1)
    ws = [as64(w) for w in weights]
    for W in ws[:-1]:
        h = torch.relu(W @ h)
    return (ws[-1] @ h).reshape(-1, 3)


def composed_rotations(omega, delta) -> torch.Tensor:
    """R(Delta_j) R(omega_j) per joint [J,3,3]."""
    return rodrigues(as64(delta)) @ rodrigues(as64(omega))


def bone_transforms_from_rotations(parents: Sequence[int], rest_joints, R: torch.Tensor) -> torch.Tensor:
    """G_j = B_j^-1 of Eq. 8 [J,3,4] from per-joint rotations R [J,3,3]:
    A_root = [R_root | J_root], A_j = A_parent [R_j | J_j - J_parent],
    B_j = A_j [I | -J_j]."""
    J = as64(rest_joints)
    rot, tr = [], []
    for j, p in enumerate(parents):
        if p < 0:
            rot.append(R[j]); tr.append(J[j])
        else:
            rot.append(rot[p] @ R[j]); tr.append(rot[p] @ (J[j] - J[p]) + tr[p])
    A_rot, A_tr = torch.stack(rot), torch.stack(tr)
    B_tr = A_tr - (A_rot @ J[:, :, None])[..., 0]
    G_rot = A_rot.transpose(1, 2)
    G_tr = -(G_rot @ B_tr[:, :, None])[..., 0]
    return torch.cat([G_rot, G_tr[:, :, None]], dim=2)


def refined_bone_transforms(parents, rest_joints, omega, delta) -> torch.Tensor:
    return bone_transforms_from_rotations(parents, rest_joints, composed_rotations(omega, delta))


def rotation_log(R) -> torch.Tensor:
    """Axis-angle [J,3] of rotations R [J,3,3], principal branch (angle in
    [0, pi]).  The angle from cos = (tr R - 1)/2 and sin = |vee(R - R^T)|/2;
    the axis from vee(R - R^T) / (2 sin), except near pi, where it is the
    dominant column of (R + R^T)/2 - cos I (proportional to a a^T), signed
    to agree with vee(R - R^T)."""
    R = as64(R)
    out = []
    for Rj in R:
        v = 0.5 * torch.stack([Rj[2, 1] - Rj[1, 2], Rj[0, 2] - Rj[2, 0], Rj[1, 0] - Rj[0, 1]])
        c = 0.5 * (torch.trace(Rj) - 1.0)
        s = torch.linalg.norm(v)
        th = torch.atan2(s, c)
        if float(th) < 1e-8:
            out.append(v)
            continue
        if float(c) > -0.5:
            out.append(v * (th / s))
            continue
        A = 0.5 * (Rj + Rj.T) - c * torch.eye(3, dtype=F64)
        k = int(torch.argmax(torch.diagonal(A)))
        a = A[:, k] / torch.linalg.norm(A[:, k])
        if float(a @ v) < 0.0:
            a = -a
        out.append(th * a)
    return torch.stack(out)


def observed_angles(omega, delta) -> torch.Tensor:
    """The observed pose theta^o's joint angles [J,3]: the axis-angle of
    R(Delta_j) R(omega_j) (what the residual network is conditioned on)."""
    return rotation_log(composed_rotations(omega, delta))
