"""FP64 oracle of the pose refiner (test infrastructure).

TEST INFRASTRUCTURE ONLY (same rules as oracle/render.py).

Paper: Sec. 4.1, Eq. 5-6.  A small MLP maps the estimated joint angles
Omega (axis-angle per joint) to adjustments Delta = MLP_theta(Omega); the
refined pose is theta^o = (J, Delta (x) Omega).  Readings (each listed in
the design doc): (x) composes rotations per joint, R(omega^o_j) = R(Delta_j)
R(omega_j); the MLP has ReLU hidden layers, no biases and a linear output
of 3 values per joint.  The bone transforms then follow Eq. 8 with the
composed rotations (oracle/render.py's forward kinematics).
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
