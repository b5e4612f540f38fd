"""FP64 CPU oracle of the posed-body volume renderer (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or call this module.  The GPU
library never uses it, and it shares no code with the GPU library: it is an
independent, plain, slow statement of what the renderer computes, in
float64 on the CPU with plain PyTorch tensor ops (no blocking, fusion or
early termination).  Gradients are taken by torch.autograd over this
forward, so the oracle's adjoint is independent of the hand-written one.

Paper: "Envisioning a Next Generation Extended Reality Conferencing System
with Efficient Photorealistic Human Rendering" (arXiv 2306.16541).
Steps and where they are defined:
  * camera rays r(t) = o + t d ............ Sec. 2.1, Eq. 2
  * samples inside the body box ........... Sec. 4.4 (last paragraph)
  * bone transforms G_i = R_i x + t_i ..... Sec. 4.2, Eq. 8, from the pose
  * inverse linear blend skinning ......... Sec. 4.2, Eq. 7 and Eq. 9
  * canonical field c, sigma = MLP(enc(x)) . Sec. 4.4, Eq. 13 (encoding: the
    multiresolution grid of Mueller et al. 2022, cited in Sec. 2.3)
  * quadrature of the rendering integral .. Sec. 2.1, Eq. 3
  * likelihood augmentation of alpha ...... Sec. 4.4 (last paragraph)
  * squared-error loss .................... Sec. 2.1 and Sec. 5.2, Eq. 14
    (MSE term only)
  * optional residual non-rigid motion .... Sec. 4.3, Eq. 11-12
    (oracle/residual.py)
  * optional frequency-encoded field ...... Sec. 4.4, Eq. 13, Fig. 9 (a Field
    with encoding = "freq"; oracle/freq_field.py)

Readings of ambiguous passages (each listed in the design doc):
  * Eq. 3: delta_i is the stratum width (t_f - t_n)/S for every sample, so
    the last sample has a finite width; the summand is
    T_i * (1 - exp(-sigma_i delta_i)) * c_i.
  * Eq. 9: w_i^c(G_i(x)) is channel i of the canonical weight volume,
    trilinearly sampled at the canonical point G_i(x); the denominator L is
    clamped below by eps_L = 1e-6.
  * Sec. 4.4 augmentation: alpha'_i = alpha_i * min(L_i, 1), with L_i the
    Eq. 9 denominator; then T_i is the running product of (1 - alpha').
  * canonical pose = rest pose; FK composes parent transforms.
  * weight volume = per-voxel softmax over bones + 1 background channel of
    free logits, vertex-aligned over the canonical box, zero outside it.
  * rendering uses the stratum midpoints (xi = 0.5); training draws xi from
    splitmix64 (oracle/rng.py).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np
import torch

F64 = torch.float64
EPS_L = 1e-6          # lower clamp of the Eq. 9 denominator
DIR_EPS = 1e-12       # |d_a| below this: the ray is parallel to slab a


def as64(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(F64)
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


# ---------------------------------------------------------------------------
# Pose -> bone transforms (Sec. 4.2, Eq. 8).
# ---------------------------------------------------------------------------

def skew(w: torch.Tensor) -> torch.Tensor:
    """[..., 3] -> cross-product matrix [..., 3, 3]."""
    z = torch.zeros_like(w[..., 0])
    return torch.stack([
        torch.stack([z, -w[..., 2], w[..., 1]], -1),
        torch.stack([w[..., 2], z, -w[..., 0]], -1),
        torch.stack([-w[..., 1], w[..., 0], z], -1)], -2)


def rodrigues(omega) -> torch.Tensor:
    """Axis-angle [J,3] -> rotation [J,3,3] by Rodrigues' formula
    R = I + sin(th) K + (1 - cos(th)) K^2, K = [k]_x, k = omega/th."""
    omega = as64(omega)
    th = torch.linalg.norm(omega, dim=-1)
    eye = torch.eye(3, dtype=F64).expand(omega.shape[:-1] + (3, 3))
    out = []
    for j in range(omega.shape[0]):
        if float(th[j]) < 1e-12:
            out.append(eye[j] + skew(omega[j]))
        else:
            K = skew(omega[j] / th[j])
            out.append(eye[j] + torch.sin(th[j]) * K + (1.0 - torch.cos(th[j])) * (K @ K))
    return torch.stack(out)


def world_transforms(parents: Sequence[int], rest_joints, axis_angle):
    """Forward kinematics: A_j = A_parent(j) o [R(omega_j) | J_j - J_parent(j)],
    A_root = [R(omega_root) | J_root].  Returns rotations [J,3,3] and
    translations [J,3] of A_j (parents must precede children)."""
    J = as64(rest_joints)
    R = rodrigues(axis_angle)
    rot, tr = [], []
    for j, p in enumerate(parents):
        if p < 0:
            rot.append(R[j]); tr.append(J[j])
        else:
            rot.append(rot[p] @ R[j]); tr.append(rot[p] @ (J[j] - J[p]) + tr[p])
    return torch.stack(rot), torch.stack(tr)


def bone_transforms(parents: Sequence[int], rest_joints, axis_angle) -> torch.Tensor:
    """G_j of Eq. 8 as [J,3,4] = [R_j | t_j], mapping an observed point to
    the canonical (rest) pose: G_j = B_j^-1 with B_j = A_j o [I | -J_j]."""
    A_rot, A_tr = world_transforms(parents, rest_joints, axis_angle)
    J = as64(rest_joints)
    B_tr = A_tr - (A_rot @ J[:, :, None])[..., 0]
    G_rot = A_rot.transpose(1, 2)
    G_tr = -(G_rot @ B_tr[:, :, None])[..., 0]
    return torch.cat([G_rot, G_tr[:, :, None]], dim=2)


# ---------------------------------------------------------------------------
# Rays and samples (Sec. 2.1 Eq. 2; Sec. 4.4 sampling inside the box).
# ---------------------------------------------------------------------------

def camera_rays(cam, H: int, W: int, pixel_ids=None):
    """Pinhole camera (x_cam = R_wc X + T).  Pixel (u, v) = (id % W, id // W)
    shoots through its centre.  Returns origin [3] and unit directions [B,3]."""
    if pixel_ids is None:
        pixel_ids = np.arange(H * W)
    pid = torch.as_tensor(np.asarray(pixel_ids, dtype=np.int64))
    u = (pid % W).to(F64)
    v = (pid // W).to(F64)
    Rwc = as64(cam.R_wc)
    Tc = as64(cam.T)
    dc = torch.stack([(u + 0.5 - float(cam.cx)) / float(cam.fx),
                      (v + 0.5 - float(cam.cy)) / float(cam.fy),
                      torch.ones_like(u)], dim=1)
    d = dc @ Rwc            # rows: R_wc^T d_cam
    d = d / torch.linalg.norm(d, dim=1, keepdim=True)
    o = -(Rwc.T @ Tc)
    return o, d


def ray_box(o: torch.Tensor, d: torch.Tensor, box_min, box_max):
    """Slab test against the body's axis-aligned box.  Returns t_near
    (clamped at 0), t_far and the hit mask (t_far > t_near)."""
    o = o.expand_as(d)
    tmin = torch.full(d.shape[:1], -math.inf, dtype=F64)
    tmax = torch.full(d.shape[:1], math.inf, dtype=F64)
    miss = torch.zeros(d.shape[:1], dtype=torch.bool)
    for a in range(3):
        lo, hi = float(box_min[a]), float(box_max[a])
        par = d[:, a].abs() < DIR_EPS
        miss |= par & ((o[:, a] < lo) | (o[:, a] > hi))
        safe = torch.where(par, torch.ones_like(d[:, a]), d[:, a])
        t1 = (lo - o[:, a]) / safe
        t2 = (hi - o[:, a]) / safe
        tmin = torch.where(par, tmin, torch.maximum(tmin, torch.minimum(t1, t2)))
        tmax = torch.where(par, tmax, torch.minimum(tmax, torch.maximum(t1, t2)))
    t_near = torch.clamp(tmin, min=0.0)
    hit = (~miss) & (tmax > t_near)
    return t_near, tmax, hit


def sample_ts(t_near: torch.Tensor, t_far: torch.Tensor, S: int, xi=None):
    """Stratified samples t_i = t_n + (i + xi_i) * delta, delta = (t_f - t_n)/S.
    xi = None means the stratum midpoints (xi = 0.5)."""
    delta = (t_far - t_near) / S
    i = torch.arange(S, dtype=F64)[None, :]
    xi = torch.full((1, S), 0.5, dtype=F64) if xi is None else as64(xi)
    return t_near[:, None] + (i + xi) * delta[:, None], delta


# ---------------------------------------------------------------------------
# Inverse linear blend skinning (Sec. 4.2, Eq. 7 and Eq. 9).
# ---------------------------------------------------------------------------

def motion_weights(logits) -> torch.Tensor:
    """Canonical blend weights W^c: softmax over the channel axis at each voxel."""
    return torch.softmax(as64(logits), dim=0)


def trilinear_zero_padded(volume: torch.Tensor, channel: torch.Tensor, q: torch.Tensor):
    """Trilinear sample of volume[channel] ([C,R,R,R], indexed [c][z][y][x])
    at grid coordinates q [...,3] = (x, y, z) in voxel units; a corner
    outside [0, R-1]^3 contributes zero."""
    R = volume.shape[-1]
    flat = volume.reshape(-1)
    i0 = torch.floor(q)
    f = q - i0
    i0 = i0.to(torch.int64)
    out = torch.zeros(q.shape[:-1], dtype=F64)
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                ix, iy, iz = i0[..., 0] + cx, i0[..., 1] + cy, i0[..., 2] + cz
                w = ((f[..., 0] if cx else 1 - f[..., 0]) *
                     (f[..., 1] if cy else 1 - f[..., 1]) *
                     (f[..., 2] if cz else 1 - f[..., 2]))
                ok = (ix >= 0) & (ix < R) & (iy >= 0) & (iy < R) & (iz >= 0) & (iz < R)
                idx = ((channel * R + iz.clamp(0, R - 1)) * R + iy.clamp(0, R - 1)) * R + ix.clamp(0, R - 1)
                out = out + torch.where(ok, w * flat[idx], torch.zeros_like(w))
    return out


def inverse_lbs(x: torch.Tensor, G: torch.Tensor, weights: torch.Tensor, box_min, box_max):
    """x [N,3] observed points; G [K,3,4]; weights [K+1,R,R,R].
    w~_i = W^c_i(G_i x);  L = sum_i w~_i;  x_skel = sum_i w~_i G_i x / max(L, eps).
    Returns x_skel [N,3], L [N]."""
    K = G.shape[0]
    R = weights.shape[-1]
    y = torch.einsum("kab,nb->nka", G[:, :, :3], x) + G[None, :, :, 3]     # [N,K,3]
    bmin, bmax = as64(box_min), as64(box_max)
    q = (y - bmin) / (bmax - bmin) * (R - 1)
    ch = torch.arange(K, dtype=torch.int64)[None, :].expand(x.shape[0], K)
    wt = trilinear_zero_padded(weights, ch, q)                              # [N,K]
    L = wt.sum(dim=1)
    xs = (wt[:, :, None] * y).sum(dim=1) / torch.clamp(L, min=EPS_L)[:, None]
    return xs, L


# ---------------------------------------------------------------------------
# Canonical field: multiresolution grid encoding + MLP (Sec. 4.4, Eq. 13).
# ---------------------------------------------------------------------------

HASH_PRIMES = (1, 2654435761, 805459861)   # spatial-hash primes of Mueller et al. 2022


def grid_index(c: torch.Tensor, N: int, T: int) -> torch.Tensor:
    """Table row of integer lattice vertex c [...,3] at a level of resolution N:
    dense x + (N+1)(y + (N+1) z) when (N+1)^3 <= T, else the spatial hash
    (x*p0 xor y*p1 xor z*p2) mod 2^32, masked to T - 1."""
    if (N + 1) ** 3 <= T:
        return c[..., 0] + (N + 1) * (c[..., 1] + (N + 1) * c[..., 2])
    m32 = 0xFFFFFFFF
    h = ((c[..., 0] * HASH_PRIMES[0]) & m32) ^ ((c[..., 1] * HASH_PRIMES[1]) & m32) \
        ^ ((c[..., 2] * HASH_PRIMES[2]) & m32)
    return h & (T - 1)


def grid_encode(x: torch.Tensor, table: torch.Tensor, level_res, box_min, box_max) -> torch.Tensor:
    """x [N,3] canonical points; table [L,T,F].  Per level: u = clamp to the
    unit cube, p = u N_l, cell i0 = min(floor(p), N_l - 1), trilinear blend
    of the 8 vertex features.  Output [N, L*F], level-major."""
    bmin, bmax = as64(box_min), as64(box_max)
    u = torch.clamp((x - bmin) / (bmax - bmin), 0.0, 1.0)
    T = table.shape[1]
    feats = []
    for l, N in enumerate(level_res):
        N = int(N)
        p = u * N
        i0 = torch.clamp(torch.floor(p), max=N - 1)
        f = p - i0
        i0 = i0.to(torch.int64)
        acc = torch.zeros((x.shape[0], table.shape[2]), dtype=F64)
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    c = i0 + torch.tensor([cx, cy, cz], dtype=torch.int64)
                    w = ((f[:, 0] if cx else 1 - f[:, 0]) *
                         (f[:, 1] if cy else 1 - f[:, 1]) *
                         (f[:, 2] if cz else 1 - f[:, 2]))
                    acc = acc + w[:, None] * table[l][grid_index(c, N, T)]
        feats.append(acc)
    return torch.cat(feats, dim=1)


def mlp(feat: torch.Tensor, weights: Sequence[torch.Tensor]):
    """Bias-free MLP: ReLU hidden layers; outputs c = sigmoid(o[0:3]),
    sigma = ReLU(o[3])."""
    h = feat
    for W in weights[:-1]:
        h = torch.relu(h @ W.T)
    o = h @ weights[-1].T
    return torch.sigmoid(o[:, :3]), torch.relu(o[:, 3])


# ---------------------------------------------------------------------------
# Compositing (Sec. 2.1 Eq. 3, with the Sec. 4.4 likelihood augmentation).
# ---------------------------------------------------------------------------

def composite(sigma: torch.Tensor, rgb: torch.Tensor, L: torch.Tensor, delta: torch.Tensor, bg):
    """sigma [B,S], rgb [B,S,3], L [B,S], delta [B].
    alpha_i = 1 - exp(-sigma_i delta); alpha'_i = alpha_i * min(L_i, 1);
    T_i = prod_{j<i} (1 - alpha'_j); w_i = T_i alpha'_i;
    C = sum_i w_i c_i + T_S bg;  A = 1 - T_S.  Returns C [B,3], A [B], w [B,S]."""
    alpha = 1.0 - torch.exp(-sigma * delta[:, None])
    a = alpha * torch.clamp(L, 0.0, 1.0)
    keep = torch.cumprod(1.0 - a, dim=1)                       # T_{i+1}
    Ti = torch.cat([torch.ones_like(keep[:, :1]), keep[:, :-1]], dim=1)
    w = Ti * a
    TS = keep[:, -1]
    C = (w[:, :, None] * rgb).sum(dim=1) + TS[:, None] * as64(bg)[None, :]
    return C, 1.0 - TS, w


# ---------------------------------------------------------------------------
# Whole path.
# ---------------------------------------------------------------------------

class Field:
    """Float64 view of one scene's learnable tensors (optionally requiring grad)."""

    def __init__(self, table, mlp_weights, logits, level_res, box_min, box_max, requires_grad=False):
        self.table = as64(table).clone().requires_grad_(requires_grad)
        self.mlp = [as64(w).clone().requires_grad_(requires_grad) for w in mlp_weights]
        self.logits = as64(logits).clone().requires_grad_(requires_grad)
        self.level_res = [int(n) for n in level_res]
        self.box_min = tuple(float(v) for v in box_min)
        self.box_max = tuple(float(v) for v in box_max)

    @classmethod
    def from_scene(cls, sc, requires_grad=False):
        return cls(sc.table, sc.mlp, sc.logits, sc.level_res, sc.box_min, sc.box_max, requires_grad)


def render_rays(field: Field, G: torch.Tensor, o: torch.Tensor, d: torch.Tensor, S: int,
                xi=None, bg=(0.0, 0.0, 0.0), chunk: int = 256, return_stats: bool = False, residual=None):
    """Render rays (o, d [B,3]) with S samples each.  xi: None (midpoints) or
    [B,S].  Missed rays give (bg, 0).  Returns RGBA [B,4].  residual: None,
    or a dict with the residual motion network (oracle/residual.py:
    "weights", "w_omega", "omega", "alpha"); the field is then queried at
    x_final = x_skel + x_res (Sec. 4.3, Eq. 12)."""
    G = as64(G)
    Wc = motion_weights(field.logits)
    B = d.shape[0]
    t_n, t_f, hit = ray_box(o, d, field.box_min, field.box_max)
    out = []
    n_eval = 0
    bgt = as64(bg)
    for s in range(0, B, chunk):
        sl = slice(s, min(B, s + chunk))
        h = hit[sl]
        rgba = torch.cat([bgt.expand(h.shape[0], 3), torch.zeros(h.shape[0], 1, dtype=F64)], 1)
        if bool(h.any()):
            idx = torch.nonzero(h)[:, 0]
            dd = d[sl][idx]
            xs = None if xi is None else as64(xi)[sl][idx]
            t, delta = sample_ts(t_n[sl][idx], t_f[sl][idx], S, xs)
            x = o[None, None, :] + t[:, :, None] * dd[:, None, :]
            nb = idx.shape[0]
            x_skel, L = inverse_lbs(x.reshape(-1, 3), G, Wc, field.box_min, field.box_max)
            if residual is not None:
                from .residual import residual_offset
                x_skel = x_skel + residual_offset(x_skel, residual["omega"], residual["weights"],
                                                  residual["w_omega"], residual["alpha"])
            if getattr(field, "encoding", "grid") == "freq":
                from .freq_field import freq_field
                rgb, sigma = freq_field(x_skel, field.mlp)
            else:
                feat = grid_encode(x_skel, field.table, field.level_res, field.box_min, field.box_max)
                rgb, sigma = mlp(feat, field.mlp)
            C, A, _ = composite(sigma.reshape(nb, S), rgb.reshape(nb, S, 3), L.reshape(nb, S), delta, bgt)
            rgba = rgba.index_put((idx,), torch.cat([C, A[:, None]], 1))
            n_eval += nb * S
        out.append(rgba)
    res = torch.cat(out, 0)
    if return_stats:
        return res, {"hit_rays": int(hit.sum()), "box_samples": n_eval}
    return res


def render_image(sc, field: Optional[Field] = None, pixel_ids=None, xi=None, bg=(0.0, 0.0, 0.0),
                 axis_angle=None, cam=None, return_stats=False, residual=None):
    """Render a scene (all pixels, or the listed pixel ids) -> RGBA [B,4].
    residual: None, or {"weights", "w_omega", "alpha"} of the residual motion
    network, conditioned on the rendered pose."""
    field = Field.from_scene(sc) if field is None else field
    aa = sc.axis_angle if axis_angle is None else axis_angle
    G = bone_transforms(sc.parents, sc.rest_joints, aa)
    o, d = camera_rays(sc.cam if cam is None else cam, sc.H, sc.W, pixel_ids)
    if residual is not None:
        residual = dict(residual, omega=aa)
    return render_rays(field, G, o, d, sc.spp, xi=xi, bg=bg, return_stats=return_stats, residual=residual)


def mse_loss(rgba: torch.Tensor, target) -> torch.Tensor:
    """Mean squared error over the RGB channels of a ray batch."""
    return ((rgba[:, :3] - as64(target)) ** 2).mean()
