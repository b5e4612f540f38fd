"""Seeded synthetic inputs for the posed-body renderer.

This module only draws and lays out input data: a 24-joint body skeleton,
joint rotations, motion-weight logits, grid-encoding tables, MLP weights,
cameras, training ray batches and an ellipsoid body used to seed a density
field.  It computes none of the renderer's arithmetic (no forward
kinematics, skinning, encoding, MLP or compositing); both the GPU library
and the CPU oracle read what it returns as plain arrays.

The paper evaluates on a captured human-motion dataset at 1024x1024 with
128 samples per ray (Sec. 5.1, Sec. 5.2 "Training").  These synthetic
scenes stand in for it: same resolutions and samples per ray, a 24-joint
SMPL-like tree, and tensors drawn from fixed seeds.  No dataset item is
reproduced.

Layouts (shared by both sides, documented in include/metanerf.h):
  * motion logits / weights: float32 [n_bones + 1][R][R][R], channel-major,
    voxel (ix, iy, iz) at flat offset ix + R*(iy + R*iz); channel n_bones is
    the background channel.
  * grid table: [n_levels][T][n_feat], feature fastest.
  * MLP layer k: float32 [out][in], row-major, no bias.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

N_JOINTS = 24
N_LEVELS = 16
N_FEAT = 2
# Per-level grid resolutions floor(16 * 2**(l/3)), l = 0..15 (growth factor
# 32**(1/15) = 2**(1/3) from 16 to 512), written out as integers so that no
# side ever recomputes them in floating point.
LEVEL_RES = (16, 20, 25, 32, 40, 50, 64, 80, 101, 128, 161, 203, 256, 322, 406, 512)
BOX_MIN = (-0.5, -0.5, -0.5)
BOX_MAX = (0.5, 0.5, 0.5)

# SMPL-like joint tree: parents precede children.
PARENTS = (-1, 0, 0, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 9, 9, 12, 13, 14, 16, 17, 18, 19, 20, 21)
JOINT_NAMES = (
    "pelvis", "l_hip", "r_hip", "spine1", "l_knee", "r_knee", "spine2", "l_ankle",
    "r_ankle", "spine3", "l_foot", "r_foot", "neck", "l_collar", "r_collar", "head",
    "l_shoulder", "r_shoulder", "l_elbow", "r_elbow", "l_wrist", "r_wrist", "l_hand", "r_hand",
)
# Rest (canonical) joint positions: a T-pose inside the unit box, y up,
# pelvis at the origin.
REST_JOINTS = (
    (0.00, 0.00, 0.00), (0.06, -0.05, 0.00), (-0.06, -0.05, 0.00), (0.00, 0.06, -0.01),
    (0.07, -0.24, 0.01), (-0.07, -0.24, 0.01), (0.00, 0.13, -0.01), (0.07, -0.43, -0.01),
    (-0.07, -0.43, -0.01), (0.00, 0.19, -0.01), (0.07, -0.46, 0.06), (-0.07, -0.46, 0.06),
    (0.00, 0.30, -0.01), (0.04, 0.26, -0.01), (-0.04, 0.26, -0.01), (0.00, 0.38, 0.01),
    (0.10, 0.26, -0.01), (-0.10, 0.26, -0.01), (0.22, 0.26, -0.01), (-0.22, 0.26, -0.01),
    (0.34, 0.26, -0.01), (-0.34, 0.26, -0.01), (0.42, 0.26, -0.01), (-0.42, 0.26, -0.01),
)
# Half-thickness of the ellipsoid on the segment ending at each joint; the
# root's entry is the pelvis ellipsoid.
SEGMENT_RADIUS = (
    0.085, 0.06, 0.06, 0.09, 0.05, 0.05, 0.095, 0.04, 0.04, 0.10, 0.03, 0.03,
    0.04, 0.05, 0.05, 0.07, 0.05, 0.05, 0.035, 0.035, 0.03, 0.03, 0.03, 0.03,
)

# Tensor ids for per-tensor seed streams.
_TID_POSE, _TID_LOGITS, _TID_TABLE, _TID_MLP, _TID_RAYS, _TID_TARGET, _TID_COLOR, _TID_RES, _TID_CNN, _TID_FREQ = \
    range(1, 11)


def rng(seed: int, tensor_id: int) -> np.random.Generator:
    """Independent, reproducible stream per (master seed, tensor id)."""
    return np.random.default_rng(np.random.SeedSequence([int(seed) & 0xFFFFFFFF, int(tensor_id)]))


def dense_level_count(log2_T: int, level_res=LEVEL_RES) -> int:
    """Number of leading levels whose (N+1)^3 vertices fit in T entries."""
    T = 1 << log2_T
    return sum(1 for n in level_res if (n + 1) ** 3 <= T)


@dataclasses.dataclass
class Camera:
    """OpenCV pinhole: x_cam = R_wc @ X + T; pixel (u, v) has centre (u+0.5, v+0.5)."""
    fx: float
    fy: float
    cx: float
    cy: float
    R_wc: np.ndarray  # float32 [3, 3]
    T: np.ndarray     # float32 [3]


def camera(H: int, W: int, yaw_quarter_turns: int = 0, yaw: Optional[float] = None,
           distance: float = 3.0) -> Camera:
    """Camera on a circle of radius `distance` around the y axis, looking at
    the origin.  yaw=0 puts it at (0, 0, distance) looking down -z.  Quarter
    turns are built from exact integer matrices so that a 90-degree yaw is
    exact in float32."""
    base = np.diag([1.0, -1.0, -1.0])
    if yaw is None:
        c, s = [(1, 0), (0, 1), (-1, 0), (0, -1)][yaw_quarter_turns % 4]
    else:
        c, s = math.cos(yaw), math.sin(yaw)
    Ry = np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])
    R_wc = base @ Ry.T
    centre = Ry @ np.array([0.0, 0.0, distance])
    T = -R_wc @ centre
    return Camera(fx=2.0 * W, fy=2.0 * H, cx=W / 2.0, cy=H / 2.0,
                  R_wc=R_wc.astype(np.float32), T=T.astype(np.float32))


@dataclasses.dataclass
class Scene:
    name: str
    H: int
    W: int
    spp: int
    parents: np.ndarray       # int32 [J]
    rest_joints: np.ndarray   # float32 [J, 3]
    axis_angle: np.ndarray    # float32 [J, 3]
    res: int                  # motion-volume resolution R
    logits: np.ndarray        # float32 [J+1, R, R, R]
    level_res: np.ndarray     # int32 [L]
    log2_T: int
    table: np.ndarray         # float32 [L, T, F]
    mlp: List[np.ndarray]     # float32 [out, in] per layer
    cam: Camera
    box_min: tuple = BOX_MIN
    box_max: tuple = BOX_MAX
    seed: int = 0

    @property
    def n_bones(self) -> int:
        return int(self.parents.shape[0])

    @property
    def nominal_samples(self) -> int:
        return self.H * self.W * self.spp


def skeleton():
    return (np.array(PARENTS, dtype=np.int32), np.array(REST_JOINTS, dtype=np.float32))


def pose(seed: int, std: float, n_joints: int = N_JOINTS, tensor_id: int = _TID_POSE) -> np.ndarray:
    """Axis-angle rotations, each component ~ N(0, std^2) radians."""
    return (rng(seed, tensor_id).standard_normal((n_joints, 3)) * std).astype(np.float32)


def motion_logits(seed: int, res: int, n_channels: int = N_JOINTS + 1) -> np.ndarray:
    """Motion-weight volume logits ~ N(0, 1), [C][R][R][R]."""
    return rng(seed, _TID_LOGITS).standard_normal((n_channels, res, res, res)).astype(np.float32)


def grid_table(seed: int, log2_T: int, n_levels: int = N_LEVELS, n_feat: int = N_FEAT,
               scale: float = 0.1) -> np.ndarray:
    """Grid-encoding table ~ U(-scale, scale), [L][T][F]."""
    T = 1 << log2_T
    return rng(seed, _TID_TABLE).uniform(-scale, scale, (n_levels, T, n_feat)).astype(np.float32)


def mlp_weights(seed: int, widths) -> List[np.ndarray]:
    """Xavier-uniform (Glorot & Bengio 2010) weights, bound sqrt(6/(fan_in+fan_out))."""
    g = rng(seed, _TID_MLP)
    out = []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        out.append(g.uniform(-a, a, (fan_out, fan_in)).astype(np.float32))
    return out


RES_SHAPES = ((64, 32), (64, 64), (64, 64), (64, 96), (3, 64))   # residual motion network W1..W5 [out, in]


def residual_weights(seed: int, out_scale: float = 0.05, n_joints: int = N_JOINTS):
    """Seeded weights of the residual motion network: W1..W5 in RES_SHAPES
    and W_omega [64, 3 n_joints], Xavier-uniform; the output layer W5 is
    scaled by out_scale so that offsets stay a few hundredths of the box."""
    g = rng(seed, _TID_RES)
    ws = []
    for fan_out, fan_in in RES_SHAPES + ((64, 3 * n_joints),):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        ws.append(g.uniform(-a, a, (fan_out, fan_in)).astype(np.float32))
    ws[4] *= np.float32(out_scale)
    return ws[:5], ws[5]


FREQ_SHAPES = ((64, 64), (64, 64), (64, 64), (64, 128), (4, 64))   # the frequency-encoded field's W1..W5


def freq_field_weights(seed: int, sigma_gain: float = 30.0):
    """Seeded Xavier-uniform weights of the frequency-encoded field's skip
    MLP; the density row of W5 is scaled by sigma_gain so that the random
    field is a fog of moderate opacity (sigma up to a few tens)."""
    g = rng(seed, _TID_FREQ)
    ws = []
    for fan_out, fan_in in FREQ_SHAPES:
        a = math.sqrt(6.0 / (fan_in + fan_out))
        ws.append(g.uniform(-a, a, (fan_out, fan_in)).astype(np.float32))
    ws[4][3] *= np.float32(sigma_gain)
    return ws


SKEL_CNN_CHANNELS = (256, 128, 64, 32, 32, 25)


def skel_cnn_weights(seed: int, channels=SKEL_CNN_CHANNELS, latent: int = 256):
    """Seeded latent z ~ N(0, 1) and weights of the skeleton-motion CNN:
    w_fc [c0, latent] and w[k] [c_k, c_{k+1}, 4, 4, 4], uniform with bound
    sqrt(6 / fan_in) (a transposed-convolution output sums 8 taps per input
    channel)."""
    g = rng(seed, _TID_CNN)
    z = g.standard_normal(latent).astype(np.float32)
    w_fc = g.uniform(-1, 1, (channels[0], latent)).astype(np.float32) * np.float32(math.sqrt(6.0 / latent))
    ws = []
    for k in range(5):
        a = math.sqrt(6.0 / (8 * channels[k]))
        ws.append(g.uniform(-a, a, (channels[k], channels[k + 1], 4, 4, 4)).astype(np.float32))
    return z, w_fc, ws


# ---------------------------------------------------------------------------
# Ellipsoid body used to seed a density field in canonical space.
# ---------------------------------------------------------------------------

def body_ellipsoids(thickness: float = 1.0):
    """One ellipsoid per joint: the segment parent->joint (pelvis: a blob at
    the root).  Returns centres [J,3], unit long axes [J,3], half-lengths [J],
    radii [J] (float64)."""
    parents, J = PARENTS, np.array(REST_JOINTS, dtype=np.float64)
    centres, axes, half, rad = [], [], [], []
    for j, p in enumerate(parents):
        r = SEGMENT_RADIUS[j] * thickness
        if p < 0:
            centres.append(J[j]); axes.append(np.array([1.0, 0.0, 0.0]))
            half.append(1.2 * r); rad.append(0.8 * r)
        else:
            seg = J[j] - J[p]
            L = float(np.linalg.norm(seg))
            centres.append(0.5 * (J[j] + J[p])); axes.append(seg / L)
            half.append(0.5 * L + 0.5 * r); rad.append(r)
    return np.array(centres), np.array(axes), np.array(half), np.array(rad)


def inside_body(points: np.ndarray, thickness: float = 1.0) -> np.ndarray:
    """Boolean occupancy of canonical points [N,3] in the union of ellipsoids."""
    c, a, h, r = body_ellipsoids(thickness)
    occ = np.zeros(points.shape[0], dtype=bool)
    for k in range(c.shape[0]):
        v = points - c[k]
        along = v @ a[k]
        perp2 = np.einsum("ij,ij->i", v, v) - along * along
        occ |= (along / h[k]) ** 2 + perp2 / r[k] ** 2 <= 1.0
    return occ


def seed_density(table: np.ndarray, log2_T: int, level_res=LEVEL_RES, thickness: float = 1.0,
                 amplitude: float = 1.0, box_min=BOX_MIN, box_max=BOX_MAX) -> int:
    """Overwrite feature 0 of every dense level with amplitude * occupancy of
    the level's vertices (in place).  A dense level stores vertex
    (ix, iy, iz) of its (N+1)^3 lattice at entry ix + (N+1)*(iy + (N+1)*iz),
    the storage convention of the grid table.  Returns the dense level count."""
    nd = dense_level_count(log2_T, level_res)
    bmin, bmax = np.array(box_min, dtype=np.float64), np.array(box_max, dtype=np.float64)
    for l in range(nd):
        n = int(level_res[l])
        g = np.arange(n + 1, dtype=np.float64) / n
        iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
        pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1) * (bmax - bmin) + bmin
        table[l, : (n + 1) ** 3, 0] = amplitude * inside_body(pts, thickness).astype(np.float32)
    return nd


def density_mlp(weights: List[np.ndarray], n_dense: int, gain: float) -> None:
    """Reserve hidden unit 0 of every layer as a density pass-through (in place):
    layer 1 row 0 sums feature 0 of the dense levels times `gain`; later
    hidden rows 0 copy unit 0; unit 0 feeds no other unit; the output's
    density row copies unit 0."""
    first = weights[0]
    first[0, :] = 0.0
    for l in range(n_dense):
        first[0, 2 * l] = gain
    for w in weights[1:-1]:
        w[:, 0] = 0.0
        w[0, :] = 0.0
        w[0, 0] = 1.0
    last = weights[-1]
    last[:, 0] = 0.0
    last[3, :] = 0.0
    last[3, 0] = 1.0


# ---------------------------------------------------------------------------
# Workloads.
# ---------------------------------------------------------------------------

# Occupancy thickness and density gain of the seeded body (see the design doc for
# how they were chosen: about 30% of rays reach opacity > 0.5).
BODY_THICKNESS = 2.55
SIGMA_INSIDE = 100.0


def scene_small(seed: int = 16541 + 1, H: int = 64, W: int = 64, spp: int = 64) -> Scene:
    """64x64, 64 samples/ray, 32^3 motion volume, T = 2^14, MLP 32-64-64-4."""
    parents, rest = skeleton()
    return Scene(
        name=f"posed-body {H}x{W} S={spp} fp32 (R=32, T=2^14, MLP 32-64-64-4)",
        H=H, W=W, spp=spp, parents=parents, rest_joints=rest,
        axis_angle=pose(seed, 0.2), res=32, logits=motion_logits(seed, 32),
        level_res=np.array(LEVEL_RES, dtype=np.int32), log2_T=14,
        table=grid_table(seed, 14), mlp=mlp_weights(seed, (32, 64, 64, 4)),
        cam=camera(H, W), seed=seed)


def scene_body(seed: int = 16541 + 2, H: int = 512, W: int = 512, spp: int = 128,
               res: int = 64, log2_T: int = 19, pose_std: float = 0.2,
               sigma_inside: float = None, thickness: float = None) -> Scene:
    """The seeded-body scene: 24-joint skeleton, R^3 x 25 motion volume,
    16-level grid with T = 2^log2_T, MLP 32-64-64-64-4, with a density unit
    that is large inside a union of 24 ellipsoids."""
    sigma_inside = SIGMA_INSIDE if sigma_inside is None else sigma_inside
    thickness = BODY_THICKNESS if thickness is None else thickness
    parents, rest = skeleton()
    table = grid_table(seed, log2_T)
    nd = seed_density(table, log2_T, thickness=thickness)
    if nd == 0:
        raise ValueError("the seeded body needs at least one dense grid level (T >= 17^3)")
    mlp = mlp_weights(seed, (32, 64, 64, 64, 4))
    density_mlp(mlp, nd, sigma_inside / nd)
    return Scene(
        name=f"posed-body {H}x{W} S={spp} (R={res}, T=2^{log2_T}, MLP 32-64-64-64-4, seeded body)",
        H=H, W=W, spp=spp, parents=parents, rest_joints=rest,
        axis_angle=pose(seed, pose_std), res=res, logits=motion_logits(seed, res),
        level_res=np.array(LEVEL_RES, dtype=np.int32), log2_T=log2_T,
        table=table, mlp=mlp, cam=camera(H, W), seed=seed)


def train_batch(seed: int, H: int, W: int, n_rays: int):
    """Random pixel ids (uniform over the image) and U(0,1) RGB targets."""
    pix = rng(seed, _TID_RAYS).integers(0, H * W, n_rays).astype(np.int32)
    tgt = rng(seed, _TID_TARGET).uniform(0.0, 1.0, (n_rays, 3)).astype(np.float32)
    return pix, tgt


def bone_colors(seed: int, n: int = N_JOINTS) -> np.ndarray:
    return rng(seed, _TID_COLOR).uniform(0.15, 0.95, (n, 3))
