"""Analytic teacher images for the learned-part test (test infrastructure).

A body of ellipsoids with one colour per bone, rigidly skinned: the
ellipsoid on the segment ending at joint j moves with its parent bone
(the root blob with the root).  A pixel shows the colour of the nearest
ellipsoid its ray hits (opacity 1) or the background (opacity 0).  This is
ray-quadric intersection, not volume rendering, so the targets are
independent of the renderer under test; bone transforms come from the
oracle's forward kinematics.
"""
import numpy as np

import scenes
from oracle import render as O


def render_teacher(parents, rest_joints, axis_angle, cam, H, W, colors, bg=(0.0, 0.0, 0.0)):
    """RGBA [H*W, 4] float32."""
    G = O.bone_transforms(parents, rest_joints, np.asarray(axis_angle, np.float64)).numpy()   # observed -> canonical
    o, d = (t.numpy() for t in O.camera_rays(cam, H, W))
    c, ax, half, rad = scenes.body_ellipsoids(scenes.BODY_THICKNESS)
    best = np.full(d.shape[0], np.inf)
    col = np.tile(np.asarray(bg, np.float64), (d.shape[0], 1))
    for k in range(c.shape[0]):
        bone = parents[k] if parents[k] >= 0 else 0
        R, t = G[bone, :, :3], G[bone, :, 3]
        oc = R @ o + t - c[k]                # ray origin in canonical space, relative to the centre
        dc = d @ R.T                         # directions [B,3]
        a = ax[k]                            # long axis (half-length half[k]); radius rad[k] across it
        oa, da = float(oc @ a), dc @ a
        op, dp = oc - oa * a, dc - np.outer(da, a)
        A = da ** 2 / half[k] ** 2 + np.einsum("ij,ij->i", dp, dp) / rad[k] ** 2
        B = 2 * (oa * da / half[k] ** 2 + (dp @ op) / rad[k] ** 2)
        Cc = oa ** 2 / half[k] ** 2 + float(op @ op) / rad[k] ** 2 - 1.0
        disc = B * B - 4 * A * Cc
        ok = disc >= 0
        tt = np.where(ok, (-B - np.sqrt(np.where(ok, disc, 0))) / (2 * A), np.inf)
        tt = np.where(tt > 0, tt, np.inf)
        closer = tt < best
        best = np.where(closer, tt, best)
        col[closer] = colors[k]
    alpha = np.isfinite(best).astype(np.float64)
    return np.concatenate([col, alpha[:, None]], 1).astype(np.float32)
