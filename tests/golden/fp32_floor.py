"""FP32 noise floor of the seeded-body scene, measured with the FP64 oracle.

Writes tests/golden/fp32_floor.json.  Run from the repository root:

    python tests/golden/fp32_floor.py

Every float32 input the renderer reads (grid table, MLP weights, blend-weight
logits, joint rotations, rest joints, camera rotation and translation) is
moved by one float32 ulp up or down (a seeded random sign per element), and
the frame is rendered again in float64.  The change of each pixel measures
how far one float32 rounding of those quantities moves it: the FP32 kernels
round the ray origin and direction and every sample position once, so the
camera row is the part of their error that no float32 implementation avoids.
The scene's density gain inside the body (sigma_inside) sets how sharply the
body's edge responds to a shifted sample, so the floor is measured at two
gains.

The inputs are perturbed in groups (the field's parameters, the pose, the
camera, and all of them at once), so that the floor can be traced to its
source.  Pixels: every 8th pixel id of the 512 x 512 frame (32,768 rays, 128
samples each).  Only oracle/ and the scene generator are used.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp32_floor.json")
SIGMAS = (100.0, 300.0)
PERTURB_SEED = 20230628
PIXEL_STRIDE = 8
N_WORST = 6


def _ulp_step(a: np.ndarray, g: np.random.Generator) -> np.ndarray:
    a = np.asarray(a, np.float32)
    up = g.integers(0, 2, a.shape).astype(bool)
    return np.where(up, np.nextafter(a, np.float32(np.inf)), np.nextafter(a, np.float32(-np.inf))).astype(np.float32)


GROUPS = {
    "field": ("table", "mlp", "logits"),          # grid table, MLP weights, blend-weight logits
    "pose": ("axis_angle", "rest_joints"),        # joint rotations and rest joints (through FK)
    "camera": ("R_wc", "T"),                      # camera rotation and translation (the rays)
}
GROUPS["all"] = GROUPS["field"] + GROUPS["pose"] + GROUPS["camera"]


def perturbed(sc, names):
    """A copy of scene `sc` whose float32 inputs listed in `names` are each
    one ulp away (a seeded random direction per element, drawn in a fixed
    order so that every group sees the same steps for the same input)."""
    import copy
    g = np.random.default_rng(PERTURB_SEED)
    p = copy.copy(sc)
    cam = copy.copy(sc.cam)
    p.cam = cam
    steps = {
        "table": lambda: _ulp_step(sc.table, g),
        "mlp": lambda: [_ulp_step(w, g) for w in sc.mlp],
        "logits": lambda: _ulp_step(sc.logits, g),
        "axis_angle": lambda: _ulp_step(sc.axis_angle, g),
        "rest_joints": lambda: _ulp_step(sc.rest_joints, g),
        "R_wc": lambda: _ulp_step(sc.cam.R_wc, g),
        "T": lambda: _ulp_step(sc.cam.T, g),
    }
    for name, make in steps.items():     # always draw, keep only the listed ones
        v = make()
        if name in names:
            if name in ("R_wc", "T"):
                setattr(cam, name, v)
            else:
                setattr(p, name, v)
    return p


def floor_at(sigma: float, pixel_ids: np.ndarray, groups=tuple(GROUPS)):
    """Per group: per-pixel max over RGBA of |render(inputs) - render(inputs
    one ulp away)|."""
    import oracle
    import scenes
    sc = scenes.scene_body(sigma_inside=sigma)
    a = oracle.render_image(sc, pixel_ids=pixel_ids).numpy()
    out = {}
    for gname in groups:
        b = oracle.render_image(perturbed(sc, GROUPS[gname]), pixel_ids=pixel_ids).numpy()
        out[gname] = np.abs(a - b).max(axis=1)
    return out


def main():
    import scenes
    sc = scenes.scene_body()
    pid = np.arange(0, sc.H * sc.W, PIXEL_STRIDE)
    out = {"scene": "scenes.scene_body() (512x512, 128 samples/ray, T=2^19, R=64)",
           "pixels": f"every {PIXEL_STRIDE}th pixel id ({pid.size} rays)",
           "perturbation_seed": PERTURB_SEED, "groups": {k: list(v) for k, v in GROUPS.items()},
           "sigma_inside": {}}
    for s in SIGMAS:
        t0 = time.time()
        res = {}
        for gname, d in floor_at(s, pid).items():
            order = np.argsort(-d)[:N_WORST]
            res[gname] = {"max": float(d.max()), "p99_9": float(np.quantile(d, 0.999)), "mean": float(d.mean()),
                          "worst": [[int(pid[k]), float(d[k])] for k in order]}
            print(f"sigma_inside={s:g} {gname:7s}: max {d.max():.3e}, p99.9 {np.quantile(d, 0.999):.3e}", flush=True)
        out["sigma_inside"][str(int(s))] = res
        print(f"({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
