"""mnr_render_noalloc (library-owned work-queue counters, no workspace,
nothing allocated) against mnr_render with a caller workspace, through the
C ABI: two calls in a row on one stream, the second on a smaller frame, then
a ray list.  The forward pass has no atomics and a fixed sample-to-lane
mapping, so the two entry points must agree bit for bit."""
import numpy as np
import pytest
import torch

import scenes
from helpers import oracle_render

pytestmark = pytest.mark.gpu


def _setup(sc):
    import paper_2306_16541_amd as m
    fld, _ = m.upload_scene(sc, "cuda")
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam, sc.box_min, sc.box_max)
    return m, fld, pose, cam


def test_noalloc_matches_render_with_workspace_on_consecutive_calls():
    big = scenes.scene_body(H=96, W=80, spp=96, res=32, log2_T=16)
    small = scenes.scene_body(H=40, W=24, spp=64, res=32, log2_T=16)
    outs = []
    for sc in (big, small):
        m, fld, pose, cam = _setup(sc)
        ref = m.render(fld, pose, cam, sc.H, sc.W, sc.spp)
        got = m.render_noalloc(fld, pose, cam, sc.H, sc.W, sc.spp)
        torch.cuda.synchronize()
        outs.append((sc, ref.cpu().numpy(), got.cpu().numpy()))
    for sc, ref, got in outs:
        print(f"noalloc {sc.H}x{sc.W}x{sc.spp}: max |noalloc - render| = {np.abs(got - ref).max():.3e}", flush=True)
        np.testing.assert_array_equal(got, ref)
    sc, _, got = outs[1]
    assert np.abs(got - oracle_render(sc)).max() <= 1e-5


def test_noalloc_ray_list_and_repeat():
    sc = scenes.scene_body(H=64, W=64, spp=128, res=32, log2_T=16)
    m, fld, pose, cam = _setup(sc)
    g = np.random.default_rng(3)
    for n in (1500, 300):
        pid = torch.as_tensor(g.integers(0, sc.H * sc.W, n).astype(np.int32), device="cuda")
        ref = m.render(fld, pose, cam, sc.H, sc.W, sc.spp, pixel_ids=pid)
        a = m.render_noalloc(fld, pose, cam, sc.H, sc.W, sc.spp, pixel_ids=pid)
        b = m.render_noalloc(fld, pose, cam, sc.H, sc.W, sc.spp, pixel_ids=pid)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a.cpu().numpy(), ref.cpu().numpy())
        np.testing.assert_array_equal(b.cpu().numpy(), ref.cpu().numpy())
