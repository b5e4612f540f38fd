"""GPU parity of the residual non-rigid motion network (Sec. 4.3, Eq. 11-12)
against the FP64 oracle.

The network runs on BF16 MFMA with FP32 accumulation (the mixed-precision
path), so the bar is the mixed path's: PSNR >= 45 dB against the oracle
evaluated on the FP32 master weights.  A zero output layer must leave the
render bitwise unchanged, and the residual must visibly move the image.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from helpers import psnr

pytestmark = pytest.mark.gpu


def _render(sc, tdt, mdt, res=None, pixel_ids=None, alpha=4.0):
    import paper_2306_16541_amd as m
    fld, _ = m.upload_scene(sc, "cuda", tdt, mdt)
    if res is not None:
        fld.set_residual(res[0], res[1], alpha)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    pid = None if pixel_ids is None else torch.as_tensor(np.asarray(pixel_ids, np.int32), device="cuda")
    out = m.render(fld, pose, m.make_camera(sc.cam), sc.H, sc.W, sc.spp, m.make_opts(), pid)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _oracle(sc, res, pixel_ids=None, alpha=4.0):
    return oracle.render_image(sc, pixel_ids=pixel_ids,
                               residual={"weights": res[0], "w_omega": res[1], "alpha": alpha}).numpy()


@pytest.mark.parametrize("tdt,alpha", [(1, 4.0), (0, 2.5), (1, 0.0)])
def test_residual_render_matches_oracle(tdt, alpha):
    sc = scenes.scene_body(H=48, W=64, spp=128)
    res = scenes.residual_weights(21)
    g = _render(sc, tdt, 2, res, alpha=alpha)
    o = _oracle(sc, res, alpha=alpha)
    plain = oracle.render_image(sc).numpy()
    moved = float(np.abs(o - plain).max())
    p = psnr(g[:, :3], o[:, :3])
    print(f"[residual tdt={tdt} alpha={alpha}] PSNR {p:.2f} dB, max-abs {np.abs(g - o).max():.3e}, "
          f"oracle moved by the residual {moved:.3e}", flush=True)
    assert moved > 1e-2
    assert p >= 45.0


def test_residual_ray_list_matches_oracle():
    sc = scenes.scene_body(H=40, W=56, spp=96)
    res = scenes.residual_weights(22)
    pid = np.random.default_rng(4).integers(0, sc.H * sc.W, 500)
    g = _render(sc, 1, 2, res, pixel_ids=pid)
    o = _oracle(sc, res, pixel_ids=pid)
    assert psnr(g[:, :3], o[:, :3]) >= 45.0


def test_zero_output_layer_is_bitwise_plain():
    sc = scenes.scene_body(H=32, W=48, spp=128)
    ws, w_omega = scenes.residual_weights(23)
    ws[4] = np.zeros_like(ws[4])
    a = _render(sc, 1, 2, (ws, w_omega))
    b = _render(sc, 1, 2, None)
    assert np.array_equal(a, b)


def test_residual_needs_the_bf16_path():
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=16, W=16, spp=32)
    with pytest.raises(m.MnrError, match="BF16"):
        _render(sc, 0, 0, scenes.residual_weights(24))
