"""Shared test helpers: run the GPU library and the oracle on the same scene."""
import numpy as np
import torch

import oracle
import scenes


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def gpu_render(sc, table_dtype=0, mlp_dtype=0, pixel_ids=None, ert_tau=1e-6, bg=(0.0, 0.0, 0.0),
               stratified=False, seed=0, axis_angle=None, cam=None, count=False):
    import paper_2306_16541_amd as m
    fld, _ = m.upload_scene(sc, "cuda", table_dtype, mlp_dtype)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle if axis_angle is None else axis_angle)
    c = m.make_camera(sc.cam if cam is None else cam, sc.box_min, sc.box_max)
    opts = m.make_opts(ert_tau=ert_tau, bg=bg, stratified=stratified, seed=seed)
    pid = None if pixel_ids is None else torch.as_tensor(np.asarray(pixel_ids, np.int32), device="cuda")
    counter = torch.zeros(1, dtype=torch.int64, device="cuda") if count else None
    out = m.render(fld, pose, c, sc.H, sc.W, sc.spp, opts, pid, counter=counter)
    torch.cuda.synchronize()
    if count:
        return out.cpu().numpy(), int(counter.item())
    return out.cpu().numpy()


def oracle_render(sc, pixel_ids=None, bg=(0.0, 0.0, 0.0), xi=None, axis_angle=None, cam=None, freq=None,
                  residual=None, alpha=4.0):
    """freq: W1..W5 of the frequency-encoded field instead of the scene's
    grid field; residual: (W1..W5, W_omega) of the residual motion network
    at window position alpha."""
    field = None
    if freq is not None:
        field = oracle.Field.from_scene(sc)
        field.encoding = "freq"
        field.mlp = [oracle.as64(w) for w in freq]
    res = None if residual is None else {"weights": residual[0], "w_omega": residual[1], "alpha": alpha}
    return oracle.render_image(sc, field=field, pixel_ids=pixel_ids, bg=bg, xi=xi, axis_angle=axis_angle, cam=cam,
                               residual=res).numpy()
