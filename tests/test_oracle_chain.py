"""More pins of the FP64 oracle (CPU only): the whole ray chain against the
uniform-density closed form, the camera's pixel mapping on a non-square
image, the blend-weight softmax axis, and where the skeleton CNN's
activations sit.

Each test names the mistake in the oracle that it catches.
"""
import math

import numpy as np
import torch
import torch.nn.functional as F

import scenes
from oracle import render as O
from oracle.skel_cnn import SLOPE, skel_cnn_logits

F64 = torch.float64


# ------------------------------------------------ camera (Sec. 2.1) --------

def test_camera_pixel_mapping_on_a_non_square_image():
    # 3 rows x 5 columns, cx != cy, fx != fy and a rotation that is not
    # symmetric, so swapping u and v, cx and cy, fx and fy, or R and R^T all
    # change the corner rays.  Values below are worked out by hand:
    # pixel id = v * W + u; d_cam = ((u + .5 - cx)/fx, (v + .5 - cy)/fy, 1);
    # d = R^T d_cam with R = [[0,-1,0],[1,0,0],[0,0,1]] gives
    # (d_cam_y, -d_cam_x, d_cam_z); o = -R^T T.
    cam = scenes.Camera(fx=2.0, fy=3.0, cx=2.0, cy=1.25,
                        R_wc=np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.float32),
                        T=np.array([0.1, -0.2, 3.0], np.float32))
    o, d = O.camera_rays(cam, 3, 5, [0, 4, 10, 14, 7])
    np.testing.assert_allclose(o.numpy(), [0.2, 0.1, -3.0], rtol=1e-7)
    want = {
        0: (-0.25, 0.75, 1.0),               # u=0, v=0: d_cam = (-0.75, -0.25, 1)
        4: (-0.25, -1.25, 1.0),              # u=4, v=0: d_cam = ( 1.25, -0.25, 1)
        10: (1.25 / 3, 0.75, 1.0),           # u=0, v=2: d_cam = (-0.75, 5/12, 1)
        14: (1.25 / 3, -1.25, 1.0),          # u=4, v=2: d_cam = ( 1.25, 5/12, 1)
        7: (0.25 / 3, -0.25, 1.0),           # u=2, v=1: d_cam = ( 0.25, 1/12, 1)
    }
    for row, pid in enumerate([0, 4, 10, 14, 7]):
        e = np.array(want[pid])
        np.testing.assert_allclose(d[row].numpy(), e / np.linalg.norm(e), atol=1e-15)


# --------------------------------------------- samples (Sec. 4.4) ----------

def test_sample_positions_by_hand():
    # t_n = 1, t_f = 3, S = 4: stratum width 0.5, midpoints 1.25 .. 2.75;
    # a jitter xi moves sample i to 1 + (i + xi) * 0.5.
    t, delta = O.sample_ts(torch.tensor([1.0], dtype=F64), torch.tensor([3.0], dtype=F64), 4)
    np.testing.assert_array_equal(t.numpy(), [[1.25, 1.75, 2.25, 2.75]])
    assert float(delta[0]) == 0.5
    t, _ = O.sample_ts(torch.tensor([1.0], dtype=F64), torch.tensor([3.0], dtype=F64), 4,
                       np.array([[0.0, 0.25, 0.5, 0.999]]))
    np.testing.assert_allclose(t.numpy(), [[1.0, 1.625, 2.25, 2.9995]], atol=1e-15)


def _chord_by_bisection(o, d, lo=-0.5, hi=0.5):
    """Length of the segment of the ray o + t d (t >= 0) inside the box
    [lo, hi]^3, found from the point-in-box test alone: scan for an inside
    point, then bisect both crossings to full precision."""
    inside = lambda t: bool(np.all((o + t * d >= lo) & (o + t * d <= hi)))
    ts = np.linspace(0.0, 8.0, 200001)
    pts = o[None, :] + ts[:, None] * d[None, :]
    ins = ts[np.all((pts >= lo) & (pts <= hi), axis=1)]
    if ins.size == 0:
        return 0.0
    step = ts[1] - ts[0]
    def cross(a, b):                      # inside(a) != inside(b)
        ia = inside(a)
        for _ in range(200):
            m = 0.5 * (a + b)
            if inside(m) == ia:
                a = m
            else:
                b = m
        return 0.5 * (a + b)
    t_in = 0.0 if inside(0.0) else cross(ins[0], ins[0] - step)
    t_out = cross(ins[-1], ins[-1] + step)
    return t_out - t_in


def _uniform_scene(H, W, S, sigma, colour_logit, yaw):
    """Identity pose, a background logit of -1e3 (so the bone weights sum to
    1 at every voxel and L = 1 in the box), a constant grid table and an MLP
    whose output is the same for every sample: sigma and sigmoid(colour_logit)."""
    parents, rest = scenes.skeleton()
    R, L_, T, Fe = 8, 16, 2 ** 10, 2
    logits = np.zeros((25, R, R, R), np.float32)
    logits[24] = -1e3
    table = np.full((L_, T, Fe), 0.25, np.float32)
    w1 = np.full((4, 32), 1.0 / 8.0)                 # every hidden unit = 32 * 0.25 / 8 = 1
    w2 = np.zeros((4, 4))
    w2[:3] = np.asarray(colour_logit)[:, None] / 4.0
    w2[3] = sigma / 4.0
    return scenes.Scene(name="uniform", H=H, W=W, spp=S, parents=parents, rest_joints=rest,
                        axis_angle=np.zeros((24, 3), np.float32), res=R, logits=logits,
                        level_res=np.array(scenes.LEVEL_RES, np.int32), log2_T=10, table=table,
                        mlp=[w1, w2], cam=scenes.camera(H, W, yaw=yaw))


def test_render_uniform_density_equals_closed_form_over_the_box_chord():
    # Uniform sigma over the chord Lc that a ray cuts from the body box gives
    # opacity 1 - exp(-sigma Lc) (Sec. 2.1, Eq. 2 and 3), whatever S is.  The
    # chain camera -> slab clip -> sample widths -> warp -> encode -> MLP ->
    # composite must reproduce it; the chord comes from bisection on the
    # point-in-box test, not from the oracle's slab clip.  A wrong stratum
    # width (chord / (S - 1)), a clip that loses t_near or the likelihood
    # factor applied where L = 1 all break it.
    H, W, sigma = 6, 9, 2.3
    colour_logit = np.array([0.4, -1.1, 2.0])
    pix = np.arange(H * W)
    for S, yaw in ((1, 0.0), (5, 0.4), (64, -1.0)):
        sc = _uniform_scene(H, W, S, sigma, colour_logit, yaw)
        # fx = 2W puts the image corners outside the box; widen the view so
        # some rays miss and some clip a box edge
        sc.cam.fx, sc.cam.fy = 0.6 * W, 0.6 * H
        rgba = O.render_image(sc, pixel_ids=pix).numpy()
        o, d = O.camera_rays(sc.cam, H, W, pix)
        on, dn = o.numpy(), d.numpy()
        n_hit = 0
        for k in range(pix.shape[0]):
            Lc = _chord_by_bisection(on, dn[k])
            A = 1.0 - math.exp(-sigma * Lc)
            assert abs(rgba[k, 3] - A) < 1e-12, (S, yaw, k, rgba[k, 3], A)
            c = 1.0 / (1.0 + np.exp(-colour_logit))
            np.testing.assert_allclose(rgba[k, :3], c * A, atol=1e-12)
            n_hit += Lc > 0
        assert 0 < n_hit < pix.shape[0]              # some rays miss, some hit


# ----------------------------------------- blend weights (Sec. 4.2) --------

def test_motion_weights_softmax_is_over_channels_at_each_voxel():
    # Two channels on a 2^3 grid with a different logit pair at every voxel:
    # W_0 = 1 / (1 + exp(b - a)) at each voxel, and the channels sum to 1.
    # A softmax over a spatial axis gives other values and other sums.
    g = np.random.default_rng(3)
    lg = g.normal(0, 2, (2, 2, 2, 2))
    w = O.motion_weights(lg).numpy()
    for z in range(2):
        for y in range(2):
            for x in range(2):
                a, b = lg[0, z, y, x], lg[1, z, y, x]
                assert abs(w[0, z, y, x] - 1.0 / (1.0 + math.exp(b - a))) < 1e-15
                assert abs(w[1, z, y, x] - 1.0 / (1.0 + math.exp(a - b))) < 1e-15
    w25 = O.motion_weights(scenes.motion_logits(9, 6)).numpy()
    np.testing.assert_allclose(w25.sum(axis=0), 1.0, atol=1e-14)
    assert w25.min() > 0.0


def test_identity_pose_likelihood_is_one_minus_background_weight():
    # With G_i = I every bone samples the same point, so
    # L = sum_{i<24} W_i(x) = 1 - W_bg(x) by the partition of unity; taking the
    # wrong channel as background, or summing all 25, breaks it.
    g = np.random.default_rng(4)
    lg = scenes.motion_logits(11, 10)
    Wc = O.motion_weights(lg)
    x = torch.as_tensor(g.uniform(-0.5, 0.5, (400, 3)))
    G = torch.cat([torch.eye(3, dtype=F64).expand(24, 3, 3), torch.zeros(24, 3, 1, dtype=F64)], 2)
    _, L = O.inverse_lbs(x, G, Wc, (-0.5,) * 3, (0.5,) * 3)
    q = (x + 0.5) * 9.0
    bg = O.trilinear_zero_padded(Wc, torch.full((400,), 24, dtype=torch.int64), q)
    np.testing.assert_allclose(L.numpy(), 1.0 - bg.numpy(), atol=1e-14)


# ----------------------------------------- skeleton CNN (Fig. 7) -----------

def _tconv_loop(x, w):
    """Transposed convolution (kernel 4, stride 2, padding 1) by definition:
    input voxel v adds w[i, o, k] x[i, v] to output voxel 2 v - 1 + k per axis."""
    ci, D = x.shape[0], x.shape[1]
    out = np.zeros((w.shape[1], 2 * D, 2 * D, 2 * D))
    for i in range(ci):
        for vz in range(D):
            for vy in range(D):
                for vx in range(D):
                    for kz in range(4):
                        for ky in range(4):
                            for kx in range(4):
                                oz, oy, ox = 2 * vz - 1 + kz, 2 * vy - 1 + ky, 2 * vx - 1 + kx
                                if 0 <= oz < 2 * D and 0 <= oy < 2 * D and 0 <= ox < 2 * D:
                                    out[:, oz, oy, ox] += w[i, :, kz, ky, kx] * x[i, vz, vy, vx]
    return out


def _lrelu(v):
    return np.where(v > 0, v, SLOPE * v)


def test_two_convolutions_by_hand_fix_the_activation_positions():
    # FC -> LeakyReLU -> conv -> LeakyReLU -> conv (no activation after the
    # last).  The first convolution of a single voxel is the kernel's centre
    # 2^3 taps times the FC output; the second follows the definition loop.
    # Mixed signs everywhere, so a missing, extra or misplaced LeakyReLU (or a
    # wrong slope) changes the result.
    g = np.random.default_rng(12)
    z = g.standard_normal(6)
    w_fc = g.standard_normal((2, 6))
    w1 = g.standard_normal((2, 3, 4, 4, 4))
    w2 = g.standard_normal((3, 2, 4, 4, 4))
    a = _lrelu(w_fc @ z)                                       # [2]
    h1 = np.einsum("i,iozyx->ozyx", a, w1[:, :, 1:3, 1:3, 1:3])
    assert (h1 < 0).any() and (h1 > 0).any()
    want = _tconv_loop(_lrelu(h1), w2)
    assert (want < 0).any() and (want > 0).any()
    got = skel_cnn_logits(z, w_fc, [w1, w2]).numpy()
    np.testing.assert_allclose(got, want, atol=1e-12)
    # the same through torch's operator, as a check of the loop itself
    t = F.conv_transpose3d(torch.as_tensor(_lrelu(h1))[None], torch.as_tensor(w2), stride=2, padding=1)[0]
    np.testing.assert_allclose(t.numpy(), want, atol=1e-12)
