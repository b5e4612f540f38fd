"""Pins of the residual-motion oracle (oracle/residual.py) against values
the definition fixes: special values of the window and of sin/cos, special
cases that collapse the network to a closed form, and the zero-output case
that must leave the render unchanged."""
import math

import numpy as np
import torch

import oracle
import scenes
from oracle.residual import K_BANDS, hann_window, posenc, residual_offset


def test_hann_window_special_values():
    assert torch.equal(hann_window(0.0), torch.zeros(K_BANDS, dtype=torch.float64))
    assert torch.equal(hann_window(float(K_BANDS)), torch.ones(K_BANDS, dtype=torch.float64))
    w = hann_window(2.5)               # bands 0, 1 open, band 2 half open, band 3 closed
    assert torch.allclose(w, torch.tensor([1.0, 1.0, 0.5, 0.0], dtype=torch.float64), atol=1e-15)
    a = np.linspace(0, K_BANDS, 41)
    ws = torch.stack([hann_window(float(v)) for v in a])
    assert bool((ws[1:] >= ws[:-1]).all())     # opening the window never closes a band


def test_posenc_special_values_and_order():
    s2 = math.sqrt(0.5)
    g = posenc(torch.tensor([[0.25, 0.5, -0.25]], dtype=torch.float64), float(K_BANDS))[0]
    want = [0.25, 0.5, -0.25,
            s2, 1.0, -s2, s2, 0.0, s2,            # band 0: sin(pi x_c), cos(pi x_c)
            1.0, 0.0, -1.0, 0.0, -1.0, 0.0,       # band 1: 2 pi x
            0.0, 0.0, 0.0, -1.0, 1.0, -1.0,       # band 2: 4 pi x
            0.0, 0.0, 0.0, 1.0, 1.0, 1.0,         # band 3: 8 pi x
            0.0, 0.0, 0.0, 0.0, 0.0]              # padding to 32
    assert g.shape == (32,)
    assert torch.allclose(g, torch.tensor(want, dtype=torch.float64), atol=1e-12)
    g0 = posenc(torch.tensor([[0.3, -0.2, 0.1]], dtype=torch.float64), 0.0)[0]
    assert torch.equal(g0[3:], torch.zeros(29, dtype=torch.float64))   # window closed: only x itself


def _pose():
    return torch.as_tensor(scenes.pose(3, 0.2), dtype=torch.float64)


def test_skip_connection_alone():
    # W1 = 0 and W_omega = 0: h1..h3 are zero, so the 4th layer sees only the
    # skip input and x_res = W5 ReLU(W4[:, 64:] gamma).
    g = np.random.default_rng(0)
    ws = [g.standard_normal(s) for s in scenes.RES_SHAPES]
    ws[0][:] = 0.0
    x = torch.as_tensor(g.uniform(-0.5, 0.5, (7, 3)))
    got = residual_offset(x, _pose(), [torch.as_tensor(w) for w in ws], torch.zeros(64, 72), 3.3)
    gam = posenc(x, 3.3).numpy()
    want = np.maximum(gam @ ws[3][:, 64:].T, 0.0) @ ws[4].T
    assert np.allclose(got.numpy(), want, atol=1e-12)


def test_pose_condition_through_identity_layers():
    # W1 = 0, identity hidden layers and no skip input: every point gets the
    # same offset, the selected rows of ReLU(W_omega Omega).
    g = np.random.default_rng(1)
    w_omega = g.standard_normal((64, 72))
    eye = np.eye(64)
    W4 = np.concatenate([eye, np.zeros((64, 32))], axis=1)
    W5 = np.zeros((3, 64)); W5[0, 5] = 1.0; W5[1, 17] = -2.0; W5[2, 40] = 0.5
    ws = [np.zeros((64, 32)), eye, eye, W4, W5]
    om = _pose()
    x = torch.as_tensor(g.uniform(-0.5, 0.5, (5, 3)))
    got = residual_offset(x, om, [torch.as_tensor(w) for w in ws], torch.as_tensor(w_omega), 4.0).numpy()
    b = np.maximum(w_omega @ om.numpy().reshape(-1), 0.0)
    want = np.array([b[5], -2.0 * b[17], 0.5 * b[40]])
    assert np.allclose(got, np.broadcast_to(want, got.shape), atol=1e-12)


def test_zero_output_layer_leaves_the_render_unchanged():
    sc = scenes.scene_small(H=12, W=10, spp=16)
    ws, w_omega = scenes.residual_weights(5)
    ws[4] = np.zeros_like(ws[4])
    a = oracle.render_image(sc, residual={"weights": ws, "w_omega": w_omega, "alpha": 4.0})
    b = oracle.render_image(sc)
    assert torch.equal(a, b)
    ws2, _ = scenes.residual_weights(5)
    c = oracle.render_image(sc, residual={"weights": ws2, "w_omega": w_omega, "alpha": 4.0})
    assert float((c - b).abs().max()) > 1e-4    # a non-zero residual moves the image
