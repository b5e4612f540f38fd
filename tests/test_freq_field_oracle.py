"""Pins of the frequency-encoded field oracle (oracle/freq_field.py): the
encoding's values at points where sin and cos are known exactly, its
layout, and closed forms of the network with layers switched off."""
import math

import numpy as np
import torch

import oracle
import scenes
from oracle.freq_field import freq_field, posenc10


def test_posenc_at_special_points():
    g = posenc10(torch.tensor([[0.5, 0.0, -0.25]], dtype=torch.float64))[0]
    assert g.shape == (64,)
    assert torch.allclose(g[:3], torch.tensor([0.5, 0.0, -0.25], dtype=torch.float64))
    # band 0: sin(pi x) = (1, 0, -sqrt(1/2)), cos(pi x) = (0, 1, sqrt(1/2))
    s2 = math.sqrt(0.5)
    assert torch.allclose(g[3:9], torch.tensor([1.0, 0.0, -s2, 0.0, 1.0, s2], dtype=torch.float64), atol=1e-15)
    # bands k >= 3: 2^k pi x is a multiple of 2 pi for every coordinate -> sin 0, cos 1
    for k in range(3, 10):
        assert torch.allclose(g[3 + 6 * k: 9 + 6 * k], torch.tensor([0.0] * 3 + [1.0] * 3, dtype=torch.float64),
                              atol=1e-12)
    assert float(g[63]) == 0.0


def test_skip_only_network_closed_form():
    # W1 = 0: h1..h3 vanish and the output is W5 ReLU(W4[:, 64:] gamma).
    g = np.random.default_rng(0)
    ws = [np.zeros((64, 64)), g.standard_normal((64, 64)), g.standard_normal((64, 64)),
          g.standard_normal((64, 128)), g.standard_normal((4, 64))]
    x = torch.as_tensor(g.uniform(-0.5, 0.5, (9, 3)))
    rgb, sigma = freq_field(x, [torch.as_tensor(w) for w in ws])
    o = np.maximum(posenc10(x).numpy() @ ws[3][:, 64:].T, 0.0) @ ws[4].T
    assert np.allclose(rgb.numpy(), 1.0 / (1.0 + np.exp(-o[:, :3])), atol=1e-12)
    assert np.allclose(sigma.numpy(), np.maximum(o[:, 3], 0.0), atol=1e-12)


def test_zero_output_layer_gives_grey_transparent_field():
    # o = 0: c = 0.5, sigma = 0, so every ray shows the background.
    sc = scenes.scene_small(H=6, W=5, spp=8)
    field = oracle.Field.from_scene(sc)
    field.encoding = "freq"
    field.mlp = [torch.zeros(s, dtype=torch.float64) for s in ((64, 64), (64, 64), (64, 64), (64, 128), (4, 64))]
    out = oracle.render_image(sc, field=field, bg=(0.2, 0.3, 0.4))
    assert torch.allclose(out[:, :3], torch.tensor([0.2, 0.3, 0.4], dtype=torch.float64).expand(30, 3))
    assert torch.equal(out[:, 3], torch.zeros(30, dtype=torch.float64))
