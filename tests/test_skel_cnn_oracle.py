"""Pins of the skeleton-motion CNN oracle (oracle/skel_cnn.py): each
transposed convolution against a direct loop over its definition on a tiny
case, the grid doubling, and the single-voxel case written out by hand."""
import numpy as np
import torch
import torch.nn.functional as F

from oracle.skel_cnn import SLOPE, skel_cnn_logits


def _tconv_loop(x, w):
    """Transposed convolution, kernel 4, stride 2, padding 1, by its
    definition: input voxel v scatters w[i, o, k] * x[i, v] to output
    voxel 2 v - 1 + k (per axis) when that lies inside the output."""
    ci, D = x.shape[0], x.shape[1]
    co = w.shape[1]
    out = np.zeros((co, 2 * D, 2 * D, 2 * D))
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


def test_transposed_convolution_matches_its_definition():
    g = np.random.default_rng(0)
    x = g.standard_normal((3, 2, 2, 2))
    w = g.standard_normal((3, 2, 4, 4, 4))
    got = F.conv_transpose3d(torch.as_tensor(x)[None], torch.as_tensor(w), stride=2, padding=1)[0].numpy()
    assert got.shape == (2, 4, 4, 4)
    assert np.allclose(got, _tconv_loop(x, w), atol=1e-12)


def test_single_voxel_network_by_hand():
    # c0 = 1 channel at one voxel, one convolution: the 2^3 output is the
    # centre 2x2x2 of the kernel times LeakyReLU(w_fc z) (taps 1 and 2 of 4).
    g = np.random.default_rng(1)
    z = g.standard_normal(5)
    w_fc = g.standard_normal((1, 5))
    w1 = g.standard_normal((1, 3, 4, 4, 4))
    a = float(w_fc @ z)
    a = a if a > 0 else SLOPE * a
    want = a * w1[0][:, 1:3, 1:3, 1:3]
    got = skel_cnn_logits(z, w_fc, [w1]).numpy()
    assert np.allclose(got, want, atol=1e-12)


def test_five_convolutions_reach_32_cubed_and_the_last_has_no_activation():
    g = np.random.default_rng(2)
    ch = [8, 6, 5, 4, 3, 25]
    ws = [g.standard_normal((ch[k], ch[k + 1], 4, 4, 4)) * 0.3 for k in range(5)]
    out = skel_cnn_logits(g.standard_normal(16), g.standard_normal((8, 16)), ws)
    assert out.shape == (25, 32, 32, 32)
    assert float(out.min()) < 0 and float(out.max()) > 0       # no activation after the last layer
