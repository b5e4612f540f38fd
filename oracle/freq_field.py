"""FP64 oracle of the paper's own canonical field (test infrastructure).

TEST INFRASTRUCTURE ONLY (same rules as oracle/render.py).

Paper: Sec. 4.4, Eq. 13 and Fig. 9.  c, sigma = MLP_nerf(gamma(x_final)),
gamma a standard positional encoding, with a skip connection of the
encoding into the fourth layer.  Readings (each listed in the design doc):
gamma(x) = [x, sin(2^k pi x_c), cos(2^k pi x_c) for k = 0..9] (the 10
bands NeRF uses for positions; 63 values, zero-padded to 64), the
canonical coordinate itself as input; layers W1 (64 -> 64), W2, W3
(64 -> 64), W4 ([h3; gamma], 128 -> 64), W5 (64 -> 4); ReLU; no biases;
outputs as the grid field's: c = sigmoid(o[0:3]), sigma = ReLU(o[3]).
The skip takes gamma(x_final) (the figure's caption names x_skel, read as
a slip since the network's input is x_final).
"""
from __future__ import annotations

import math
from typing import Sequence

import torch

from .render import as64

N_BANDS = 10
ENC_WIDTH = 64


def posenc10(x: torch.Tensor) -> torch.Tensor:
    """gamma(x) [B, 64]: x, then per band k: sin(2^k pi x_c) (c = 0..2), cos(2^k pi x_c), then one zero."""
    x = as64(x)
    parts = [x]
    for k in range(N_BANDS):
        arg = (2.0 ** k) * math.pi * x
        parts.append(torch.sin(arg))
        parts.append(torch.cos(arg))
    g = torch.cat(parts, dim=1)
    return torch.cat([g, torch.zeros(x.shape[0], ENC_WIDTH - g.shape[1], dtype=g.dtype)], dim=1)


def freq_field(x: torch.Tensor, weights: Sequence):
    """(rgb [B,3], sigma [B]) of MLP_nerf(gamma(x)) with the skip at layer 4."""
    W1, W2, W3, W4, W5 = (as64(w) for w in weights)
    g = posenc10(x)
    h = torch.relu(g @ W1.T)
    h = torch.relu(h @ W2.T)
    h = torch.relu(h @ W3.T)
    h = torch.relu(torch.cat([h, g], dim=1) @ W4.T)
    o = h @ W5.T
    return torch.sigmoid(o[:, :3]), torch.relu(o[:, 3])
