"""FP64 oracle of the residual non-rigid motion (test infrastructure).

TEST INFRASTRUCTURE ONLY (same rules as oracle/render.py): only tests/,
__graft_entry__.smoke() and bench.py's cpu_baseline leg may use it, and it
shares no code with the GPU library.

Paper: Sec. 4.3, Eq. 11-12 and Fig. 8 (the residual motion network), with
the coarse-to-fine window of the encoding's frequency bands that Sec. 4.3
and Sec. 5.2 take from HumanNeRF.  What it computes, per skinned point
x_skel (the output of the inverse LBS of Eq. 9):

  gamma(x)  = [x_0, x_1, x_2,
               for k = 0..K-1:  w_k sin(2^k pi x_c) (c = 0, 1, 2),
                                w_k cos(2^k pi x_c) (c = 0, 1, 2),
               0, ... 0]                          (zero-padded to 32 values)
  w_k(a)    = (1 - cos(pi * clamp(a - k, 0, 1))) / 2       (truncated Hann
              window over the bands; Park et al. 2021, as used by HumanNeRF)
  h1 = ReLU(W1 gamma + W_omega Omega)      (the pose condition of Eq. 11)
  h2 = ReLU(W2 h1),  h3 = ReLU(W3 h2)
  h4 = ReLU(W4 [h3 ; gamma])               (skip connection at the 4th layer)
  x_res = W5 h4,     x_final = x_skel + x_res                    (Eq. 12)

Readings (the paper gives the structure, not the sizes; each is listed in
the design doc): K = 4 bands; the encoding's input is the canonical coordinate
itself; Omega is the observed pose's 24 axis-angle vectors, joint-major
(72 values); hidden width 64; no biases besides the pose term.
"""
from __future__ import annotations

import math
from typing import Sequence

import torch

from .render import as64

K_BANDS = 4
ENC_WIDTH = 32          # 3 + 6 K = 27 values, zero-padded
HIDDEN = 64


def hann_window(alpha: float, K: int = K_BANDS) -> torch.Tensor:
    """w_k = (1 - cos(pi clamp(alpha - k, 0, 1))) / 2 for k = 0..K-1."""
    k = torch.arange(K, dtype=torch.float64)
    return 0.5 * (1.0 - torch.cos(math.pi * torch.clamp(alpha - k, 0.0, 1.0)))


def posenc(x: torch.Tensor, alpha: float, K: int = K_BANDS) -> torch.Tensor:
    """gamma(x) [B, 32] of points x [B, 3] with the band window at alpha."""
    x = as64(x)
    w = hann_window(alpha, K)
    parts = [x]
    for k in range(K):
        arg = (2.0 ** k) * math.pi * x
        parts.append(w[k] * torch.sin(arg))
        parts.append(w[k] * torch.cos(arg))
    g = torch.cat(parts, dim=1)
    return torch.cat([g, torch.zeros(x.shape[0], ENC_WIDTH - g.shape[1], dtype=g.dtype)], dim=1)


def residual_offset(x_skel: torch.Tensor, omega, weights: Sequence[torch.Tensor], w_omega, alpha: float):
    """x_res [B, 3] = MLP_res(gamma(x_skel), Omega).  weights = (W1 [64,32],
    W2 [64,64], W3 [64,64], W4 [64,96], W5 [3,64]); w_omega [64, 72];
    omega: the pose's axis-angle vectors [24, 3]."""
    W1, W2, W3, W4, W5 = (as64(w) for w in weights)
    g = posenc(x_skel, alpha)
    bias = as64(w_omega) @ as64(omega).reshape(-1)
    h = torch.relu(g @ W1.T + bias[None, :])
    h = torch.relu(h @ W2.T)
    h = torch.relu(h @ W3.T)
    h = torch.relu(torch.cat([h, g], dim=1) @ W4.T)
    return h @ W5.T
