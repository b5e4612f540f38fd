"""The renderer's MLP code run unfused (mnr_probe_mlp) against the FP64
oracle's MLP (Sec. 4.4 Eq. 13: bias-free, ReLU hidden layers, sigmoid
colour and ReLU density heads), on the same features and weights.

Tolerances: F32 MFMA with FP32 accumulation in another order than the
oracle's: |gpu - oracle| <= 1e-5 (1 + |oracle|).  BF16: inputs and weights
are exactly the BF16 values the kernel reads (so the oracle sees them
too); the kernel also rounds each hidden layer's activations to BF16
(relative error <= 2^-9 each, three rounded layers), so the bound is
2e-2 (1 + |oracle|) per output with a mean error below 2e-3.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu


def _features(n, seed):
    g = np.random.default_rng(seed)
    f = g.uniform(-1.0, 1.0, (n, 32))
    f[:, 0] = g.uniform(0.0, 1.0, n)           # the density feature is an occupancy in [0, 1]
    return f


def _oracle(feat64, weights):
    rgb, sigma = oracle.mlp(torch.as_tensor(feat64, dtype=torch.float64),
                            [torch.as_tensor(w, dtype=torch.float64) for w in weights])
    return torch.cat([rgb, sigma[:, None]], 1).numpy()


@pytest.mark.parametrize("mlp_dt", [0, 2])
@pytest.mark.parametrize("sc_fn", [lambda: scenes.scene_small(H=8, W=8, spp=8), lambda: scenes.scene_body(H=8, W=8)])
def test_unfused_mlp_matches_oracle(mlp_dt, sc_fn):
    import paper_2306_16541_amd as m
    sc = sc_fn()
    fld, _ = m.upload_scene(sc, "cuda", m.F32, mlp_dt)
    for n, seed in [(0, 1), (1, 2), (229, 3), (100_003, 4)]:     # empty, one sample, ragged, many chunks
        f64 = _features(n, seed)
        if mlp_dt == m.BF16:
            feat = torch.as_tensor(f64, dtype=torch.float32).to(torch.bfloat16).cuda()
        else:
            feat = torch.as_tensor(f64, dtype=torch.float32).cuda()
        out = m.probe_mlp(fld, feat)
        torch.cuda.synchronize()
        assert out.shape == (n, 4)
        if n == 0:
            continue
        w = [t.float().cpu().double().numpy() for t in fld.mlp]           # exactly what the kernel reads
        want = _oracle(feat.float().cpu().double().numpy(), w)
        got = out.cpu().double().numpy()
        err = np.abs(got - want) / (1.0 + np.abs(want))
        print(f"[probe_mlp dt={mlp_dt} layers={len(w)} n={n}] max rel {err.max():.2e} mean {err.mean():.2e}",
              flush=True)
        if mlp_dt == m.F32:
            assert err.max() <= 1e-5
        else:
            assert err.max() <= 2e-2 and err.mean() <= 2e-3
