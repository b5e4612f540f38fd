"""Pins of the FP64 CPU oracle against closed forms, invariants, hand-computed
values and brute-force quadrature (CPU only).

Each test pins one part of the oracle to something other than the oracle
itself, so that a dropped term, a wrong sign or index or a transposed
operand in it fails here.
"""
import math

import os

import numpy as np
import pytest
import torch

import oracle
import scenes
from oracle import render as O
from oracle.rng import splitmix64, stratified_xi

F64 = torch.float64


# ---------------------------------------------------------------- RNG ------

def test_splitmix64_published_first_output():
    # The published first output of SplitMix64 seeded with 0 (a cited text
    # fixture under tests/golden/).
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "splitmix64_seed0.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    assert rows
    for seed, idx, hex_out, signed_out in rows:
        got = int(splitmix64(int(seed), np.array([int(idx)]))[0])
        assert got == int(hex_out, 16)
        assert got - (1 << 64) == int(signed_out)


def test_stratified_xi_range_and_counter_layout():
    xi = stratified_xi(7, 5, 16)
    assert xi.shape == (5, 16) and xi.min() >= 0.0 and xi.max() < 1.0
    # counter n = ray * S + sample
    direct = (splitmix64(7, np.array([3 * 16 + 9])) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    assert xi[3, 9] == direct[0]


# ---------------------------------------------------- composite (Eq. 3) ----

def _comp(sigma, rgb, L, delta, bg=(0.0, 0.0, 0.0)):
    return O.composite(torch.as_tensor(sigma, dtype=F64), torch.as_tensor(rgb, dtype=F64),
                       torch.as_tensor(L, dtype=F64), torch.as_tensor(delta, dtype=F64), bg)


@pytest.mark.parametrize("S", [1, 7, 64, 192])
def test_composite_uniform_density_closed_form(S):
    # Uniform sigma over a chord of length Lc with alpha' = alpha (L >= 1):
    # opacity 1 - exp(-sigma Lc), colour c0 * (1 - exp(-sigma Lc)) + bg exp(-sigma Lc).
    sig, Lc = 3.7, 1.3
    c0 = np.array([0.2, 0.5, 0.9])
    bg = (0.1, 0.3, 0.6)
    C, A, w = _comp(np.full((1, S), sig), np.broadcast_to(c0, (1, S, 3)), np.full((1, S), 1.7),
                    np.array([Lc / S]), bg)
    T = math.exp(-sig * Lc)
    assert abs(float(A[0]) - (1 - T)) < 1e-13
    np.testing.assert_allclose(C[0].numpy(), c0 * (1 - T) + np.array(bg) * T, rtol=0, atol=1e-13)


def test_composite_invariants():
    g = np.random.default_rng(3)
    B, S = 50, 40
    sigma = g.exponential(5.0, (B, S)) * (g.random((B, S)) < 0.7)
    rgb = g.random((B, S, 3))
    L = g.uniform(0.0, 1.6, (B, S))
    delta = g.uniform(0.001, 0.05, B)
    C, A, w = _comp(sigma, rgb, L, delta)
    # sum of weights = 1 - T_S = opacity, within [0, 1]
    np.testing.assert_allclose(w.sum(1).numpy(), A.numpy(), atol=1e-13)
    assert float(w.sum(1).max()) <= 1.0 + 1e-15 and float(w.min()) >= 0.0
    # transmittance non-increasing
    alpha = 1 - np.exp(-sigma * delta[:, None]) * 1.0
    a = alpha * np.clip(L, 0, 1)
    T = np.cumprod(np.concatenate([np.ones((B, 1)), 1 - a], 1), 1)
    assert np.all(np.diff(T, axis=1) <= 0)
    # the augmentation: L = 0 everywhere -> nothing is seen
    bg = (0.25, 0.5, 0.75)
    C0, A0, _ = _comp(sigma, rgb, np.zeros((B, S)), delta, bg)
    np.testing.assert_array_equal(C0.numpy(), np.broadcast_to(bg, (B, 3)))
    np.testing.assert_array_equal(A0.numpy(), 0.0)


def test_composite_colour_derivative_is_weight():
    g = np.random.default_rng(4)
    sigma = torch.as_tensor(g.exponential(4.0, (3, 20)))
    rgb = torch.as_tensor(g.random((3, 20, 3)), dtype=F64).requires_grad_(True)
    L = torch.as_tensor(g.uniform(0.5, 1.2, (3, 20)))
    C, A, w = O.composite(sigma, rgb, L, torch.full((3,), 0.03, dtype=F64), (0.0, 0.0, 0.0))
    C[:, 1].sum().backward()
    np.testing.assert_allclose(rgb.grad[:, :, 1].numpy(), w.detach().numpy(), atol=1e-15)
    np.testing.assert_array_equal(rgb.grad[:, :, 0].numpy(), 0.0)


def test_composite_opacity_derivative_uniform():
    # d/dsigma of 1 - exp(-sigma Lc) is Lc exp(-sigma Lc) for uniform sigma.
    S, Lc, s0 = 32, 0.9, 2.5
    sig = torch.tensor(s0, dtype=F64, requires_grad=True)
    C, A, _ = O.composite(sig.expand(1, S), torch.zeros(1, S, 3, dtype=F64), torch.ones(1, S, dtype=F64),
                          torch.tensor([Lc / S], dtype=F64), (0.0, 0.0, 0.0))
    A.sum().backward()
    assert abs(float(sig.grad) - Lc * math.exp(-s0 * Lc)) < 1e-13


def _exact_integral(sigma_f, Sigma_f, c_f, Lc):
    """Eq. 2 by adaptive quadrature: C = int_0^Lc T(t) sigma(t) c(t) dt with
    T(t) = exp(-Sigma(t)), Sigma the closed-form integral of sigma."""
    from scipy.integrate import quad
    return np.array([quad(lambda t: math.exp(-Sigma_f(t)) * sigma_f(t) * c_f(t)[k], 0.0, Lc,
                          epsabs=1e-14, epsrel=1e-13, limit=400)[0] for k in range(3)])


def test_quadrature_converges_to_rendering_integral():
    a, b, Lc = 2.0, 1.5, 1.4
    sigma_f = lambda t: a + b * math.sin(3 * t)
    Sigma_f = lambda t: a * t + b * (1 - math.cos(3 * t)) / 3
    c_f = lambda t: (0.5 + 0.4 * math.cos(3 * t), 0.5 + 0.3 * math.sin(2 * t), 0.2 + 0.1 * t)
    exact = _exact_integral(sigma_f, Sigma_f, c_f, Lc)
    errs = []
    for S in (32, 64, 128, 256):
        t = (np.arange(S) + 0.5) * Lc / S
        sig = np.array([sigma_f(v) for v in t])[None]
        rgb = np.array([c_f(v) for v in t])[None]
        C, _, _ = _comp(sig, rgb, np.ones((1, S)), np.array([Lc / S]))
        errs.append(np.abs(C[0].numpy() - exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.6 < r < 4.4 for r in ratios), (errs, ratios)   # second order (midpoints)
    assert errs[-1] < 5e-5


def test_quadrature_exact_for_piecewise_constant_field():
    from scipy.integrate import quad
    S, Lc = 9, 1.1
    d = Lc / S
    g = np.random.default_rng(5)
    sk, ck = g.uniform(0, 6, S), g.random((S, 3))
    Sigma_edges = np.concatenate([[0.0], np.cumsum(sk * d)])
    exact = np.zeros(3)
    for k in range(S):
        for ch in range(3):
            exact[ch] += quad(lambda t: math.exp(-(Sigma_edges[k] + sk[k] * (t - k * d))) * sk[k] * ck[k, ch],
                              k * d, (k + 1) * d, epsabs=1e-15, epsrel=1e-14)[0]
    C, A, _ = _comp(sk[None], ck[None], np.ones((1, S)), np.array([d]))
    np.testing.assert_allclose(C[0].numpy(), exact, rtol=1e-11, atol=1e-14)
    assert abs(float(A[0]) - (1 - math.exp(-Sigma_edges[-1]))) < 1e-13


# -------------------------------------------------------- FK (Eq. 8) ------

def test_rodrigues_known_and_orthonormal():
    R = O.rodrigues(np.array([[0.0, 0.0, math.pi / 2], [0.0, 0.0, 0.0], [1e-14, 0.0, 0.0]]))
    np.testing.assert_allclose(R[0].numpy(), [[0, -1, 0], [1, 0, 0], [0, 0, 1]], atol=1e-15)
    np.testing.assert_array_equal(R[1].numpy(), np.eye(3))
    g = np.random.default_rng(1)
    R = O.rodrigues(g.normal(0, 1.0, (30, 3)))
    for r in R.numpy():
        np.testing.assert_allclose(r @ r.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(r) - 1) < 1e-14


def test_fk_two_joint_chain_by_hand():
    # root at the origin, child at (1,0,0); root turned +90 deg about z.
    G = O.bone_transforms([-1, 0], [[0, 0, 0], [1, 0, 0]], [[0, 0, math.pi / 2], [0, 0, 0]]).numpy()
    apply = lambda g, x: g[:, :3] @ np.array(x, dtype=np.float64) + g[:, 3]
    # canonical (2,0,0) sits at observed (0,2,0); canonical (1,0,0) at (0,1,0)
    np.testing.assert_allclose(apply(G[1], [0, 2, 0]), [2, 0, 0], atol=1e-15)
    np.testing.assert_allclose(apply(G[0], [0, 1, 0]), [1, 0, 0], atol=1e-15)


def test_fk_rest_pose_is_identity_and_inverse():
    parents, rest = scenes.skeleton()
    G = O.bone_transforms(parents, rest, np.zeros((24, 3))).numpy()
    np.testing.assert_array_equal(G[:, :, :3], np.broadcast_to(np.eye(3), (24, 3, 3)))
    np.testing.assert_allclose(G[:, :, 3], 0.0, atol=1e-17)
    om = scenes.pose(11, 0.3).astype(np.float64)
    G = O.bone_transforms(parents, rest, om).numpy()
    Ar, At = [t.numpy() for t in O.world_transforms(parents, rest, om)]
    J = rest.astype(np.float64)
    for j in range(24):
        Bm = np.eye(4); Bm[:3, :3] = Ar[j]; Bm[:3, 3] = At[j] - Ar[j] @ J[j]
        Gm = np.eye(4); Gm[:3, :] = G[j]
        np.testing.assert_allclose(Gm @ Bm, np.eye(4), atol=1e-14)


def test_fk_rotation_only_moves_subtree():
    parents, rest = scenes.skeleton()
    om = scenes.pose(12, 0.2).astype(np.float64)
    G0 = O.bone_transforms(parents, rest, om).numpy()
    om2 = om.copy(); om2[18] += [0.3, -0.2, 0.5]        # left elbow
    G1 = O.bone_transforms(parents, rest, om2).numpy()
    subtree = {18, 20, 22}
    for j in range(24):
        if j in subtree:
            assert np.abs(G1[j] - G0[j]).max() > 1e-3
        else:
            np.testing.assert_array_equal(G1[j], G0[j])


# ------------------------------------------------------ rays and box ------

def test_camera_centre_ray_and_box():
    cam = scenes.camera(64, 64)
    o, d = O.camera_rays(cam, 64, 64, [32 * 64 + 32])
    np.testing.assert_allclose(o.numpy(), [0, 0, 3], atol=1e-15)
    e = np.array([0.5 / 128, -0.5 / 128, -1.0]); e /= np.linalg.norm(e)
    np.testing.assert_allclose(d[0].numpy(), e, atol=1e-15)
    tn, tf, hit = O.ray_box(torch.tensor([0.0, 0.0, 3.0], dtype=F64),
                            torch.tensor([[0.0, 0.0, -1.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]], dtype=F64),
                            (-0.5,) * 3, (0.5,) * 3)
    assert float(tn[0]) == 2.5 and float(tf[0]) == 3.5 and bool(hit[0])
    assert not bool(hit[1]) and not bool(hit[2])           # parallel outside; pointing away
    tn, tf, hit = O.ray_box(torch.tensor([0.1, 0.0, 0.0], dtype=F64), torch.tensor([[0.0, 1.0, 0.0]], dtype=F64),
                            (-0.5,) * 3, (0.5,) * 3)
    assert float(tn[0]) == 0.0 and float(tf[0]) == 0.5 and bool(hit[0])   # origin inside


# --------------------------------------------------- warp (Eq. 7, 9) ------

def test_trilinear_volume_linear_and_zero_padding():
    R = 6
    z, y, x = np.meshgrid(*[np.arange(R, dtype=np.float64)] * 3, indexing="ij")
    vol = torch.as_tensor((1 + 2 * x + 3 * y + 5 * z)[None])
    g = np.random.default_rng(2)
    q = torch.as_tensor(g.uniform(0, R - 1, (200, 3)))
    v = O.trilinear_zero_padded(vol, torch.zeros(200, dtype=torch.int64), q).numpy()
    qn = q.numpy()
    np.testing.assert_allclose(v, 1 + 2 * qn[:, 0] + 3 * qn[:, 1] + 5 * qn[:, 2], rtol=1e-14)
    edge = torch.tensor([[-0.5, 1.0, 1.0], [R - 1.0, R - 1.0, R - 1.0], [R - 0.75, 0.0, 0.0], [-1.0, 2, 2]], dtype=F64)
    v = O.trilinear_zero_padded(vol, torch.zeros(4, dtype=torch.int64), edge).numpy()
    np.testing.assert_allclose(v, [0.5 * (1 + 3 + 5), 1 + 10 * (R - 1), 0.75 * (1 + 2 * (R - 1)), 0.0], rtol=1e-15)


def test_warp_identity_pose_is_identity():
    g = np.random.default_rng(6)
    Wc = O.motion_weights(scenes.motion_logits(5, 16))
    x = torch.as_tensor(g.uniform(-0.5, 0.5, (300, 3)))
    G = torch.cat([torch.eye(3, dtype=F64).expand(24, 3, 3), torch.zeros(24, 3, 1, dtype=F64)], 2)
    xs, L = O.inverse_lbs(x, G, Wc, (-0.5,) * 3, (0.5,) * 3)
    assert float(L.min()) > 0.5
    np.testing.assert_allclose(xs.numpy(), x.numpy(), atol=1e-15)


def test_warp_single_bone_is_rigid_and_blend_is_convex():
    g = np.random.default_rng(7)
    Rm = O.rodrigues(np.array([[0.3, -0.7, 0.2]]))[0]
    G1 = torch.cat([Rm, torch.tensor([[0.05], [-0.1], [0.02]], dtype=F64)], 1)[None]
    Wc = O.motion_weights(g.normal(0, 1, (2, 12, 12, 12)))
    x = torch.as_tensor(g.uniform(-0.35, 0.35, (200, 3)))
    xs, L = O.inverse_lbs(x, G1, Wc, (-0.5,) * 3, (0.5,) * 3)
    ok = L.numpy() > 1e-3
    assert ok.sum() > 150
    np.testing.assert_allclose(xs.numpy()[ok], (x @ Rm.T + G1[0, :, 3]).numpy()[ok], atol=1e-15)
    # 24 bones: the warped point lies in the bounding box of the G_i x
    parents, rest = scenes.skeleton()
    G = O.bone_transforms(parents, rest, scenes.pose(3, 0.3).astype(np.float64))
    Wc = O.motion_weights(scenes.motion_logits(9, 16))
    xs, L = O.inverse_lbs(x, G, Wc, (-0.5,) * 3, (0.5,) * 3)
    y = torch.einsum("kab,nb->nka", G[:, :, :3], x) + G[None, :, :, 3]
    assert torch.all(xs >= y.min(1).values - 1e-14) and torch.all(xs <= y.max(1).values + 1e-14)


def test_render_invariant_under_joint_rotation_of_body_and_camera():
    # Root turned +90 deg about y with the camera turned the same way: the
    # unit box maps to itself and the image must not change.
    sc = scenes.scene_small(H=24, W=24, spp=24)
    om = sc.axis_angle.astype(np.float64).copy()
    om[0] = 0.0
    base = oracle.render_image(sc, axis_angle=om).numpy()
    om[0] = [0.0, math.pi / 2, 0.0]
    turned = oracle.render_image(sc, axis_angle=om, cam=scenes.camera(24, 24, yaw_quarter_turns=1)).numpy()
    assert np.abs(base[:, 3]).max() > 1e-3
    np.testing.assert_allclose(turned, base, atol=1e-12)


# ----------------------------------------------------- grid encoding ------

def test_grid_hash_hand_computed():
    T = 1 << 19
    c = torch.tensor([[1, 2, 3], [511, 500, 7]], dtype=torch.int64)
    # (1*1 ^ 2*2654435761 ^ 3*805459861) mod 2^32 = 0xAC69F5DC -> & (2^19-1) = 128476
    np.testing.assert_array_equal(O.grid_index(c, 512, T).numpy(), [128476, 117080])
    # a dense level: x + (N+1)(y + (N+1) z)
    np.testing.assert_array_equal(O.grid_index(c[:1], 16, T).numpy(), [1 + 17 * (2 + 17 * 3)])


def test_grid_reproduces_linear_field_on_dense_levels():
    res = (16, 20)
    T = 1 << 14
    a = np.array([[0.3, -0.2, 0.7], [1.1, 0.4, -0.5]])   # per feature
    b = np.array([0.05, -0.3])
    table = np.zeros((2, T, 2))
    for l, N in enumerate(res):
        g = np.arange(N + 1)
        iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
        idx = (ix + (N + 1) * (iy + (N + 1) * iz)).ravel()
        uv = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], 1) / N
        table[l, idx] = uv @ a.T + b
    x = np.random.default_rng(8).uniform(-0.6, 0.6, (300, 3))
    f = O.grid_encode(torch.as_tensor(x), torch.as_tensor(table), res, (-0.5,) * 3, (0.5,) * 3).numpy()
    u = np.clip(x + 0.5, 0, 1)
    for l in range(2):
        np.testing.assert_allclose(f[:, 2 * l:2 * l + 2], u @ a.T + b, atol=1e-14)


def test_grid_is_continuous_across_cell_faces():
    table = torch.as_tensor(scenes.grid_table(4, 19).astype(np.float64))
    res = scenes.LEVEL_RES
    u0 = np.array([[0.25, 0.5, 0.75]])          # exactly on faces at every level with N % 4 == 0
    pts = np.concatenate([u0, u0 - 1e-13, u0 + 1e-13, [[1.0, 1.0, 1.0]], [[1.0 - 1e-13] * 3]]) - 0.5
    f = O.grid_encode(torch.as_tensor(pts), table, res, (-0.5,) * 3, (0.5,) * 3).numpy()
    np.testing.assert_allclose(f[1], f[0], atol=1e-10)
    np.testing.assert_allclose(f[2], f[0], atol=1e-10)
    np.testing.assert_allclose(f[4], f[3], atol=1e-10)


# ---------------------------------------------------------------- MLP ------

def test_mlp_hand_evaluated():
    W1 = torch.tensor([[1.0, 1.0], [2.0, 0.5]], dtype=F64)
    W2 = torch.tensor([[1.0, 2.0], [0.0, -1.0], [3.0, 0.0], [0.5, 4.0]], dtype=F64)
    c, s = O.mlp(torch.tensor([[1.0, -2.0]], dtype=F64), [W1, W2])
    # hidden relu([-1, 1]) = [0, 1]; out = [2, -1, 0, 4]
    np.testing.assert_allclose(c[0].numpy(), [0.8807970779778823, 0.2689414213699951, 0.5], atol=1e-15)
    assert float(s[0]) == 4.0
    c, s = O.mlp(torch.ones(3, 32, dtype=F64), [torch.zeros(64, 32, dtype=F64), torch.zeros(4, 64, dtype=F64)])
    np.testing.assert_array_equal(c.numpy(), 0.5)
    np.testing.assert_array_equal(s.numpy(), 0.0)


# ----------------------------------------------------------- gradients -----

def _tiny_setup(seed=21):
    sc = scenes.scene_body(H=32, W=32, spp=12, res=8, log2_T=14, pose_std=0.2, seed=seed)
    pid = np.array([16 * 32 + 16, 12 * 32 + 14, 20 * 32 + 17, 9 * 32 + 16, 26 * 32 + 13, 16 * 32 + 7])
    tgt = np.random.default_rng(seed).random((len(pid), 3))
    xi = stratified_xi(seed, len(pid), sc.spp)
    return sc, pid, tgt, xi


def _loss(sc, field, pid, tgt, xi):
    G = O.bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle)
    o, d = O.camera_rays(sc.cam, sc.H, sc.W, pid)
    return O.mse_loss(O.render_rays(field, G, o, d, sc.spp, xi=xi), tgt)


def test_autograd_gradient_matches_central_differences():
    sc, pid, tgt, xi = _tiny_setup()
    field = O.Field.from_scene(sc, requires_grad=True)
    loss = _loss(sc, field, pid, tgt, xi)
    loss.backward()
    g = np.random.default_rng(0)
    groups = [("table", field.table)] + [(f"mlp{k}", w) for k, w in enumerate(field.mlp)] + [("logits", field.logits)]
    checked = 0
    for name, p in groups:
        grad = p.grad.reshape(-1).numpy()
        touched = np.nonzero(grad)[0]
        assert touched.size > 0, name
        pick = np.unique(np.concatenate([touched[np.argsort(-np.abs(grad[touched]))[:6]],
                                         g.choice(touched, min(6, touched.size), replace=False)]))
        flat = p.detach().reshape(-1)
        for i in pick:
            base = float(flat[i])
            h = 1e-6 * max(1.0, abs(base))
            vals = []
            for s in (-1, 0, 1):
                with torch.no_grad():
                    flat[i] = base + s * h
                vals.append(float(_loss(sc, field, pid, tgt, xi)))
            with torch.no_grad():
                flat[i] = base
            fd = (vals[2] - vals[0]) / (2 * h)
            left, right = (vals[1] - vals[0]) / h, (vals[2] - vals[1]) / h
            if abs(left - right) > 1e-3 * max(abs(fd), 1e-8):
                continue                     # a kink (ReLU, cell face, clamp) inside the stencil
            assert abs(fd - grad[i]) <= 1e-6 * abs(fd) + 1e-10, (name, i, fd, grad[i])
            checked += 1
    assert checked >= 40


def test_softmax_gradient_sums_to_zero_per_voxel():
    sc, pid, tgt, xi = _tiny_setup(22)
    field = O.Field.from_scene(sc, requires_grad=True)
    _loss(sc, field, pid, tgt, xi).backward()
    s = field.logits.grad.sum(0)
    assert float(field.logits.grad.abs().max()) > 0
    assert float(s.abs().max()) < 1e-15


# ------------------------------------------------------------ workloads ----

@pytest.mark.slow
def test_body_scene_covers_about_thirty_percent_of_rays():
    sc = scenes.scene_body()
    pid = np.array([v * 512 + u for v in range(3, 512, 8) for u in range(5, 512, 8)])
    img = oracle.render_image(sc, pixel_ids=pid).numpy()
    frac = float((img[:, 3] > 0.5).mean())
    assert 0.27 <= frac <= 0.33, frac
    assert float((img[:, 3] > 1 - 1e-6).mean()) > 0.1      # early termination has work to skip
