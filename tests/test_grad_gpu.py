"""GPU adjoint vs the FP64 oracle's gradient (autograd over the oracle's
forward, itself pinned to central differences on the CPU), on a 16-ray
subset with stratified jitter.  Also a directional finite-difference check
of the GPU gradient against the oracle loss.

Tolerances, per parameter group:
  * every entry: |g_gpu - g_oracle| <= tau * max|g_oracle|, tau = 1e-4 on
    the FP32 path (FP32 forward and adjoint, unordered float atomics: about
    1e-6 relative per term, a few thousand terms per entry) and 1e-1 with
    the BF16 MLP: every MLP product rounds both operands to 8-bit mantissas
    (up to 2^-8 relative per product), and a table or weight gradient
    passes through the four layers forward and again backward, so its
    typical relative error is ~8 x 2^-8 = 3e-2 (the measured relative L2
    error of the groups); the largest deviation over ~10^4 entries is up to
    about three times that;
  * relative L2 error of the group: 2e-3 (FP32) and 5e-2 (BF16).
Per-entry central differences of the FP64 oracle loss check the largest
GPU entries of every group directly (parameters whose stencil crosses a
ReLU zero or grid-cell face are detected by their one-sided slopes and
skipped).  The full-size field (T = 2^19, R = 64, 512 x 512 camera) is
checked on the first 16 rays of the training batch.
"""
import numpy as np
import pytest
import torch

import scenes
from oracle import render as O
from oracle.rng import stratified_xi

pytestmark = pytest.mark.gpu

SEED = 77


def _scene():
    return scenes.scene_body(H=32, W=32, spp=128, res=32, log2_T=16, seed=16541 + 4)


def _rays(sc, n=16):
    g = np.random.default_rng(5)
    pid = np.array([(12 + g.integers(0, 8)) * sc.W + 12 + g.integers(0, 8) for _ in range(n // 2)] +
                   list(g.integers(0, sc.H * sc.W, n - n // 2)), dtype=np.int32)
    tgt = g.random((n, 3)).astype(np.float32)
    return pid, tgt


def gpu_grads(sc, pid, tgt, mlp_dtype, ert_tau=1e-6, binned=False, table_dtype=0):
    """binned: the table gradient goes through the binned scatter (records
    summed in LDS) instead of global atomics.  table_dtype: the renderer's
    copy of the table (FP32 or FP16)."""
    import paper_2306_16541_amd as m
    fld, _ = m.upload_scene(sc, "cuda", table_dtype, mlp_dtype)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=ert_tau, stratified=True, seed=SEED)
    pid_t = torch.as_tensor(pid, device="cuda")
    tgt_t = torch.as_tensor(tgt, device="cuda")
    n = len(pid)
    tch = torch.zeros(n, m.saved_size(sc.spp), device="cuda")
    rgba = m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, t_chunks=tch)
    grad_rgba = torch.empty(n, 4, device="cuda")
    loss = torch.zeros(1, device="cuda")
    m.mse_loss(rgba, tgt_t, grad_rgba, loss)
    g_table = torch.zeros(sc.table.shape, device="cuda")
    g_w = [torch.zeros(w.shape, device="cuda") for w in sc.mlp]
    g_wc = torch.zeros(sc.logits.shape, device="cuda")
    ws = m.adjoint_workspace(fld, n, sc.spp) if binned else None
    assert ws is not None or not binned
    m.render_backward(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, tch, grad_rgba, g_table, g_w, g_wc,
                      adjoint_ws=ws)
    g_logits = torch.zeros_like(g_wc)
    m.softmax_bwd(fld.weights, g_wc, g_logits)
    torch.cuda.synchronize()
    return (float(loss.item()), g_table.cpu().numpy(), [w.cpu().numpy() for w in g_w], g_logits.cpu().numpy(),
            rgba.cpu().numpy())


def oracle_grads(sc, pid, tgt):
    field = O.Field.from_scene(sc, requires_grad=True)
    G = O.bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle)
    o, d = O.camera_rays(sc.cam, sc.H, sc.W, pid)
    rgba = O.render_rays(field, G, o, d, sc.spp, xi=stratified_xi(SEED, len(pid), sc.spp))
    loss = O.mse_loss(rgba, tgt)
    loss.backward()
    return (float(loss.detach()), field.table.grad.numpy(), [w.grad.numpy() for w in field.mlp], field.logits.grad.numpy(),
            rgba.detach().numpy())


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-30))


TAU = {0: 1e-4, 2: 1e-1}


def _elementwise(name, a, b, tau, b_alt=None):
    """Every entry of a within tau * max|b| of b.  With b_alt (the oracle
    gradient at inputs moved by one float32 ulp): entries that b and b_alt
    disagree on by more than that sit on a kink (a sample within rounding of
    a ReLU zero or a cell face flips side); there a must match either."""
    scale = max(np.abs(b).max(), 1e-30)
    d = np.abs(a - b)
    kink = np.zeros(b.shape, bool) if b_alt is None else np.abs(b - b_alt) > tau * scale
    if b_alt is not None:
        d = np.where(kink, np.minimum(d, np.abs(a - b_alt)), d)
    err = float(d.max() / scale)
    print(f"  {name:7s} max|g_gpu - g_oracle| / max|g_oracle| = {err:.3e}"
          f" ({int(kink.sum())} entries on a kink)", flush=True)
    assert err <= tau, (name, err)


def _one_ulp_pose(sc, seed=5):
    """The scene with its joint rotations and rest joints one float32 ulp
    away (seeded directions): a probe for gradient kinks."""
    import dataclasses
    g = np.random.default_rng(seed)
    step = lambda v: np.where(g.integers(0, 2, v.shape).astype(bool), np.nextafter(v, np.float32(np.inf)),
                              np.nextafter(v, np.float32(-np.inf))).astype(np.float32)
    return dataclasses.replace(sc, axis_angle=step(sc.axis_angle), rest_joints=step(sc.rest_joints))


def _cos(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30))


@pytest.mark.parametrize("mlp_dtype,tol,binned", [(0, 2e-3, False), (2, 5e-2, False), (0, 2e-3, True),
                                                   (2, 5e-2, True)])
def test_adjoint_matches_oracle_gradient(mlp_dtype, tol, binned):
    sc = _scene()
    pid, tgt = _rays(sc)
    lg, tg, wg, logg, rg = gpu_grads(sc, pid, tgt, mlp_dtype, binned=binned)
    lo, to, wo, logo, ro = oracle_grads(sc, pid, tgt)
    assert (ro[:, 3] > 0.5).sum() >= 4                 # the subset sees the body
    print(f"[dtype {mlp_dtype}] loss gpu {lg:.8f} oracle {lo:.8f}; rgba max-abs {np.abs(rg - ro).max():.2e}")
    assert abs(lg - lo) <= (1e-5 if mlp_dtype == 0 else 1e-2) * abs(lo)
    groups = [("table", tg, to), ("logits", logg, logo)] + [(f"w{k}", a, b) for k, (a, b) in enumerate(zip(wg, wo))]
    for name, a, b in groups:
        r, c = _rel(a, b), _cos(a, b)
        print(f"  {name:7s} rel-L2 {r:.3e} cos {c:.6f} |g| {np.linalg.norm(b):.3e}", flush=True)
        assert np.linalg.norm(b) > 0, name
        assert r <= tol, name
        _elementwise(name, a, b, TAU[mlp_dtype])
    # partition of unity of the grid scatter: per-level sums agree
    sg, so = tg.reshape(tg.shape[0], -1).sum(1), to.reshape(to.shape[0], -1).sum(1)
    np.testing.assert_allclose(sg, so, rtol=0, atol=max(tol, 1e-4) * np.abs(so).max())
    # softmax adjoint: gradients of each voxel's logits sum to zero
    assert np.abs(logg.sum(0)).max() <= 1e-6 * max(np.abs(logg).max(), 1e-12) + 1e-12


def test_adjoint_with_fp16_table():
    # The renderer reading an FP16 copy of the table (mixed-precision
    # training keeps FP32 masters): the adjoint is that of the field with
    # the table rounded to FP16, so the FP64 oracle on the rounded table is
    # the reference, element by element as for the FP32 table.
    import dataclasses
    import paper_2306_16541_amd as m
    sc = _scene()
    sc16 = dataclasses.replace(sc, table=sc.table.astype(np.float16).astype(np.float32))
    pid, tgt = _rays(sc)
    for binned in (False, True):
        lg, tg, wg, logg, rg = gpu_grads(sc, pid, tgt, 0, binned=binned, table_dtype=m.F16)
        lo, to, wo, logo, ro = oracle_grads(sc16, pid, tgt)
        print(f"[fp16 table, binned {binned}] loss gpu {lg:.8f} oracle {lo:.8f}", flush=True)
        assert abs(lg - lo) <= 1e-5 * abs(lo)
        groups = [("table", tg, to), ("logits", logg, logo)] + [(f"w{k}", a, b) for k, (a, b) in enumerate(zip(wg, wo))]
        for name, a, b in groups:
            assert np.linalg.norm(b) > 0, name
            assert _rel(a, b) <= 2e-3, (name, _rel(a, b))
            _elementwise(name, a, b, TAU[0])


def test_adjoint_directional_derivative_matches_oracle_differences():
    # Move every parameter (table, MLP weights, logits) along the GPU
    # gradient g and take central differences of the FP64 oracle loss: the
    # directional derivative must equal g . g_true / |g| = |g| when the
    # adjoint is right.  The step is small enough that no ReLU or cell-face
    # kink lies inside the stencil (checked with the one-sided slopes).
    sc = _scene()
    pid, tgt = _rays(sc)
    _, tg, wg, logg, _ = gpu_grads(sc, pid, tgt, 0, ert_tau=0.0)
    gnorm = np.sqrt(sum(float((a.astype(np.float64) ** 2).sum()) for a in [tg, logg] + wg))
    G = O.bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle)
    o, d = O.camera_rays(sc.cam, sc.H, sc.W, pid)
    xi = stratified_xi(SEED, len(pid), sc.spp)

    def loss_at(eps):
        f = O.Field(sc.table.astype(np.float64) + eps * tg / gnorm,
                    [w.astype(np.float64) + eps * g / gnorm for w, g in zip(sc.mlp, wg)],
                    sc.logits.astype(np.float64) + eps * logg / gnorm, sc.level_res, sc.box_min, sc.box_max)
        return float(O.mse_loss(O.render_rays(f, G, o, d, sc.spp, xi=xi), tgt))

    eps = 1e-7
    lm, l0, lp = loss_at(-eps), loss_at(0.0), loss_at(eps)
    left, right, fd = (l0 - lm) / eps, (lp - l0) / eps, (lp - lm) / (2 * eps)
    print(f"  |g| {gnorm:.6e}  directional fd {fd:.6e}  one-sided {left:.6e} {right:.6e}", flush=True)
    assert abs(left - right) <= 1e-4 * abs(fd)
    assert abs(fd - gnorm) <= 1e-3 * gnorm


def _groups(table, logits, ws):
    return [("table", table), ("logits", logits)] + [(f"w{k}", w) for k, w in enumerate(ws)]


def test_largest_adjoint_entries_match_oracle_central_differences():
    # For the 10 largest GPU gradient entries of each group (grid table,
    # blend-weight logits, each MLP layer): perturb that one parameter of the
    # FP64 oracle by +-h and difference its loss.  Early termination off, so
    # both sides differentiate the same sum.
    sc = _scene()
    pid, tgt = _rays(sc)
    _, tg, wg, logg, _ = gpu_grads(sc, pid, tgt, 0, ert_tau=0.0)
    G = O.bone_transforms(sc.parents, sc.rest_joints, sc.axis_angle)
    o, d = O.camera_rays(sc.cam, sc.H, sc.W, pid)
    xi = stratified_xi(SEED, len(pid), sc.spp)
    base = {"table": sc.table.astype(np.float64), "logits": sc.logits.astype(np.float64)}
    for k, w in enumerate(sc.mlp):
        base[f"w{k}"] = w.astype(np.float64)

    def loss_with(name, idx, step):
        p = {k: v for k, v in base.items()}
        p[name] = base[name].copy()
        p[name][idx] += step
        f = O.Field(p["table"], [p[f"w{k}"] for k in range(len(sc.mlp))], p["logits"], sc.level_res,
                    sc.box_min, sc.box_max)
        return float(O.mse_loss(O.render_rays(f, G, o, d, sc.spp, xi=xi), tgt))

    l0 = loss_with("table", (0, 0, 0), 0.0)
    for name, g in _groups(tg, logg, wg):
        flat = np.argsort(-np.abs(g).ravel())[:10]
        gmax = float(np.abs(g).max())
        checked = 0
        for fi in flat:
            idx = np.unravel_index(fi, g.shape)
            h = 1e-6 * max(1.0, abs(float(base[name][idx])))
            lp, lm = loss_with(name, idx, h), loss_with(name, idx, -h)
            fd, left, right = (lp - lm) / (2 * h), (l0 - lm) / h, (lp - l0) / h
            if abs(left - right) > 1e-3 * abs(fd) + 1e-9:
                print(f"  {name} {idx}: one-sided slopes {left:.6e} / {right:.6e} disagree: kink, skipped")
                continue
            checked += 1
            assert abs(float(g[idx]) - fd) <= 1e-4 * gmax, (name, idx, float(g[idx]), fd)
        print(f"  {name:7s} {checked} of 10 largest entries match central differences (max|g| {gmax:.3e})",
              flush=True)
        assert checked >= 7, name


@pytest.mark.slow
def test_adjoint_on_the_full_size_field():
    # The training step's field: the 512 x 512 body scene with T = 2^19
    # entries per level and a 64^3 blend-weight volume; the first 16 rays of
    # the training batch, stratified, FP32 and BF16 MLP.
    sc = scenes.scene_body()
    pid, tgt = scenes.train_batch(7, sc.H, sc.W, 8192)
    pid, tgt = pid[:16], tgt[:16]
    lo, to, wo, logo, ro = oracle_grads(sc, pid, tgt)
    print(f"[full-size field] {(ro[:, 3] > 0.01).sum()} of 16 rays touch the body", flush=True)
    for mlp_dtype, tol in ((0, 2e-3), (2, 5e-2)):
        lg, tg, wg, logg, rg = gpu_grads(sc, pid, tgt, mlp_dtype, binned=True)
        print(f"[dtype {mlp_dtype}] loss gpu {lg:.8f} oracle {lo:.8f}", flush=True)
        assert abs(lg - lo) <= (1e-5 if mlp_dtype == 0 else 1e-2) * abs(lo)
        for name, a, b in [("table", tg, to), ("logits", logg, logo)] + \
                [(f"w{k}", a, b) for k, (a, b) in enumerate(zip(wg, wo))]:
            assert np.linalg.norm(b) > 0, name
            assert _rel(a, b) <= tol, (name, _rel(a, b))
            _elementwise(name, a, b, TAU[mlp_dtype])


@pytest.mark.parametrize("res", [32, 24])
def test_binned_scatter_equals_atomic_scatter(res):
    # The same adjoint with the table and blend-weight gradients summed
    # through the binned scatter and through global atomics: the same sums
    # in another order (float32 reassociation only), on a batch of 512 rays.
    # With a blend-weight volume whose side is not a power of two (24) only
    # the table is binned and dL/dW^c keeps run-summed atomics.
    sc = scenes.scene_body(H=64, W=64, spp=128, res=res, log2_T=16, seed=16541 + 4)
    g = np.random.default_rng(9)
    pid = g.integers(0, sc.H * sc.W, 512).astype(np.int32)
    tgt = g.random((512, 3)).astype(np.float32)
    a = gpu_grads(sc, pid, tgt, 0, binned=False)
    b = gpu_grads(sc, pid, tgt, 0, binned=True)
    ta, tb = a[1], b[1]
    err = float(np.abs(ta - tb).max() / np.abs(ta).max())
    print(f"  binned vs atomic table gradient: max diff {err:.2e} of max, "
          f"{int((ta != 0).sum())} nonzero entries", flush=True)
    assert (ta != 0).sum() > 10000
    assert err <= 1e-5
    # the blend-weight gradient (records of corner pairs when binned), seen
    # through the softmax adjoint as the logits' gradient
    la, lb = a[3], b[3]
    err_l = float(np.abs(la - lb).max() / np.abs(la).max())
    print(f"  binned vs atomic logits gradient: max diff {err_l:.2e} of max, "
          f"{int((la != 0).sum())} nonzero entries", flush=True)
    assert (la != 0).sum() > 1000
    assert err_l <= 1e-5
    for x, y in zip(a[2], b[2]):       # the MLP gradients are untouched by the switch
        assert float(np.abs(x - y).max()) <= 1e-5 * float(np.abs(x).max())


def test_ray_list_processing_order():
    # With a ray list and an adjoint workspace, the adjoint processes the
    # rays in a spatially coherent order kept at the end of the workspace:
    # a permutation of the rows, sorted by the Morton index of the pixel's
    # cell in a 64 x 64 grid over the image.
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=48, W=80, spp=64, res=32, log2_T=16, seed=16541 + 4)
    g = np.random.default_rng(12)
    n = 1000
    pid = g.integers(0, sc.H * sc.W, n).astype(np.int32)
    tgt = g.random((n, 3)).astype(np.float32)
    fld, _ = m.upload_scene(sc, "cuda", m.F32, 0)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=0.0, stratified=True, seed=SEED)
    pid_t = torch.as_tensor(pid, device="cuda")
    tch = torch.zeros(n, m.saved_size(sc.spp), device="cuda")
    rgba = m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, t_chunks=tch)
    grad_rgba = torch.empty(n, 4, device="cuda")
    m.mse_loss(rgba, torch.as_tensor(tgt, device="cuda"), grad_rgba)
    ws = m.adjoint_workspace(fld, n, sc.spp)
    m.render_backward(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t, tch, grad_rgba,
                      torch.zeros(sc.table.shape, device="cuda"), [torch.zeros(w.shape, device="cuda") for w in sc.mlp],
                      torch.zeros(sc.logits.shape, device="cuda"), adjoint_ws=ws)
    torch.cuda.synchronize()
    tail = -(-n * 4 // 256) * 256           # the order is the workspace's last part
    order = ws[ws.numel() - tail:ws.numel() - tail + 4 * n].view(torch.int32).cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(n))

    def cell(p):
        x = (p % sc.W) * 64 // sc.W
        y = (p // sc.W) * 64 // sc.H
        return sum((((x >> b) & 1) << (2 * b)) | (((y >> b) & 1) << (2 * b + 1)) for b in range(6))
    cells = np.array([cell(int(p)) for p in pid[order]])
    assert np.all(np.diff(cells) >= 0)


def test_binned_scatter_non_finite_gradient():
    # A non-finite loss gradient on one ray: the adjoint's bound on the
    # record values is then NaN, and the binned scatter sums in floats
    # instead of fixed point.  The rows that ray reaches are NaN in both
    # paths and every other entry agrees.
    sc = scenes.scene_body(H=64, W=64, spp=128, res=32, log2_T=16, seed=16541 + 4)
    import paper_2306_16541_amd as m
    g = np.random.default_rng(10)
    pid = torch.as_tensor(g.integers(0, sc.H * sc.W, 256).astype(np.int32), device="cuda")
    fld, _ = m.upload_scene(sc, "cuda", m.F32, 0)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=0.0, stratified=True, seed=SEED)
    tch = torch.zeros(256, m.saved_size(sc.spp), device="cuda")
    rgba = m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid, t_chunks=tch)
    hit = torch.nonzero(rgba[:, 3] > 0.5)[:, 0]
    assert hit.numel() > 0
    grad_rgba = torch.full((256, 4), 1e-2, device="cuda")
    grad_rgba[int(hit[0]), 0] = float("nan")
    out = []
    for binned in (False, True):
        g_table = torch.zeros(sc.table.shape, device="cuda")
        g_w = [torch.zeros(w.shape, device="cuda") for w in sc.mlp]
        g_wc = torch.zeros(sc.logits.shape, device="cuda")
        ws = m.adjoint_workspace(fld, 256, sc.spp) if binned else None
        m.render_backward(fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid, tch, grad_rgba, g_table, g_w, g_wc,
                          adjoint_ws=ws)
        torch.cuda.synchronize()
        out.append((g_table.cpu().numpy(), g_wc.cpu().numpy()))
    for (a, b), name in zip(zip(out[0], out[1]), ("table", "dL/dW^c")):
        na, nb = np.isnan(a), np.isnan(b)
        print(f"  {name}: {int(na.sum())} NaN entries (atomic), {int(nb.sum())} (binned)", flush=True)
        assert na.sum() > 0 and np.array_equal(na, nb), name
        fa, fb = a[~na], b[~nb]
        assert float(np.abs(fa - fb).max()) <= 1e-5 * float(np.abs(fa).max()), name


def test_binned_scatter_largest_table():
    # T = 2^24: the 4 hashed levels fill the key space (4096 bins of 2^14
    # rows, each summed in four 2^12-row parts); the dense levels and the
    # blend weights keep atomics.  Binned against atomic, hashed level by
    # hashed level, on 256 rays.
    print("[largest table] building the 2^24-row scene", flush=True)
    sc = scenes.scene_body(H=64, W=64, spp=64, res=32, log2_T=24, seed=16541 + 4)
    g = np.random.default_rng(11)
    pid = g.integers(0, sc.H * sc.W, 256).astype(np.int32)
    tgt = g.random((256, 3)).astype(np.float32)
    hashed = [l for l, n in enumerate(sc.level_res) if (int(n) + 1) ** 3 > 1 << 24]
    assert len(hashed) == 4
    a = gpu_grads(sc, pid, tgt, 0, binned=False)
    print("[largest table] atomic adjoint done", flush=True)
    b = gpu_grads(sc, pid, tgt, 0, binned=True)
    print("[largest table] binned adjoint done", flush=True)
    for l in hashed:
        ta, tb = a[1][l], b[1][l]
        mx = float(np.abs(ta).max())
        err = float(np.abs(ta - tb).max()) / mx
        print(f"  level {l} (N={int(sc.level_res[l])}): max diff {err:.2e} of max, "
              f"{int((ta != 0).sum())} nonzero entries", flush=True)
        assert mx > 0 and err <= 1e-5, (l, err)
    for l in range(len(sc.level_res)):  # the dense levels took the same atomics in both runs
        if l not in hashed:
            assert float(np.abs(a[1][l] - b[1][l]).max()) <= 1e-5 * float(np.abs(a[1][l]).max() + 1e-30), l


def test_binned_scatter_splits_crowded_bins():
    # The full-size field's coarse dense levels put hundreds of thousands of
    # records into one 4096-row bin (level 0 has 17^3 rows), which the
    # binned scatter sums with several blocks; against global atomics, level
    # by level, on 4096 rays of the training batch.
    sc = scenes.scene_body()
    pid, tgt = scenes.train_batch(7, sc.H, sc.W, 8192)
    pid, tgt = pid[:4096], tgt[:4096]
    a = gpu_grads(sc, pid, tgt, 0, binned=False)
    b = gpu_grads(sc, pid, tgt, 0, binned=True)
    assert abs(a[0] - b[0]) <= 1e-6 * abs(a[0])
    for l, n in enumerate(sc.level_res):
        ta, tb = a[1][l], b[1][l]
        mx = float(np.abs(ta).max())
        err = float(np.abs(ta - tb).max()) / mx
        if l in (0, 6, 7, 15):
            print(f"  level {l} (N={int(n)}, {'dense' if (int(n) + 1) ** 3 <= 1 << 19 else 'hashed'}): "
                  f"max diff {err:.2e} of max, {int((ta != 0).sum())} nonzero entries", flush=True)
        assert mx > 0, l
        assert err <= 1e-5, (l, err)
    la, lb = a[3], b[3]
    err_l = float(np.abs(la - lb).max() / np.abs(la).max())
    print(f"  logits (blend-weight records): max diff {err_l:.2e} of max", flush=True)
    assert err_l <= 1e-5


@pytest.mark.parametrize("ert_tau", [0.0, 1e-6])
def test_adjoint_after_full_frame_forward(ert_tau):
    # Full-frame forward (ray-packet kernel, per-sample early termination)
    # followed by the adjoint over every pixel, against the oracle (which
    # never terminates early; the gradient dropped by termination is bounded
    # by the threshold).  Every entry within 1e-4 of the group's largest.
    # The 256 rays of this frame put a few samples within float32 rounding
    # of a ReLU zero: one unit's row of W1, and some blend-weight logits,
    # then take the other side's gradient.  Such entries are found by
    # differentiating the oracle again at a pose one ulp away and must match
    # one of the two oracle gradients.
    import paper_2306_16541_amd as m
    sc = scenes.scene_body(H=16, W=16, spp=64, res=32, log2_T=16, seed=16541 + 9)
    fld, _ = m.upload_scene(sc, "cuda", m.F32, m.F32)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=ert_tau)
    n = sc.H * sc.W
    tgt = np.random.default_rng(1).random((n, 3)).astype(np.float32)
    tch = torch.zeros(n, m.saved_size(sc.spp), device="cuda")
    rgba = m.render(fld, pose, cam, sc.H, sc.W, sc.spp, opts, None, t_chunks=tch)
    grad_rgba = torch.empty(n, 4, device="cuda")
    m.mse_loss(rgba, torch.as_tensor(tgt, device="cuda"), grad_rgba)
    g_table = torch.zeros(sc.table.shape, device="cuda")
    g_w = [torch.zeros(w.shape, device="cuda") for w in sc.mlp]
    g_wc = torch.zeros(sc.logits.shape, device="cuda")
    m.render_backward(fld, pose, cam, sc.H, sc.W, sc.spp, opts, None, tch, grad_rgba, g_table, g_w, g_wc)
    g_logits = torch.zeros_like(g_wc)
    m.softmax_bwd(fld.weights, g_wc, g_logits)
    torch.cuda.synchronize()
    def oracle(s):
        field = O.Field.from_scene(s, requires_grad=True)
        G = O.bone_transforms(s.parents, s.rest_joints, s.axis_angle)
        o, d = O.camera_rays(s.cam, s.H, s.W)
        O.mse_loss(O.render_rays(field, G, o, d, s.spp), tgt).backward()
        return [field.table.grad.numpy(), field.logits.grad.numpy()] + [w.grad.numpy() for w in field.mlp]
    want, alt = oracle(sc), oracle(_one_ulp_pose(sc))
    got = [g_table.cpu().numpy(), g_logits.cpu().numpy()] + [w.cpu().numpy() for w in g_w]
    names = ["table", "logits"] + [f"w{k}" for k in range(len(g_w))]
    for name, a, b, b2 in zip(names, got, want, alt):
        r = _rel(a, b)
        print(f"  full-frame ert {ert_tau:g} {name:7s} rel-L2 {r:.3e}", flush=True)
        assert r <= 2e-3, name
        _elementwise(name, a, b, TAU[0], b2)


def test_render_fn_autograd_matches_oracle_gradient():
    # The adjoint behind torch.autograd: the loss is built and differentiated
    # by torch on the GPU, while the render and its backward are RenderFn
    # (the library's kernels).  dL/dW^c goes to the logits through the
    # library's softmax adjoint; tolerances as for the FP32 path above.
    import paper_2306_16541_amd as m
    sc = _scene()
    pid, tgt = _rays(sc)
    fld, _ = m.upload_scene(sc, "cuda", m.F32, m.F32)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    opts = m.make_opts(ert_tau=1e-6, stratified=True, seed=SEED)
    pid_t = torch.as_tensor(pid, device="cuda")
    tgt_t = torch.as_tensor(tgt, device="cuda")
    table = fld.table.requires_grad_(True)
    weights = fld.weights.requires_grad_(True)
    mlp = [w.requires_grad_(True) for w in fld.mlp]
    rgba = m.RenderFn.apply(table, weights, *mlp, (fld, pose, cam, sc.H, sc.W, sc.spp, opts, pid_t))
    loss = ((rgba[:, :3] - tgt_t) ** 2).mean()
    loss.backward()
    g_logits = torch.zeros_like(weights)
    m.softmax_bwd(weights.detach(), weights.grad, g_logits)
    torch.cuda.synchronize()
    lo, to, wo, logo, _ = oracle_grads(sc, pid, tgt)
    assert abs(float(loss.detach()) - lo) <= 1e-5 * abs(lo)
    groups = [("table", table.grad, to), ("logits", g_logits, logo)] + \
        [(f"w{k}", w.grad, b) for k, (w, b) in enumerate(zip(mlp, wo))]
    for name, a, b in groups:
        a = a.detach().cpu().numpy()
        r = _rel(a, b)
        print(f"  autograd {name:7s} rel-L2 {r:.3e}", flush=True)
        assert np.linalg.norm(b) > 0, name
        assert r <= 2e-3, name
        _elementwise(name, a, b, TAU[0])
