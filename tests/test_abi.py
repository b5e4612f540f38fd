"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, host FK matches the oracle, and invalid calls are rejected
on the host before any launch."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle
import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2306_16541_amd as m
    return m


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"\b(mnr_\w+)\s*\(", txt))
    return names


def test_every_declared_symbol_is_exported():
    m = _lib()
    names = _declared()
    assert "mnr_render" in names and "mnr_train_step" in names
    for n in sorted(names):
        assert hasattr(m.lib, n), n
    assert set(m.EXPORTED) <= names


def test_host_fk_matches_oracle():
    m = _lib()
    parents, rest = scenes.skeleton()
    for seed in (1, 2, 3):
        aa = scenes.pose(seed, 0.3)
        G = m.fk_bones(m.PoseHost(parents, rest, aa))
        Go = oracle.bone_transforms(parents, rest, aa).numpy()
        assert np.abs(G - Go).max() < 2e-7


def _args(sc):
    m = _lib()
    f = m.Field()
    f.n_levels, f.n_feat, f.log2_T = 16, 2, sc.log2_T
    f.level_res[:16] = [int(v) for v in sc.level_res]
    f.box_min[:], f.box_max[:] = [-0.5] * 3, [0.5] * 3
    f.table_dtype, f.table = 0, 0x1000                # never dereferenced: rejected first
    f.n_layers = len(sc.mlp)
    widths = [32] + [w.shape[0] for w in sc.mlp]
    f.width[: len(widths)] = widths
    f.mlp_dtype = 0
    for k in range(len(sc.mlp)):
        f.w[k] = 0x2000
    mo = m.Motion(24, sc.res, (C.c_float * 3)(-0.5, -0.5, -0.5), (C.c_float * 3)(0.5, 0.5, 0.5), 0x3000)
    pose = m.PoseHost(sc.parents, sc.rest_joints, sc.axis_angle)
    cam = m.make_camera(sc.cam)
    return m, f, mo, pose, cam


def _render(m, f, mo, pose, cam, H=8, W=8, spp=8, opts=None, pid=None, n=64, out=0x4000):
    return m.lib.mnr_render(C.byref(f), C.byref(mo), C.byref(pose.c), C.byref(cam), H, W, spp,
                            None if opts is None else C.byref(opts), pid, n, out, None, None, None, None)


def test_invalid_calls_are_rejected_before_launch():
    sc = scenes.scene_small(H=8, W=8, spp=8)
    m, f, mo, pose, cam = _args(sc)
    assert _render(m, f, mo, pose, cam, spp=0) == -2
    assert _render(m, f, mo, pose, cam, spp=2000) == -2
    assert _render(m, f, mo, pose, cam, n=63) == -2                       # full frame needs H*W rays
    assert _render(m, f, mo, pose, cam, out=None) == -1
    f.width[1] = 48
    assert _render(m, f, mo, pose, cam) == -2
    assert "hidden width" in m.lib.mnr_last_error().decode()
    f.width[1] = 64
    f.mlp_dtype = 1                                                        # F16 MLP: unsupported
    assert _render(m, f, mo, pose, cam) == -3
    f.mlp_dtype = 0
    bad = sc.axis_angle.copy(); bad[3, 1] = math.nan
    assert _render(m, f, mo, m.PoseHost(sc.parents, sc.rest_joints, bad), cam) == -1
    mo.n_bones = 23
    assert _render(m, f, mo, pose, cam) == -2
    mo.n_bones = 24
    cam.fx = -1.0
    assert _render(m, f, mo, pose, cam) == -1
    opts = m.make_opts(ert_tau=-1.0)
    cam.fx = 16.0
    assert _render(m, f, mo, pose, cam, opts=opts) == -1
    assert m.lib.mnr_zero(None, 16, None) == -1
    assert m.lib.mnr_convert(None, None, 1, 4, None) == -1
    assert m.lib.mnr_adam_step(None, None, None, None, 4, 1e-3, 0.9, 0.99, 1e-8, 1, None, 0, None) == -1
    mo.packed = 0x5008                                                     # packed copy not 16-byte aligned
    assert _render(m, f, mo, pose, cam) == -1
    mo.packed = 0
    assert m.lib.mnr_motion_pack(C.byref(mo), None) == -1                  # no packed buffer
    assert m.lib.mnr_field_pack(C.byref(f), None) == -1                    # no dense_packed buffer
    f.dense_packed = 0x6004                                                # not 16-byte aligned
    assert _render(m, f, mo, pose, cam) == -1
    assert m.lib.mnr_field_packed_bytes(C.byref(f)) == 0
    f.dense_packed = 0
    dense = sum((n + 1) * n * n * 32 for n in sc.level_res if (n + 1) ** 3 <= 1 << sc.log2_T)
    assert dense > 0 and m.lib.mnr_field_packed_bytes(C.byref(f)) == dense   # F32 groups: 4 rows x 8 B
    assert m.lib.mnr_probe_gather(None, 64, 4, 0, 8, 256, 1, None, None) == -1
    assert m.lib.mnr_probe_gather(0x1000, 64, 12, 0, 8, 256, 1, 0x2000, None) == -2
    assert m.lib.mnr_probe_gather(0x1000, 64, 4, 0, 12, 256, 1, 0x2000, None) == -2
    assert m.lib.mnr_probe_gather(0x1000, 64, 4, 128, 8, 256, 1, 0x2000, None) == -2   # window > table
    assert m.lib.mnr_probe_mfma(1, 10, 1, 0x2000, None) == -3               # F16: unsupported
    mo.res_w[0], mo.res_alpha = 0x7000, 4.0                                # residual network, F32 MLP
    for k in range(1, 6):
        mo.res_w[k] = 0x7000 + 0x1000 * k
    assert _render(m, f, mo, pose, cam) == -7                              # needs the BF16 path
    assert "BF16" in m.lib.mnr_last_error().decode()
    mo.res_w[3] = None
    assert _render(m, f, mo, pose, cam) == -1                              # a null residual weight
    mo.res_w[3] = 0xA000
    f.mlp_dtype = 2
    gw = (C.c_void_p * 4)(0x100, 0x200, 0x300, 0x400)
    assert m.lib.mnr_render_backward(C.byref(f), C.byref(mo), C.byref(pose.c), C.byref(cam), 8, 8, 8, None, None, 64,
                                     0x4000, 0x4100, 0x4200, C.cast(gw, m._PL), 0x4300, None, None, None, None,
                                     0, None) == -1
    assert "grad_res" in m.lib.mnr_last_error().decode()
    gr = (C.c_void_p * 6)(*[0x5000 + 0x100 * k for k in range(6)])
    assert m.lib.mnr_render_backward(C.byref(f), C.byref(mo), C.byref(pose.c), C.byref(cam), 8, 8, 8, None, None, 64,
                                     0x4000, 0x4100, 0x4200, C.cast(gw, m._PL), 0x4300, None, C.cast(gr, m._PL),
                                     None, None, 0, None) == -1
    assert "workspace" in m.lib.mnr_last_error().decode()
    f.mlp_dtype = 0
    for k in range(6):
        mo.res_w[k] = None
    f.encoding = 7                                                         # unknown encoding
    assert _render(m, f, mo, pose, cam) == -1
    f.encoding = 1                                                         # frequency field, F32 MLP
    f.n_layers, f.w[4] = 5, 0x2400
    f.width[:6] = [64, 64, 64, 64, 64, 4]
    assert _render(m, f, mo, pose, cam) == -7
    f.mlp_dtype = 2
    f.width[3] = 32
    assert _render(m, f, mo, pose, cam) == -2                              # widths are fixed
    f.width[3] = 64
    assert m.lib.mnr_field_packed_bytes(C.byref(f)) == 0                   # no grid, nothing to pack
    f.encoding, f.mlp_dtype, f.n_layers = 0, 0, len(sc.mlp)
    widths = [32] + [w.shape[0] for w in sc.mlp]
    f.width[: len(widths)] = widths
    assert m.lib.mnr_probe_atomic(None, 16, 1, 256, 1, 1, None) == -1
    assert m.lib.mnr_probe_atomic(0x2000, 16, 1, 256, 65, 1, None) == -2      # run > 64
    assert m.lib.mnr_probe_mlp(None, 0x1000, 64, 0x2000, None) == -1
    assert m.lib.mnr_probe_mlp(C.byref(f), None, 64, 0x2000, None) == -1
    assert m.lib.mnr_probe_mlp(C.byref(f), 0x1008, 64, 0x2000, None) == -1   # not 16-byte aligned
    assert m.lib.mnr_probe_mlp(C.byref(f), 0x1000, -1, 0x2000, None) == -2
    assert m.lib.mnr_probe_mlp(C.byref(f), None, 0, None, None) == 0         # nothing to do, no launch
    f.mlp_dtype = 1
    assert m.lib.mnr_probe_mlp(C.byref(f), 0x1000, 64, 0x2000, None) == -3   # F16 MLP
    f.mlp_dtype = 0
    f.width[1] = 48
    assert m.lib.mnr_probe_mlp(C.byref(f), 0x1000, 64, 0x2000, None) == -2
    f.width[1] = 64
    f.encoding = 1
    assert m.lib.mnr_probe_mlp(C.byref(f), 0x1000, 64, 0x2000, None) == -7   # frequency field
    f.encoding = 0


def test_packed_motion_size():
    m = _lib()
    assert m.lib.mnr_motion_packed_bytes(32, 24) == 24 * 32 * 33 * 33 * 16
    assert m.lib.mnr_motion_packed_bytes(256, 24) == 24 * 256 * 257 * 257 * 16
    assert m.lib.mnr_motion_packed_bytes(257, 24) == 0                      # beyond the 32-bit offset range
    assert m.lib.mnr_motion_packed_bytes(32, 0) == 0


def test_status_strings():
    m = _lib()
    for s, txt in [(0, "ok"), (-1, "invalid argument"), (-6, "busy")]:
        assert m.lib.mnr_status_str(s).decode() == txt


def test_bench_refuses_more_than_one_gpu():
    # One GPU only: asking bench.py for several exits with status 2 and a
    # message before any device work.
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_build_script_loads_without_the_package():
    # __graft_entry__.build() must work on a checkout with no built library:
    # the build script is loaded by path and must not import the package
    # (which loads libmetanerf.so at import).
    import subprocess
    import sys
    code = ("import sys, importlib.util\n"
            "sys.modules['paper_2306_16541_amd'] = None\n"
            f"spec = importlib.util.spec_from_file_location('_b', {os.path.join(ROOT, 'paper_2306_16541_amd', 'build.py')!r})\n"
            "mod = importlib.util.module_from_spec(spec); spec.loader.exec_module(mod)\n"
            "assert callable(mod.build)\n"
            "import __graft_entry__ as g\n"
            "import inspect; assert 'spec_from_file_location' in inspect.getsource(g.build)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0, r.stderr


def _scatter_ws_bytes(n_rays, spp, per_sample, n_keys):
    # records (12 bytes, twice), per-tile bin histograms, per-bin counts in
    # 64 tile segments, per-bin totals, places and first items, the items'
    # bins (a bin of t records is ceil(t / 65536) items) and their count,
    # each part 256-byte aligned
    a256 = lambda b: (b + 255) // 256 * 256
    cap = n_rays * spp * per_sample
    n_bins = -(-n_keys // (1 << 12))      # slices of 2^12 rows
    tiles = -(-cap // 8192)
    items = n_bins + -(-cap // 65536)
    return (a256(256) + 2 * a256(cap * 4) + 2 * a256(cap * 8) + a256(n_bins * tiles * 4) + a256(64 * n_bins * 4) +
            3 * a256(n_bins * 4) + a256(items * 4) + a256(4))


def test_adjoint_workspace_size_and_checks():
    # Adjoint workspace: binned-scatter room for 8 records per sample and
    # keyed grid level (the dense levels are keyed too while hashed levels x
    # T plus dense rows fit the key space) and 4 per sample and bone (the
    # blend-weight gradient's corner pairs, keyed from a multiple of 2^14
    # when res is a power of two); with a residual network or the
    # frequency-encoded field, 21 floats per sample slot and 64 floats of
    # bias gradient, and for the frequency-encoded field 512 bytes of saved
    # activations per slot; then 4 bytes per ray of processing order
    # (include/metanerf.h).
    m = _lib()
    sc = scenes.scene_body(H=8, W=8, spp=8, res=8, log2_T=19)
    _, f, mo, pose, cam = _args(sc)
    assert (mo.n_bones, mo.res) == (24, 8)
    nh = sum(1 for n in sc.level_res if (int(n) + 1) ** 3 > 1 << 19)
    assert nh == 9
    a256 = lambda b: (b + 255) // 256 * 256
    nk = len(sc.level_res)                 # every level is keyed
    dense_rows = sum((int(n) + 1) ** 3 for n in sc.level_res if (int(n) + 1) ** 3 <= 1 << 19)
    assert dense_rows == 4913 + 9261 + 17576 + 35937 + 68921 + 132651 + 274625
    table_keys = (nh << 19) + dense_rows   # hashed levels' keys, then the dense levels' rows
    wc0 = -(-table_keys // (1 << 14)) << 14
    n_keys = wc0 + 24 * 8 ** 3
    for n_rays, spp in ((8192, 128), (100, 7)):
        want = _scatter_ws_bytes(n_rays, spp, nk * 8 + 24 * 4, n_keys)
        order = a256(n_rays * 4)
        assert m.lib.mnr_adjoint_ws_bytes(C.byref(f), C.byref(mo), n_rays, spp) == want + order
        for k in range(6):
            mo.res_w[k] = 0x7000 + 0x100 * k
        split = a256(21 * n_rays * -(-spp // 64) * 64 * 4) + 256
        assert m.lib.mnr_adjoint_ws_bytes(C.byref(f), C.byref(mo), n_rays, spp) == want + split + order
        for k in range(6):
            mo.res_w[k] = None
    mo.res = 6          # not a power of two: the blend-weight gradient keeps atomics
    assert (m.lib.mnr_adjoint_ws_bytes(C.byref(f), C.byref(mo), 100, 7) ==
            _scatter_ws_bytes(100, 7, nk * 8, table_keys) + a256(400))
    mo.res = 8
    ff = m.Field()      # the frequency-encoded field: blend-weight records, split scratch and saved activations
    ff.encoding, ff.mlp_dtype, ff.n_layers = 1, m.BF16, 5
    ff.width[:6] = [64, 64, 64, 64, 64, 4]
    ff.box_min[:], ff.box_max[:] = [-0.5] * 3, [0.5] * 3
    for k in range(5):
        ff.w[k] = 0x9000 + 0x100 * k
    for n_rays, spp in ((8192, 128), (100, 7)):
        chunks = n_rays * -(-spp // 64)
        want = (_scatter_ws_bytes(n_rays, spp, 24 * 4, 24 * 8 ** 3) + a256(21 * chunks * 64 * 4) + 256 +
                chunks * 4 * 4 * 2 * 64 * 16 + a256(n_rays * 4))
        assert m.lib.mnr_adjoint_ws_bytes(C.byref(ff), C.byref(mo), n_rays, spp) == want
    assert m.lib.mnr_adjoint_ws_bytes(C.byref(f), C.byref(mo), 1 << 20, 1024) == 0   # >= 2^31 records
    f.log2_T = 24       # the largest table: its 4 hashed levels fill the key space (4096 slices of 2^14 rows), the rest keeps atomics
    assert m.lib.mnr_adjoint_ws_bytes(C.byref(f), C.byref(mo), 64, 8) > 0
    f.log2_T = 19
    gw = (C.c_void_p * 4)(0x100, 0x200, 0x300, 0x400)
    # a misaligned workspace and a too-small one are rejected before any launch
    for ws, nb, code in ((0x12345, 1 << 30, -1), (0x100000, 1024, -2)):
        r = m.lib.mnr_render_backward(C.byref(f), C.byref(mo), C.byref(pose.c), C.byref(cam), 8, 8, 8, None, None,
                                      64, 0x4000, 0x4100, 0x4200, C.cast(gw, m._PL), 0x4300, None, None, None, ws,
                                      nb, None)
        assert r == code, (r, m.lib.mnr_last_error().decode())
