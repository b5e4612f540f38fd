"""Python binding of libmetanerf.so, the gfx950 posed-body volume renderer.

Argument marshalling only: every step of rendering and training runs in the
library's HIP kernels; PyTorch supplies device memory and the current
stream.  The entry points keep the C names without the `mnr_` prefix
(`render`, `render_backward`, `train_step`, `fk_bones`, ...).  Importing the
package fails loudly when the built library is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmetanerf.so")

MAX_BONES, MAX_LEVELS, MAX_LAYERS = 32, 16, 5
F32, F16, BF16 = 0, 1, 2
MNR_E_BUSY = -6
_TORCH_DT = {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}


class MnrError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                          "(or python paper_2306_16541_amd/build.py); there is no CPU fallback")
    return C.CDLL(LIB_PATH)


lib = _load()


class Field(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_feat", C.c_int32), ("log2_T", C.c_int32),
                ("level_res", C.c_int32 * MAX_LEVELS), ("box_min", C.c_float * 3), ("box_max", C.c_float * 3),
                ("table_dtype", C.c_int), ("table", C.c_void_p), ("n_layers", C.c_int32),
                ("width", C.c_int32 * (MAX_LAYERS + 1)), ("mlp_dtype", C.c_int), ("w", C.c_void_p * MAX_LAYERS),
                ("dense_packed", C.c_void_p), ("encoding", C.c_int32)]


class Motion(C.Structure):
    _fields_ = [("n_bones", C.c_int32), ("res", C.c_int32), ("box_min", C.c_float * 3),
                ("box_max", C.c_float * 3), ("weights", C.c_void_p), ("packed", C.c_void_p),
                ("res_w", C.c_void_p * 6), ("res_alpha", C.c_float)]


class Pose(C.Structure):
    _fields_ = [("n_joints", C.c_int32), ("parent", C.c_void_p), ("rest_joints", C.c_void_p),
                ("axis_angle", C.c_void_p), ("delta", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("R_wc", C.c_float * 9), ("T", C.c_float * 3), ("box_min", C.c_float * 3),
                ("box_max", C.c_float * 3)]


class Opts(C.Structure):
    _fields_ = [("ert_tau", C.c_float), ("bg", C.c_float * 3), ("stratified", C.c_int32), ("seed", C.c_uint64)]


_FP = C.c_void_p
_PL = C.POINTER(C.c_void_p)


class TrainState(C.Structure):
    _fields_ = ([("table_master", _FP), ("table_grad", _FP), ("table_m", _FP), ("table_v", _FP)] +
                [("w_master", _FP * MAX_LAYERS), ("w_grad", _FP * MAX_LAYERS), ("w_m", _FP * MAX_LAYERS),
                 ("w_v", _FP * MAX_LAYERS)] +
                [("logits", _FP), ("logits_grad", _FP), ("logits_m", _FP), ("logits_v", _FP),
                 ("weights_grad", _FP), ("rgba", _FP), ("grad_rgba", _FP), ("t_chunks", _FP), ("loss", _FP),
                 ("workspace", _FP), ("adjoint_ws", _FP), ("adjoint_ws_bytes", C.c_uint64),
                 ("res_master", _FP * 6), ("res_grad", _FP * 6), ("res_m", _FP * 6), ("res_v", _FP * 6),
                 ("lr_res", C.c_float),
                 ("lr_field", C.c_float), ("lr_motion", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                 ("eps", C.c_float), ("step", C.c_int32), ("train_motion", C.c_int32)])


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype, f.argtypes = res, args
    return f


_sig("mnr_status_str", C.c_char_p, [C.c_int])
_sig("mnr_last_error", C.c_char_p, [])
_sig("mnr_version", C.c_char_p, [])
_sig("mnr_fk_bones", C.c_int, [C.POINTER(Pose), C.c_void_p])
_RENDER_COMMON = [C.POINTER(Field), C.POINTER(Motion), C.POINTER(Pose), C.POINTER(Camera), C.c_int32, C.c_int32,
                  C.c_int32, C.POINTER(Opts), C.c_void_p, C.c_int32]
_sig("mnr_render", C.c_int, _RENDER_COMMON + [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p])
_sig("mnr_render_noalloc", C.c_int, _RENDER_COMMON + [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p])
_sig("mnr_render_backward", C.c_int, _RENDER_COMMON + [C.c_void_p, C.c_void_p, C.c_void_p, _PL, C.c_void_p,
                                                       C.c_void_p, _PL, C.c_void_p, C.c_void_p, C.c_uint64,
                                                       C.c_void_p])
_sig("mnr_adjoint_ws_bytes", C.c_uint64, [C.POINTER(Field), C.POINTER(Motion), C.c_int32, C.c_int32])
_sig("mnr_fk_backward", C.c_int, [C.POINTER(Pose), C.c_void_p, C.c_void_p, C.c_void_p])
_sig("mnr_mse_loss", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p])
_sig("mnr_softmax_fwd", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p])
_sig("mnr_softmax_bwd", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p])
_sig("mnr_adam_step", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_float,
                                C.c_float, C.c_float, C.c_int32, C.c_void_p, C.c_int, C.c_void_p])
_sig("mnr_convert", C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int64, C.c_void_p])
_sig("mnr_zero", C.c_int, [C.c_void_p, C.c_size_t, C.c_void_p])
_sig("mnr_motion_packed_bytes", C.c_uint64, [C.c_int32, C.c_int32])
_sig("mnr_field_packed_bytes", C.c_uint64, [C.POINTER(Field)])
_sig("mnr_field_pack", C.c_int, [C.POINTER(Field), C.c_void_p])
_sig("mnr_motion_pack", C.c_int, [C.POINTER(Motion), C.c_void_p])
_sig("mnr_probe_gather", C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, C.c_uint32, C.c_int32, C.c_int32, C.c_uint32,
                                   C.c_void_p, C.c_void_p])
_sig("mnr_probe_mfma", C.c_int, [C.c_int, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p])
_sig("mnr_probe_atomic", C.c_int, [C.c_void_p, C.c_uint32, C.c_int32, C.c_int32, C.c_int32, C.c_uint32, C.c_void_p])
_sig("mnr_probe_lds", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p])
_sig("mnr_probe_mlp", C.c_int, [C.POINTER(Field), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p])
_sig("mnr_train_step", C.c_int, _RENDER_COMMON + [C.c_void_p, C.POINTER(TrainState), C.c_void_p])

EXPORTED = ["mnr_status_str", "mnr_last_error", "mnr_version", "mnr_fk_bones", "mnr_render", "mnr_render_noalloc",
            "mnr_render_backward", "mnr_adjoint_ws_bytes",
            "mnr_mse_loss", "mnr_softmax_fwd", "mnr_softmax_bwd", "mnr_adam_step", "mnr_convert", "mnr_zero",
            "mnr_train_step", "mnr_motion_packed_bytes", "mnr_motion_pack", "mnr_field_packed_bytes", "mnr_field_pack",
            "mnr_probe_gather", "mnr_probe_mfma", "mnr_probe_atomic", "mnr_probe_lds", "mnr_probe_mlp", "mnr_fk_backward", "mnr_refiner_apply",
            "mnr_refiner_backward", "mnr_skel_cnn_act_floats", "mnr_skel_cnn_scratch_floats", "mnr_skel_cnn_forward",
            "mnr_skel_cnn_backward", "mnr_patch_rays"]


def check(status: int, what: str = "") -> None:
    if status != 0:
        msg = lib.mnr_last_error().decode()
        raise MnrError(f"{what}: {lib.mnr_status_str(status).decode()} ({status}): {msg}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


WORKSPACE_BYTES = 64
_WS = {}


def _workspace(device) -> torch.Tensor:
    """Work-queue counters for the render entry points, one buffer per
    (device, stream) so that calls on different streams never share one."""
    key = (torch.device(device).index, torch.cuda.current_stream(device).cuda_stream)
    if key not in _WS:
        _WS[key] = torch.zeros(WORKSPACE_BYTES // 4, dtype=torch.int32, device=device)
    return _WS[key]


def version() -> str:
    return lib.mnr_version().decode()


# ---------------------------------------------------------------------------
# Host-side descriptors (plain data, no arithmetic).
# ---------------------------------------------------------------------------

class PoseHost:
    """Keeps the host arrays of an mnr_pose alive.  delta: optional pose
    refiner adjustments [n, 3] (joint j rotates by R(delta_j) R(axis_angle_j))."""

    def __init__(self, parents, rest_joints, axis_angle, delta=None):
        self.parents = np.ascontiguousarray(parents, dtype=np.int32)
        self.rest = np.ascontiguousarray(rest_joints, dtype=np.float32)
        self.aa = np.ascontiguousarray(axis_angle, dtype=np.float32)
        self.delta = None if delta is None else np.ascontiguousarray(delta, dtype=np.float32).reshape(-1, 3)
        self.c = Pose(int(self.parents.shape[0]), self.parents.ctypes.data, self.rest.ctypes.data, self.aa.ctypes.data,
                      None if self.delta is None else self.delta.ctypes.data)


def make_camera(cam, box_min=(-0.5,) * 3, box_max=(0.5,) * 3) -> Camera:
    c = Camera()
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.R_wc[:] = [float(v) for v in np.asarray(cam.R_wc, dtype=np.float32).ravel()]
    c.T[:] = [float(v) for v in np.asarray(cam.T, dtype=np.float32).ravel()]
    c.box_min[:] = list(box_min)
    c.box_max[:] = list(box_max)
    return c


def make_opts(ert_tau=1e-6, bg=(0.0, 0.0, 0.0), stratified=False, seed=0) -> Opts:
    return Opts(float(ert_tau), (C.c_float * 3)(*bg), int(bool(stratified)), int(seed) & 0xFFFFFFFFFFFFFFFF)


def fk_bones(pose: PoseHost) -> np.ndarray:
    G = np.zeros((pose.parents.shape[0], 3, 4), dtype=np.float32)
    check(lib.mnr_fk_bones(C.byref(pose.c), G.ctypes.data), "fk_bones")
    return G


class DeviceField:
    """A canonical field resident on the GPU: grid table + MLP weights (in
    the dtypes the renderer reads) and the motion-weight volume.  With
    packed=True it also holds the packed copies of the dense grid levels and
    of the blend weights, which the renderer reads instead; call repack()
    after changing `table` or `weights` in place."""

    def __init__(self, table: torch.Tensor, mlp: Sequence[torch.Tensor], weights: torch.Tensor, level_res,
                 box_min=(-0.5,) * 3, box_max=(0.5,) * 3, n_feat: int = 2, packed: bool = True):
        self.table, self.mlp, self.weights = table, list(mlp), weights
        dt = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
        f = Field()
        f.n_levels, f.n_feat = int(table.shape[0]), n_feat
        f.log2_T = int(table.shape[1]).bit_length() - 1
        f.level_res[: len(level_res)] = [int(n) for n in level_res]
        f.box_min[:], f.box_max[:] = list(box_min), list(box_max)
        f.table_dtype, f.table = dt[table.dtype], table.data_ptr()
        f.n_layers = len(self.mlp)
        widths = [int(self.mlp[0].shape[1])] + [int(w.shape[0]) for w in self.mlp]
        f.width[: len(widths)] = widths
        f.mlp_dtype = dt[self.mlp[0].dtype]
        for k, w in enumerate(self.mlp):
            f.w[k] = w.data_ptr()
        self.dense_packed = None
        if packed:
            nb = int(lib.mnr_field_packed_bytes(C.byref(f)))
            if nb > 0:
                self.dense_packed = torch.empty(nb // 2, dtype=torch.float16, device=table.device)
                f.dense_packed = self.dense_packed.data_ptr()
        self.c = f
        m = Motion()
        m.n_bones, m.res = int(weights.shape[0]) - 1, int(weights.shape[-1])
        m.box_min[:], m.box_max[:] = list(box_min), list(box_max)
        m.weights = weights.data_ptr()
        self.packed = None
        if packed:
            nb = int(lib.mnr_motion_packed_bytes(m.res, m.n_bones))
            if nb == 0:
                raise MnrError(f"no packed copy for res {m.res}, {m.n_bones} bones")
            self.packed = torch.empty(nb // 4, dtype=torch.float32, device=weights.device)
            m.packed = self.packed.data_ptr()
        self.m = m
        self.repack()

    @classmethod
    def frequency(cls, mlp: Sequence[torch.Tensor], weights: torch.Tensor, box_min=(-0.5,) * 3, box_max=(0.5,) * 3,
                  packed: bool = True) -> "DeviceField":
        """The paper's own field (include/metanerf.h, MNR_ENC_FREQ): BF16
        W1..W5 of the 10-band positional encoding's skip MLP, no grid."""
        self = cls.__new__(cls)
        self.table, self.mlp, self.weights = None, list(mlp), weights
        f = Field()
        f.box_min[:], f.box_max[:] = list(box_min), list(box_max)
        f.encoding, f.mlp_dtype, f.n_layers = 1, BF16, 5
        f.width[:6] = [64, 64, 64, 64, 64, 4]
        for k, w in enumerate(self.mlp):
            f.w[k] = w.data_ptr()
        self.c = f
        self.dense_packed = None
        m = Motion()
        m.n_bones, m.res = int(weights.shape[0]) - 1, int(weights.shape[-1])
        m.box_min[:], m.box_max[:] = list(box_min), list(box_max)
        m.weights = weights.data_ptr()
        self.packed = None
        if packed:
            nb = int(lib.mnr_motion_packed_bytes(m.res, m.n_bones))
            self.packed = torch.empty(nb // 4, dtype=torch.float32, device=weights.device)
            m.packed = self.packed.data_ptr()
        self.m = m
        self.repack()
        return self

    def set_residual(self, weights: Sequence, w_omega, alpha: float = 4.0) -> None:
        """Turn on the residual motion network (include/metanerf.h, mnr_motion):
        FP32 W1..W5 and W_omega (arrays or tensors), stored as BF16 copies
        made by the library's conversion kernel; alpha = Hann window position."""
        dev = self.weights.device
        ws = [torch.as_tensor(w, dtype=torch.float32, device=dev) for w in list(weights) + [w_omega]]
        self.res_w = [convert(w.contiguous(), BF16) for w in ws]
        for k, w in enumerate(self.res_w):
            self.m.res_w[k] = w.data_ptr()
        self.m.res_alpha = float(alpha)

    def clear_residual(self) -> None:
        for k in range(6):
            self.m.res_w[k] = None
        self.res_w = None

    def repack(self) -> None:
        if self.dense_packed is not None:
            check(lib.mnr_field_pack(C.byref(self.c), _stream()), "field_pack")
        if self.packed is not None:
            check(lib.mnr_motion_pack(C.byref(self.m), _stream()), "motion_pack")


def softmax_fwd(logits: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    out = torch.empty_like(logits) if out is None else out
    check(lib.mnr_softmax_fwd(_ptr(logits), _ptr(out), int(logits.shape[0]), int(logits[0].numel()), _stream()),
          "softmax_fwd")
    return out


def softmax_bwd(weights, grad_weights, grad_logits) -> None:
    check(lib.mnr_softmax_bwd(_ptr(weights), _ptr(grad_weights), _ptr(grad_logits), int(weights.shape[0]),
                              int(weights[0].numel()), _stream()), "softmax_bwd")


def probe_gather(table: torch.Tensor, row_bytes: int, window_bytes: int, gathers_per_lane: int, n_lanes: int,
                 seed: int = 1, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Random-gather ceiling probe (include/metanerf_probe.h)."""
    out = torch.empty(n_lanes, dtype=torch.float32, device=table.device) if out is None else out
    check(lib.mnr_probe_gather(_ptr(table), table.numel() * table.element_size(), row_bytes, window_bytes,
                               gathers_per_lane, n_lanes, seed, _ptr(out), _stream()), "probe_gather")
    return out


def probe_atomic(acc: torch.Tensor, atomics_per_lane: int, n_lanes: int, run: int = 1, seed: int = 1) -> None:
    """Scattered float-atomic ceiling probe (include/metanerf_probe.h)."""
    check(lib.mnr_probe_atomic(_ptr(acc), acc.numel(), atomics_per_lane, n_lanes, run, seed, _stream()),
          "probe_atomic")


PROBE_LDS_OPS = ("float_atomic_add", "u32_atomic_add", "u64_atomic_add", "float_read_add_write", "store_b32")


def probe_lds(op: int, iters: int, n_blocks: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """LDS operation throughput probe (include/metanerf_probe.h); op indexes PROBE_LDS_OPS."""
    out = torch.empty(n_blocks * 1024, dtype=torch.float32, device="cuda") if out is None else out
    check(lib.mnr_probe_lds(op, iters, n_blocks, _ptr(out), _stream()), "probe_lds")
    return out


def probe_mfma(dtype: int, iters: int, n_blocks: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Dense MFMA-loop ceiling probe (include/metanerf_probe.h)."""
    out = torch.empty(n_blocks * 256, dtype=torch.float32, device="cuda") if out is None else out
    check(lib.mnr_probe_mfma(dtype, iters, n_blocks, _ptr(out), _stream()), "probe_mfma")
    return out


def probe_mlp(field, feat: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The field's MLP run unfused over feat [n, 32] (the MLP's dtype) into
    out [n, 4] = (rgb, sigma) (include/metanerf_probe.h)."""
    n = feat.shape[0]
    out = torch.empty(n, 4, dtype=torch.float32, device=feat.device) if out is None else out
    check(lib.mnr_probe_mlp(C.byref(field.c), _ptr(feat), n, _ptr(out), _stream()), "probe_mlp")
    return out


def convert(src: torch.Tensor, dtype: int) -> torch.Tensor:
    dst = torch.empty(src.shape, dtype=_TORCH_DT[dtype], device=src.device)
    check(lib.mnr_convert(_ptr(src), _ptr(dst), dtype, src.numel(), _stream()), "convert")
    return dst


def zero_(t: torch.Tensor) -> torch.Tensor:
    check(lib.mnr_zero(_ptr(t), t.numel() * t.element_size(), _stream()), "zero")
    return t


def upload_scene(sc, device="cuda", table_dtype: int = F32, mlp_dtype: int = F32, packed: bool = True):
    """Copy a scenes.Scene's arrays to the GPU and build a DeviceField
    (softmax and precision conversion run in the library's kernels).
    Returns (DeviceField, fp32 masters dict)."""
    table32 = torch.as_tensor(sc.table, device=device)
    w32 = [torch.as_tensor(w, device=device) for w in sc.mlp]
    logits = torch.as_tensor(sc.logits, device=device)
    weights = softmax_fwd(logits)
    table = table32 if table_dtype == F32 else convert(table32, table_dtype)
    mlp = w32 if mlp_dtype == F32 else [convert(w, mlp_dtype) for w in w32]
    fld = DeviceField(table, mlp, weights, sc.level_res, sc.box_min, sc.box_max, packed=packed)
    return fld, {"table": table32, "mlp": w32, "logits": logits}


def n_chunks(spp: int) -> int:
    return (spp + 63) // 64


def saved_size(spp: int) -> int:
    """Floats per ray of the forward's saved state (t_chunks): transmittance
    at each 64-sample chunk start plus the processed-sample count."""
    return n_chunks(spp) + 1


def render(field: DeviceField, pose: PoseHost, cam: Camera, H: int, W: int, spp: int, opts: Optional[Opts] = None,
           pixel_ids: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
           counter: Optional[torch.Tensor] = None, t_chunks: Optional[torch.Tensor] = None,
           dynamic: bool = True) -> torch.Tensor:
    """RGBA [n_rays, 4] (full frame: [H*W, 4], row-major pixels).  dynamic:
    pass a work-queue workspace (dynamic load balancing) or not (static split)."""
    n = H * W if pixel_ids is None else int(pixel_ids.numel())
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32, device=field.weights.device)
    check(lib.mnr_render(C.byref(field.c), C.byref(field.m), C.byref(pose.c), C.byref(cam), H, W, spp,
                         None if opts is None else C.byref(opts), _ptr(pixel_ids), n, _ptr(out), _ptr(t_chunks),
                         _ptr(counter), _ptr(_workspace(out.device)) if dynamic else None, _stream()), "render")
    return out


def render_noalloc(field: DeviceField, pose: PoseHost, cam: Camera, H: int, W: int, spp: int,
                   opts: Optional[Opts] = None, pixel_ids: Optional[torch.Tensor] = None,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """render() through mnr_render_noalloc: the library's own work-queue
    counters instead of a workspace (the library allocates nothing)."""
    n = H * W if pixel_ids is None else int(pixel_ids.numel())
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32, device=field.weights.device)
    check(lib.mnr_render_noalloc(C.byref(field.c), C.byref(field.m), C.byref(pose.c), C.byref(cam), H, W, spp,
                                 None if opts is None else C.byref(opts), _ptr(pixel_ids), n, _ptr(out), None, None,
                                 _stream()), "render_noalloc")
    return out


def adjoint_ws_bytes(field: DeviceField, n_rays: int, spp: int) -> int:
    """Bytes of the adjoint workspace (0: nothing to use it for)."""
    return int(lib.mnr_adjoint_ws_bytes(C.byref(field.c), C.byref(field.m), int(n_rays), int(spp)))


def adjoint_workspace(field: DeviceField, n_rays: int, spp: int) -> Optional[torch.Tensor]:
    """A device buffer for the adjoint (binned scatter of the table and
    blend-weight gradients, split adjoints, the ray list's processing order),
    or None when there is nothing to use it for."""
    nb = adjoint_ws_bytes(field, n_rays, spp)
    if nb == 0:
        return None
    return torch.empty(nb, dtype=torch.uint8, device=field.weights.device)


def render_backward(field: DeviceField, pose: PoseHost, cam: Camera, H: int, W: int, spp: int, opts: Optional[Opts],
                    pixel_ids: Optional[torch.Tensor], t_chunks: torch.Tensor, grad_rgba: torch.Tensor,
                    grad_table: Optional[torch.Tensor], grad_w: List[torch.Tensor], grad_weights: torch.Tensor,
                    grad_bones: Optional[torch.Tensor] = None, adjoint_ws: Optional[torch.Tensor] = None,
                    grad_res: Optional[List[torch.Tensor]] = None) -> None:
    """Accumulates the adjoint into the gradient buffers; grad_bones
    (optional, [n_bones, 3, 4]) receives dL/dG of the bone transforms.
    adjoint_ws (from adjoint_workspace): binned scatter of the table and
    blend-weight gradients instead of atomics, and the residual network's split
    adjoint, whose gradients (W1..W5, W_omega) go to grad_res.  The
    frequency-encoded field has no table (grad_table None) and needs
    adjoint_ws."""
    n = H * W if pixel_ids is None else int(pixel_ids.numel())
    gw = (C.c_void_p * len(grad_w))(*[g.data_ptr() for g in grad_w])
    gr = None if grad_res is None else C.cast((C.c_void_p * 6)(*[g.data_ptr() for g in grad_res]), _PL)
    nb = 0 if adjoint_ws is None else adjoint_ws.numel() * adjoint_ws.element_size()
    check(lib.mnr_render_backward(C.byref(field.c), C.byref(field.m), C.byref(pose.c), C.byref(cam), H, W, spp,
                                  None if opts is None else C.byref(opts), _ptr(pixel_ids), n, _ptr(t_chunks),
                                  _ptr(grad_rgba), _ptr(grad_table), C.cast(gw, _PL), _ptr(grad_weights),
                                  _ptr(grad_bones), gr, _ptr(_workspace(grad_rgba.device)), _ptr(adjoint_ws), nb,
                                  _stream()),
          "render_backward")


def fk_backward(pose: PoseHost, grad_G: np.ndarray):
    """Host adjoint of the forward kinematics: (dL/d delta, dL/d axis_angle),
    each [n, 3], from dL/dG [n, 3, 4]."""
    n = pose.parents.shape[0]
    g = np.ascontiguousarray(grad_G, dtype=np.float32)
    gd = np.zeros((n, 3), np.float32)
    ga = np.zeros((n, 3), np.float32)
    check(lib.mnr_fk_backward(C.byref(pose.c), g.ctypes.data, gd.ctypes.data, ga.ctypes.data), "fk_backward")
    return gd, ga


_sig("mnr_patch_rays", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_void_p])


def patch_rays(H: int, W: int, n_patches: int = 6, size: int = 20, seed: int = 0) -> np.ndarray:
    """Pixel ids of a patch ray batch (include/metanerf.h, mnr_patch_rays)."""
    out = np.zeros(n_patches * size * size, dtype=np.int32)
    check(lib.mnr_patch_rays(H, W, n_patches, size, seed, out.ctypes.data), "patch_rays")
    return out


class SkelCnn(C.Structure):
    _fields_ = [("latent", C.c_int32), ("channels", C.c_int32 * 6), ("z", C.c_void_p), ("w_fc", C.c_void_p),
                ("w", C.c_void_p * 5)]


_sig("mnr_skel_cnn_act_floats", C.c_uint64, [C.POINTER(SkelCnn)])
_sig("mnr_skel_cnn_scratch_floats", C.c_uint64, [C.POINTER(SkelCnn)])
_sig("mnr_skel_cnn_forward", C.c_int, [C.POINTER(SkelCnn), C.c_void_p, C.c_void_p, C.c_void_p])
_sig("mnr_skel_cnn_backward", C.c_int, [C.POINTER(SkelCnn), C.c_void_p, C.c_void_p, C.c_void_p, _PL, C.c_void_p,
                                        C.c_void_p])


class SkeletonCNN:
    """Skeleton-motion CNN (include/metanerf.h, mnr_skel_cnn) with its
    device buffers: latent z, weights, saved activations, gradient and Adam
    state; the blend-weight logits come out of forward()."""

    def __init__(self, z, w_fc, ws, device="cuda"):
        t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float32), device=device).contiguous()
        self.z, self.w_fc, self.ws = t(z), t(w_fc), [t(w) for w in ws]
        c = SkelCnn()
        c.latent = int(self.z.numel())
        c.channels[:] = [int(self.w_fc.shape[0])] + [int(w.shape[1]) for w in self.ws]
        c.z, c.w_fc = self.z.data_ptr(), self.w_fc.data_ptr()
        for k, w in enumerate(self.ws):
            c.w[k] = w.data_ptr()
        self.c = c
        na, ns = int(lib.mnr_skel_cnn_act_floats(C.byref(c))), int(lib.mnr_skel_cnn_scratch_floats(C.byref(c)))
        if na == 0:
            raise MnrError("skel_cnn: " + lib.mnr_last_error().decode())
        self.act = torch.zeros(na, device=device)
        self.scratch = torch.zeros(ns, device=device)
        self.params = [self.w_fc] + self.ws
        self.grads = [torch.zeros_like(p) for p in self.params]
        self.m1 = [torch.zeros_like(p) for p in self.params]
        self.m2 = [torch.zeros_like(p) for p in self.params]
        self.t = 0

    def forward(self, logits: Optional[torch.Tensor] = None) -> torch.Tensor:
        c5 = self.c.channels[5]
        logits = torch.empty(c5, 32, 32, 32, device=self.z.device) if logits is None else logits
        check(lib.mnr_skel_cnn_forward(C.byref(self.c), _ptr(self.act), _ptr(logits), _stream()), "skel_cnn_forward")
        return logits

    def backward(self, grad_logits: torch.Tensor) -> None:
        """Accumulate dL/dweights into self.grads."""
        gw = (C.c_void_p * 5)(*[g.data_ptr() for g in self.grads[1:]])
        check(lib.mnr_skel_cnn_backward(C.byref(self.c), _ptr(self.act), _ptr(grad_logits), _ptr(self.grads[0]),
                                        C.cast(gw, _PL), _ptr(self.scratch), _stream()), "skel_cnn_backward")

    def step(self, lr: float, beta1: float = 0.9, beta2: float = 0.99, eps: float = 1e-8) -> None:
        """Adam (the library's kernel) on every weight, then clear the gradients."""
        self.t += 1
        for p, g, m1, m2 in zip(self.params, self.grads, self.m1, self.m2):
            adam_step(p, g, m1, m2, lr, self.t, beta1, beta2, eps)
            zero_(g)


class Refiner(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("width", C.c_int32 * (MAX_LAYERS + 1)), ("w", C.c_void_p * MAX_LAYERS)]


_sig("mnr_refiner_apply", C.c_int, [C.POINTER(Refiner), C.c_int32, C.c_void_p, C.c_void_p])
_sig("mnr_refiner_backward", C.c_int, [C.POINTER(Refiner), C.c_int32, C.c_void_p, C.c_void_p, _PL])
_sig("mnr_refiner_adam", C.c_int, [C.POINTER(Refiner), C.c_int32, _PL, _PL, _PL, _PL, C.c_int32, C.c_float,
                                   C.c_float, C.c_float, C.c_float])


class PoseRefiner:
    """Host pose refiner MLP_theta (include/metanerf.h, mnr_refiner): FP32
    weights [out, in] held in numpy arrays, evaluated and differentiated by
    the library in double precision; Adam (beta 0.9/0.99) by the library on
    the host."""

    def __init__(self, weights: Sequence[np.ndarray], lr: float = 5e-5, beta1: float = 0.9, beta2: float = 0.99,
                 eps: float = 1e-8):
        self.w = [np.ascontiguousarray(w, dtype=np.float32) for w in weights]
        self.g = [np.zeros_like(w) for w in self.w]
        self.m1 = [np.zeros_like(w) for w in self.w]
        self.m2 = [np.zeros_like(w) for w in self.w]
        self.lr, self.b1, self.b2, self.eps, self.t = lr, beta1, beta2, eps, 0
        r = Refiner()
        r.n_layers = len(self.w)
        widths = [self.w[0].shape[1]] + [w.shape[0] for w in self.w]
        r.width[: len(widths)] = widths
        for k, w in enumerate(self.w):
            r.w[k] = w.ctypes.data
        self.c = r

    def apply(self, axis_angle) -> np.ndarray:
        om = np.ascontiguousarray(axis_angle, dtype=np.float32)
        d = np.zeros_like(om)
        check(lib.mnr_refiner_apply(C.byref(self.c), om.shape[0], om.ctypes.data, d.ctypes.data), "refiner_apply")
        return d

    def backward(self, axis_angle, grad_delta) -> None:
        """Accumulate dL/dW into self.g."""
        om = np.ascontiguousarray(axis_angle, dtype=np.float32)
        gd = np.ascontiguousarray(grad_delta, dtype=np.float32)
        ptrs = (C.c_void_p * len(self.g))(*[g.ctypes.data for g in self.g])
        check(lib.mnr_refiner_backward(C.byref(self.c), om.shape[0], om.ctypes.data, gd.ctypes.data,
                                       C.cast(ptrs, _PL)), "refiner_backward")

    def step(self) -> None:
        """Adam (the library's mnr_refiner_adam) on the accumulated gradients,
        which it then clears."""
        self.t += 1
        arr = lambda xs: C.cast((C.c_void_p * len(xs))(*[x.ctypes.data for x in xs]), _PL)
        check(lib.mnr_refiner_adam(C.byref(self.c), self.w[0].shape[1] // 3, arr(self.w), arr(self.g), arr(self.m1),
                                   arr(self.m2), self.t, self.lr, self.b1, self.b2, self.eps), "refiner_adam")


def mse_loss(rgba: torch.Tensor, target: torch.Tensor, grad_rgba: torch.Tensor,
             loss: Optional[torch.Tensor] = None) -> None:
    check(lib.mnr_mse_loss(_ptr(rgba), _ptr(target), int(rgba.shape[0]), _ptr(grad_rgba), _ptr(loss), _stream()),
          "mse_loss")


def adam_step(param, grad, m, v, lr, step, beta1=0.9, beta2=0.99, eps=1e-8, lowp=None) -> None:
    dt = F32 if lowp is None else {torch.float16: F16, torch.bfloat16: BF16}[lowp.dtype]
    check(lib.mnr_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), lr, beta1, beta2, eps, step,
                            _ptr(lowp), dt, _stream()), "adam_step")


class RenderFn(torch.autograd.Function):
    """Differentiable render of a ray batch: inputs are the field's table, MLP
    weights and canonical blend weights (W^c); the adjoint is the library's
    hand-written backward kernel."""

    @staticmethod
    def forward(ctx, table, weights, *mlp_and_cfg):
        *mlp, cfg = mlp_and_cfg
        field, pose, cam, H, W, spp, opts, pixel_ids = cfg
        n = H * W if pixel_ids is None else int(pixel_ids.numel())
        tch = torch.empty((n, saved_size(spp)), dtype=torch.float32, device=table.device)
        field.repack()  # weights may have changed since the last call
        out = render(field, pose, cam, H, W, spp, opts, pixel_ids, t_chunks=tch)
        ctx.cfg = cfg
        ctx.save_for_backward(tch)
        ctx.shapes = (table.shape, weights.shape, [w.shape for w in mlp])
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (tch,) = ctx.saved_tensors
        field, pose, cam, H, W, spp, opts, pixel_ids = ctx.cfg
        dev = tch.device
        g_table = torch.zeros(ctx.shapes[0], dtype=torch.float32, device=dev)
        g_weights = torch.zeros(ctx.shapes[1], dtype=torch.float32, device=dev)
        g_w = [torch.zeros(s, dtype=torch.float32, device=dev) for s in ctx.shapes[2]]
        render_backward(field, pose, cam, H, W, spp, opts, pixel_ids, tch, grad_out.contiguous().float(),
                        g_table, g_w, g_weights)
        return (g_table, g_weights, *g_w, None)


class Trainer:
    """Device-resident training state for mnr_train_step: FP32 masters, Adam
    moments, gradient and scratch buffers, and the low-precision copies the
    renderer reads.  Buffers are allocated once (by torch) and reused."""

    def __init__(self, table32: torch.Tensor, mlp32: Sequence[torch.Tensor], logits32: torch.Tensor, level_res,
                 table_dtype: int = F32, mlp_dtype: int = F32, max_rays: int = 8192, spp: int = 128,
                 lr_field: float = 5e-4, lr_motion: float = 5e-5, beta1: float = 0.9, beta2: float = 0.99,
                 eps: float = 1e-8, train_motion: bool = True, box_min=(-0.5,) * 3, box_max=(0.5,) * 3,
                 skel_cnn: Optional["SkeletonCNN"] = None, binned_scatter: bool = True,
                 residual: Optional[tuple] = None, lr_res: float = 5e-4):
        """skel_cnn: generate the blend-weight logits with the skeleton-motion
        CNN (logits32 is then ignored) and train its weights instead of free
        logits (lr_motion applies to them).  binned_scatter: give the adjoint
        a workspace for the binned scatter of the table and blend-weight
        gradients (else it adds them with atomics).  residual: (W1..W5, W_omega, alpha)
        of the residual motion network, trained with Adam at lr_res (the
        window position alpha is the caller's schedule: set_alpha)."""
        dev = table32.device
        self.table32 = table32.contiguous().clone()
        self.mlp32 = [w.contiguous().clone() for w in mlp32]
        self.cnn = skel_cnn
        self.logits = logits32.contiguous().clone() if skel_cnn is None else skel_cnn.forward()
        self.weights = softmax_fwd(self.logits)
        self.table = self.table32 if table_dtype == F32 else convert(self.table32, table_dtype)
        self.mlp = self.mlp32 if mlp_dtype == F32 else [convert(w, mlp_dtype) for w in self.mlp32]
        self.field = DeviceField(self.table, self.mlp, self.weights, level_res, box_min, box_max)
        self._setup(dev, max_rays, spp, lr_field, lr_motion, beta1, beta2, eps, train_motion,
                    binned_scatter or residual is not None, residual, lr_res)

    @classmethod
    def frequency(cls, mlp32: Sequence[torch.Tensor], logits32: torch.Tensor, max_rays: int = 8192, spp: int = 128,
                  lr_field: float = 5e-4, lr_motion: float = 5e-5, beta1: float = 0.9, beta2: float = 0.99,
                  eps: float = 1e-8, train_motion: bool = True, box_min=(-0.5,) * 3, box_max=(0.5,) * 3,
                  skel_cnn: Optional["SkeletonCNN"] = None, residual: Optional[tuple] = None,
                  lr_res: float = 5e-4) -> "Trainer":
        """Trainer of the paper's own field (DeviceField.frequency): FP32
        masters of W1..W5 (W4 [64][128]) with BF16 copies for the renderer,
        no grid table; its adjoint always uses the adjoint workspace."""
        self = cls.__new__(cls)
        dev = mlp32[0].device
        self.table32 = self.table = None
        self.mlp32 = [w.to(torch.float32).contiguous().clone() for w in mlp32]
        self.cnn = skel_cnn
        self.logits = logits32.contiguous().clone() if skel_cnn is None else skel_cnn.forward()
        self.weights = softmax_fwd(self.logits)
        self.mlp = [convert(w, BF16) for w in self.mlp32]
        self.field = DeviceField.frequency(self.mlp, self.weights, box_min, box_max)
        self._setup(dev, max_rays, spp, lr_field, lr_motion, beta1, beta2, eps, train_motion, True, residual, lr_res)
        return self

    def _setup(self, dev, max_rays, spp, lr_field, lr_motion, beta1, beta2, eps, train_motion, with_ws, residual,
               lr_res) -> None:
        self.res32 = None
        if residual is not None:
            rw, w_omega, alpha = residual
            self.res32 = [torch.as_tensor(np.asarray(w, dtype=np.float32), device=dev).contiguous().clone()
                          for w in list(rw) + [w_omega]]
            self.field.set_residual(self.res32[:5], self.res32[5], alpha)
        z = lambda t: torch.zeros_like(t, dtype=torch.float32)
        self.buf = {
            "w_grad": [z(w) for w in self.mlp32], "w_m": [z(w) for w in self.mlp32], "w_v": [z(w) for w in self.mlp32],
            "logits_grad": z(self.logits), "logits_m": z(self.logits), "logits_v": z(self.logits),
            "weights_grad": z(self.logits),
            "rgba": torch.zeros(max_rays, 4, device=dev), "grad_rgba": torch.zeros(max_rays, 4, device=dev),
            "t_chunks": torch.zeros(max_rays * saved_size(spp), device=dev), "loss": torch.zeros(1, device=dev),
            "workspace": torch.zeros(WORKSPACE_BYTES // 4, dtype=torch.int32, device=dev),
        }
        if self.table32 is not None:
            self.buf.update({"table_grad": z(self.table32), "table_m": z(self.table32), "table_v": z(self.table32)})
        self.max_rays, self.max_spp = max_rays, spp
        s = TrainState()
        b = self.buf
        if self.table32 is not None:
            s.table_master, s.table_grad, s.table_m, s.table_v = (
                t.data_ptr() for t in (self.table32, b["table_grad"], b["table_m"], b["table_v"]))
        for k in range(len(self.mlp32)):
            s.w_master[k], s.w_grad[k] = self.mlp32[k].data_ptr(), b["w_grad"][k].data_ptr()
            s.w_m[k], s.w_v[k] = b["w_m"][k].data_ptr(), b["w_v"][k].data_ptr()
        s.logits, s.logits_grad = self.logits.data_ptr(), b["logits_grad"].data_ptr()
        s.logits_m, s.logits_v = b["logits_m"].data_ptr(), b["logits_v"].data_ptr()
        s.weights_grad, s.rgba, s.grad_rgba = b["weights_grad"].data_ptr(), b["rgba"].data_ptr(), b["grad_rgba"].data_ptr()
        s.t_chunks, s.loss = b["t_chunks"].data_ptr(), b["loss"].data_ptr()
        s.workspace = b["workspace"].data_ptr()
        self.adjoint_ws = adjoint_workspace(self.field, max_rays, spp) if with_ws else None
        if self.adjoint_ws is not None:
            s.adjoint_ws, s.adjoint_ws_bytes = self.adjoint_ws.data_ptr(), self.adjoint_ws.numel()
        if self.res32 is not None:
            b["res_grad"], b["res_m"], b["res_v"] = ([z(w) for w in self.res32] for _ in range(3))
            for k in range(6):
                s.res_master[k], s.res_grad[k] = self.res32[k].data_ptr(), b["res_grad"][k].data_ptr()
                s.res_m[k], s.res_v[k] = b["res_m"][k].data_ptr(), b["res_v"][k].data_ptr()
        s.lr_res = lr_res
        s.lr_field, s.lr_motion, s.beta1, s.beta2, s.eps = lr_field, lr_motion, beta1, beta2, eps
        s.step, s.train_motion = 0, (2 if self.cnn is not None else 1) if train_motion else 0
        self.state = s

    def step(self, pose: PoseHost, cam: Camera, H: int, W: int, spp: int, pixel_ids: torch.Tensor,
             target: torch.Tensor, seed: int, ert_tau: float = 1e-6) -> None:
        n = int(pixel_ids.numel())
        if n > self.max_rays or spp > self.max_spp:
            raise ValueError("batch larger than the trainer's buffers")
        self.state.step += 1
        opts = make_opts(ert_tau=ert_tau, stratified=True, seed=seed)
        check(lib.mnr_train_step(C.byref(self.field.c), C.byref(self.field.m), C.byref(pose.c), C.byref(cam), H, W,
                                 spp, C.byref(opts), _ptr(pixel_ids), n, _ptr(target), C.byref(self.state), _stream()),
              "train_step")
        if self.cnn is not None and self.state.train_motion == 2:
            # dL/dlogits -> the CNN's weights; regenerate logits, W^c and its packed copy
            self.cnn.backward(self.buf["logits_grad"])
            self.cnn.step(self.state.lr_motion, self.state.beta1, self.state.beta2, self.state.eps)
            self.cnn.forward(self.logits)
            softmax_fwd(self.logits, out=self.weights)
            if self.field.packed is not None:
                check(lib.mnr_motion_pack(C.byref(self.field.m), _stream()), "motion_pack")

    def set_alpha(self, alpha: float) -> None:
        """Window position of the residual network's frequency bands."""
        self.field.m.res_alpha = float(alpha)

    def loss(self) -> float:
        return float(self.buf["loss"].item())

    def state_dict(self) -> dict:
        b = self.buf
        sd = {"step": int(self.state.step), "mlp": [w.cpu() for w in self.mlp32],
              "logits": self.logits.cpu(), "w_m": [t.cpu() for t in b["w_m"]], "w_v": [t.cpu() for t in b["w_v"]],
              "logits_m": b["logits_m"].cpu(), "logits_v": b["logits_v"].cpu()}
        if self.table32 is not None:
            sd.update({"table": self.table32.cpu(), "table_m": b["table_m"].cpu(), "table_v": b["table_v"].cpu()})
        return sd

    def load_state_dict(self, sd: dict) -> None:
        """Restore masters and Adam moments in place, then refresh the
        renderer's copies (softmax and precision conversion kernels)."""
        b = self.buf
        if self.table32 is not None:
            self.table32.copy_(sd["table"])
        for w, v in zip(self.mlp32, sd["mlp"]):
            w.copy_(v)
        self.logits.copy_(sd["logits"])
        for key in (("table_m", "table_v") if self.table32 is not None else ()) + ("logits_m", "logits_v"):
            b[key].copy_(sd[key])
        for key in ("w_m", "w_v"):
            for t, v in zip(b[key], sd[key]):
                t.copy_(v)
        self.state.step = int(sd["step"])
        softmax_fwd(self.logits, out=self.weights)
        if self.table is not None and self.table is not self.table32:
            check(lib.mnr_convert(_ptr(self.table32), _ptr(self.table), self.field.c.table_dtype, self.table32.numel(),
                                  _stream()), "convert")
        for w32, w in zip(self.mlp32, self.mlp):
            if w is not w32:
                check(lib.mnr_convert(_ptr(w32), _ptr(w), self.field.c.mlp_dtype, w32.numel(), _stream()), "convert")
        self.field.repack()


# ---------------------------------------------------------------------------
# Render server (include/metanerf_server.h).
# ---------------------------------------------------------------------------

class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
                ("failed", C.c_uint64), ("ticks", C.c_uint64), ("tiles", C.c_uint64), ("queued", C.c_int32),
                ("admitted", C.c_int32), ("tracked", C.c_int32), ("resident_bytes", C.c_uint64),
                ("inflight_bytes", C.c_uint64)]


_sig("mnr_server_create", C.c_int, [C.c_uint64, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)])
_sig("mnr_server_add_user", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Field), C.POINTER(Motion)])
_sig("mnr_server_submit", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Pose), C.POINTER(Camera), C.c_int32, C.c_int32,
                                    C.c_int32, C.POINTER(Opts), C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)])
_sig("mnr_server_poll", C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.c_void_p])
_sig("mnr_server_wait", C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, C.c_void_p])
_sig("mnr_server_get_stats", C.c_int, [C.c_void_p, C.POINTER(ServerStats)])
_sig("mnr_server_destroy", C.c_int, [C.c_void_p])
EXPORTED += ["mnr_server_create", "mnr_server_add_user", "mnr_server_submit", "mnr_server_poll", "mnr_server_wait",
             "mnr_server_get_stats", "mnr_server_destroy"]


class Server:
    """Continuous-batching render server with per-user resident fields."""

    def __init__(self, mem_budget: int, max_slots: int = 32, tiles_per_tick: int = 1024):
        h = C.c_void_p()
        check(lib.mnr_server_create(int(mem_budget), int(max_slots), int(tiles_per_tick), C.byref(h)), "server_create")
        self.h = h
        self._keep = {}

    def add_user(self, user: int, field: DeviceField) -> None:
        check(lib.mnr_server_add_user(self.h, int(user), C.byref(field.c), C.byref(field.m)), "server_add_user")
        self._keep[("user", user)] = field

    def submit(self, user: int, pose: PoseHost, cam: Camera, H: int, W: int, spp: int, out: torch.Tensor,
               opts: Optional[Opts] = None) -> int:
        """Queue a frame into `out`.  The server's write is ordered after the
        work queued on torch's current stream, and `out` is kept alive here
        until poll or wait reports the request finished."""
        t = C.c_uint64()
        check(lib.mnr_server_submit(self.h, int(user), C.byref(pose.c), C.byref(cam), H, W, spp,
                                    None if opts is None else C.byref(opts), _ptr(out), _stream(), C.byref(t)),
              "server_submit")
        self._keep[("out", int(t.value))] = out
        return int(t.value)

    def poll(self, ticket: int):
        done = C.c_int32()
        ts = (C.c_int64 * 4)()
        st = lib.mnr_server_poll(self.h, C.c_uint64(ticket), C.byref(done), ts)
        if done.value:
            self._keep.pop(("out", ticket), None)
        check(st, "server_poll")
        return bool(done.value), list(ts)

    def wait(self, ticket: int, timeout_ms: int = 60000):
        ts = (C.c_int64 * 4)()
        st = lib.mnr_server_wait(self.h, C.c_uint64(ticket), int(timeout_ms), ts)
        if st != MNR_E_BUSY:
            self._keep.pop(("out", ticket), None)
        check(st, "server_wait")
        return list(ts)

    def stats(self) -> dict:
        s = ServerStats()
        check(lib.mnr_server_get_stats(self.h, C.byref(s)), "server_stats")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self) -> None:
        if self.h:
            check(lib.mnr_server_destroy(self.h), "server_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
