"""Thin Python binding over the C ABI: torch supplies device memory and the
current stream; every step of the hot path runs in the HIP library."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi as A


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _device(device=None) -> torch.device:
    return torch.device(device if device is not None else "cuda")


# ---------------------------------------------------------------- networks
@dataclass
class PackedMLP:
    shape: dict
    dtype: str
    blob: torch.Tensor   # uint8 device tensor

    def struct(self) -> A.Mlp:
        s = A.MlpShape(**{k: int(v) for k, v in self.shape.items()})
        return A.Mlp(shape=s, dtype=A.DTYPES[self.dtype], blob=self.blob.data_ptr())


def mlp_shape(in_kind="xyz", enc_L=10, width=256, n_hidden=8, n_out=1, rgb_width=0, dir_L=0) -> dict:
    return dict(in_kind=A.IN_KINDS[in_kind] if isinstance(in_kind, str) else int(in_kind), enc_L=enc_L,
                width=width, n_hidden=n_hidden, n_out=n_out, rgb_width=rgb_width, dir_L=dir_L)


def packed_bytes(shape: dict, dtype: str) -> int:
    lib = A.load()
    s = A.MlpShape(**{k: int(v) for k, v in shape.items()})
    n = lib.nedf_mlp_packed_bytes(C.byref(s), A.DTYPES[dtype])
    if n == 0:
        raise A.NedfError(A.STATUS and 2, "nedf_mlp_packed_bytes", lib.nedf_last_error().decode())
    return int(n)


def pack_host(W, b, shape: dict, dtype: str = "bf16", fp8_scales=None) -> np.ndarray:
    """Pack float32 layers (PyTorch [out, in] layout, hidden layers, head,
    then colour layers) into the blob layout; returns host bytes."""
    lib = A.load()
    s = A.MlpShape(**{k: int(v) for k, v in shape.items()})
    n = packed_bytes(shape, dtype)
    Ws = [np.ascontiguousarray(w, dtype=np.float32) for w in W]
    bs = [np.ascontiguousarray(x, dtype=np.float32) for x in b]
    Wp = (C.c_void_p * len(Ws))(*[w.ctypes.data for w in Ws])
    bp = (C.c_void_p * len(bs))(*[x.ctypes.data for x in bs])
    out = np.zeros(n, dtype=np.uint8)
    sc = None
    if fp8_scales is not None:
        sc = np.ascontiguousarray(fp8_scales, dtype=np.float32)
    A.check(lib.nedf_pack_mlp(C.byref(s), A.DTYPES[dtype], Wp, bp,
                              None if sc is None else sc.ctypes.data, out.ctypes.data, n), "nedf_pack_mlp")
    return out


def pack_mlp(W, b, shape: dict, dtype: str = "bf16", device=None, fp8_scales=None) -> PackedMLP:
    host = pack_host(W, b, shape, dtype, fp8_scales)
    blob = torch.from_numpy(host).to(_device(device))
    return PackedMLP(shape=dict(shape), dtype=dtype, blob=blob)


# ---------------------------------------------------------------- objects and scenes
@dataclass
class ObjectSpec:
    field: str = "sphere"
    bound: float = 1.0
    param: tuple = (0, 0, 0, 0, 0, 0)
    sigma_mode: str = "softplus"
    density: PackedMLP | None = None
    nedf: PackedMLP | None = None

    def struct(self) -> A.Object:
        o = A.Object()
        o.field = A.FIELDS[self.field]
        o.sigma_mode = A.SIGMA_MODES[self.sigma_mode]
        o.bound = float(self.bound)
        p = list(self.param) + [0.0] * (6 - len(self.param))
        for i in range(6):
            o.param[i] = float(p[i])
        if self.density is not None:
            o.density = self.density.struct()
        if self.nedf is not None:
            o.nedf = self.nedf.struct()
        return o


def object_from_model(model, dtype: str = "bf16", device=None, nedf_model=None) -> ObjectSpec:
    """Build an ObjectSpec from a model description with the attributes
    ``kind``, ``bound``, ``params``, ``trunk`` (W, b lists) and ``rgb``."""
    p = model.params
    if model.kind == "sphere":
        return ObjectSpec("sphere", model.bound, (p["sigma_max"], p["radius"], p["width"]))
    if model.kind == "slab":
        return ObjectSpec("slab", model.bound, (p["sigma0"], p["z0"], p["z1"]))
    if model.kind in ("mlp", "nerf"):
        tr = model.trunk
        width = tr.W[0].shape[0]
        n_hidden = len(tr.W) - 1
        rgb_w = 0
        W, b = list(tr.W), list(tr.b)
        if model.kind == "nerf" and model.rgb is not None:
            rgb_w = model.rgb.W[0].shape[0]
            W += list(model.rgb.W)
            b += list(model.rgb.b)
        shape = mlp_shape("xyz", p["enc_L"], width, n_hidden, 1, rgb_w, p.get("dir_L", 0))
        dens = pack_mlp(W, b, shape, dtype, device)
        if p["sigma_mode"] == "sdf":
            mode, param = "sdf", (p["sigma_max"], p["width"], p["sdf_shape"])
        else:
            mode = "softplus_masked" if p.get("masked", False) else "softplus"
            param = ()
        spec = ObjectSpec("mlp", model.bound, param, mode, dens)
        if nedf_model is not None:
            t = nedf_model.trunk
            nshape = mlp_shape("pluecker", nedf_model.params["enc_L"], t.W[0].shape[0], len(t.W) - 1, 2)
            spec.nedf = pack_mlp(t.W, t.b, nshape, dtype, device)
        return spec
    raise ValueError(model.kind)


@dataclass
class SceneGPU:
    objects: list
    inst_object: torch.Tensor     # int32 [n]
    inst_G: torch.Tensor          # float64 [n, 13]
    inst_w2l: torch.Tensor        # float32 [n, 16]
    _structs: object = field(default=None, repr=False)

    def struct(self) -> A.Scene:
        arr = (A.Object * len(self.objects))(*[o.struct() for o in self.objects])
        self._structs = arr
        return A.Scene(n_objects=len(self.objects), objects=C.cast(arr, C.POINTER(A.Object)),
                       n_inst=int(self.inst_object.numel()), inst_object=self.inst_object.data_ptr(),
                       inst_w2l=self.inst_w2l.data_ptr())


def compose_transforms(inst_G: torch.Tensor) -> torch.Tensor:
    lib = A.load()
    n = inst_G.shape[0]
    w2l = torch.empty((n, A.W2L_FLOATS), dtype=torch.float32, device=inst_G.device)
    A.check(lib.nedf_compose_transforms(inst_G.data_ptr(), n, w2l.data_ptr(), _stream()),
            "nedf_compose_transforms")
    return w2l


def make_scene(objects, instances, device=None) -> SceneGPU:
    """``instances``: iterable with attributes model (object index), R, T, s."""
    dev = _device(device)
    G = np.zeros((len(instances), 13), np.float64)
    ids = np.zeros(len(instances), np.int32)
    for k, inst in enumerate(instances):
        G[k, 0:9] = np.asarray(inst.R, np.float64).reshape(9)
        G[k, 9:12] = np.asarray(inst.T, np.float64)
        G[k, 12] = float(inst.s)
        ids[k] = int(inst.model)
    inst_G = torch.from_numpy(G).to(dev)
    inst_object = torch.from_numpy(ids).to(dev)
    return SceneGPU(list(objects), inst_object, inst_G, compose_transforms(inst_G))


# ---------------------------------------------------------------- rays
def camera_rays(cam) -> A.Rays:
    r = A.Rays()
    r.kind = 0
    c = r.camera
    for i in range(3):
        c.eye[i], c.at[i], c.up[i] = float(cam.eye[i]), float(cam.at[i]), float(cam.up[i])
    c.fov_y_deg = float(cam.fov_y_deg)
    c.width, c.height = int(cam.width), int(cam.height)
    return r


def array_rays(o: torch.Tensor, d: torch.Tensor) -> A.Rays:
    assert o.is_contiguous() and d.is_contiguous() and o.dtype == torch.float32 and d.dtype == torch.float32
    r = A.Rays()
    r.kind = 1
    r.origins = o.data_ptr() if o.numel() else None
    r.dirs = d.data_ptr() if d.numel() else None
    r.n = int(o.shape[0])
    r._keep = (o, d)
    return r


def n_rays(rays: A.Rays) -> int:
    return rays.camera.width * rays.camera.height if rays.kind == 0 else int(rays.n)


# ---------------------------------------------------------------- entry points
class Workspace:
    """Caller-owned device workspace, grown on demand (allocation happens here,
    in the binding, never inside a library call)."""

    def __init__(self, device=None):
        self.dev = _device(device)
        self.buf = torch.empty(0, dtype=torch.uint8, device=self.dev)

    def get(self, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
        return self.buf


def march_depth(scene: SceneGPU, rays: A.Rays, n_samples: int = 128, clip_to_bound: bool = True,
                t_near: float = 0.0, t_far: float = 0.0, hit_threshold: float = 0.5, dtype: str = "f32",
                opacity: bool = True, ws: Workspace | None = None, pair_capacity: int = 0, out=None):
    """Plain volume-rendering marcher composed over instances.  Returns
    (depth float32 [n], id int32 [n], opacity float32 [n] or None)."""
    lib = A.load()
    n = n_rays(rays)
    dev = scene.inst_w2l.device
    if out is None:
        depth = torch.empty(n, dtype=torch.float32, device=dev)
        ident = torch.empty(n, dtype=torch.int32, device=dev)
        opac = torch.empty(n, dtype=torch.float32, device=dev) if opacity else None
    else:
        depth, ident, opac = out
    sc = scene.struct()
    opts = A.MarchOpts(n_samples=n_samples, clip_to_bound=int(clip_to_bound), t_near=t_near, t_far=t_far,
                       hit_threshold=hit_threshold, dtype=A.DTYPES[dtype])
    nbytes = lib.nedf_workspace_size(A.OPS["march"], C.byref(sc), C.byref(rays), int(pair_capacity))
    ws = ws or Workspace(dev)
    buf = ws.get(nbytes)
    A.check(lib.nedf_march_depth(C.byref(sc), C.byref(rays), C.byref(opts), _ptr(depth), _ptr(ident),
                                 _ptr(opac), buf.data_ptr(), int(nbytes), _stream()), "nedf_march_depth")
    return depth, ident, opac


def check_status(ws: Workspace) -> int:
    lib = A.load()
    return int(lib.nedf_check_status(ws.buf.data_ptr(), _stream()))


def ws_counters(ws: Workspace) -> tuple:
    lib = A.load()
    out = (C.c_int64 * 2)()
    A.check(lib.nedf_ws_counters(ws.buf.data_ptr(), _stream(), out), "nedf_ws_counters")
    return int(out[0]), int(out[1])


def profile_enable(on: bool = True) -> None:
    A.check(A.load().nedf_profile_enable(int(on)), "nedf_profile_enable")


def profile_read(max_stages: int = 64) -> dict:
    """Per-stage (total_ms, count) recorded since profile_enable."""
    lib = A.load()
    names = C.create_string_buffer(64 * max_stages)
    ms = (C.c_double * max_stages)()
    cnt = (C.c_int32 * max_stages)()
    n = C.c_int32()
    A.check(lib.nedf_profile_read(max_stages, names, ms, cnt, C.byref(n)), "nedf_profile_read")
    out = {}
    for k in range(n.value):
        nm = names.raw[64 * k:64 * k + 64].split(b"\0", 1)[0].decode()
        out[nm] = (float(ms[k]), int(cnt[k]))
    return out
