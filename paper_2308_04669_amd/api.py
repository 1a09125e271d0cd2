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


def object_from_model(model, dtype: str = "bf16", device=None, nedf_model=None, nedf_dtype: str | None = None,
                      nedf_scales=None) -> ObjectSpec:
    """Build an ObjectSpec from a model description with the attributes
    ``kind``, ``bound``, ``params``, ``trunk`` (W, b lists) and ``rgb``."""
    p = model.params
    colour = tuple(p.get("colour", (0.8, 0.8, 0.8)))
    if model.kind in ("sphere", "slab"):
        if model.kind == "sphere":
            spec = ObjectSpec("sphere", model.bound, (p["sigma_max"], p["radius"], p["width"]) + colour)
        else:
            spec = ObjectSpec("slab", model.bound, (p["sigma0"], p["z0"], p["z1"]) + colour)
        if nedf_model is not None:
            spec.nedf = _pack_nedf(nedf_model, nedf_dtype or dtype, device, nedf_scales)
        return spec
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
            spec.nedf = _pack_nedf(nedf_model, nedf_dtype or dtype, device, nedf_scales)
        return spec
    raise ValueError(model.kind)


def _pack_nedf(nedf_model, dtype, device, fp8_scales=None) -> PackedMLP:
    t = nedf_model.trunk
    if nedf_model.kind == "nedf16":
        # classifier form: head, two layers per residual block, tail
        nshape = mlp_shape("points16", nedf_model.params["enc_L"], t.W[0].shape[0], nedf_model.params["n_blocks"],
                           t.W[-1].shape[0])
        return pack_mlp(t.W, t.b, nshape, dtype, device)
    nshape = mlp_shape("pluecker", nedf_model.params["enc_L"], t.W[0].shape[0], len(t.W) - 1, 2)
    return pack_mlp(t.W, t.b, nshape, dtype, device, fp8_scales=fp8_scales)


def fp8_calibrate(W, b, o_l: torch.Tensor, d_l: torch.Tensor, enc_L: int = 8, in_kind: str = "pluecker"):
    """Per-hidden-layer E4M3 scales {w_scale, a_scale} from a GPU calibration
    pass over the rays (o_l, d_l) (float32 [B, 3], B a multiple of 64)."""
    lib = A.load()
    dev = o_l.device
    shape = mlp_shape(in_kind, enc_L, W[0].shape[0], len(W) - 1, W[-1].shape[0])
    s = A.MlpShape(**{k: int(v) for k, v in shape.items()})
    B = int(o_l.shape[0])
    Wt = [torch.from_numpy(np.ascontiguousarray(w, np.float32)).to(dev) for w in W]
    bt = [torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev) for x in b]
    Wp = (C.c_void_p * len(Wt))(*[t.data_ptr() for t in Wt])
    bp = (C.c_void_p * len(bt))(*[t.data_ptr() for t in bt])
    n = lib.nedf_fp8_calibrate_workspace_size(C.byref(s), B)
    ws = torch.empty(int(n), dtype=torch.uint8, device=dev)
    scales = torch.zeros(2 * (len(W) - 1), dtype=torch.float32, device=dev)
    A.check(lib.nedf_fp8_calibrate(C.byref(s), Wp, bp, o_l.data_ptr(), d_l.data_ptr(), B, scales.data_ptr(),
                                   ws.data_ptr(), int(n), _stream()), "nedf_fp8_calibrate")
    torch.cuda.current_stream().synchronize()
    return scales.cpu().numpy().astype(np.float64)


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
    in the binding, never inside a library call).  ``pair_hint`` sizes the
    pair lists of calls that pass no explicit capacity: instead of the
    library's worst case (every ray against every instance) it is the given
    count, and ``ws_counters`` updates it to 1.25 x the culled pairs it reads
    plus 2^20 (a frame sized from the previous frame's culling).  A call
    whose lists overflow reports NEDF_ERR_CAPACITY through ``check_status``."""

    def __init__(self, device=None, pair_hint: int = 0):
        self.dev = _device(device)
        self.buf = torch.empty(0, dtype=torch.uint8, device=self.dev)
        self.pair_hint = int(pair_hint)

    def capacity(self, pair_capacity: int) -> int:
        return int(pair_capacity) if pair_capacity else self.pair_hint

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
    ws = ws or Workspace(dev)
    nbytes = lib.nedf_workspace_size(A.OPS["march"], C.byref(sc), C.byref(rays), ws.capacity(pair_capacity))
    buf = ws.get(nbytes)
    A.check(lib.nedf_march_depth(C.byref(sc), C.byref(rays), C.byref(opts), _ptr(depth), _ptr(ident),
                                 _ptr(opac), buf.data_ptr(), int(nbytes), _stream()), "nedf_march_depth")
    return depth, ident, opac


def infer_opts(dtype="bf16", p_lo=0.2, p_hi=0.8, refine_steps=3, refine_h=0.05, n_samples=128,
               hit_threshold=0.5) -> A.InferOpts:
    m = A.MarchOpts(n_samples=n_samples, clip_to_bound=1, t_near=0.0, t_far=0.0, hit_threshold=hit_threshold,
                    dtype=A.DTYPES[dtype])
    return A.InferOpts(dtype=A.DTYPES[dtype], p_lo=p_lo, p_hi=p_hi, refine_steps=refine_steps,
                       refine_h=refine_h, march=m)


def infer_depth_id(scene: SceneGPU, rays: A.Rays, dtype: str = "bf16", p_lo: float = 0.2, p_hi: float = 0.8,
                   refine_steps: int = 3, refine_h: float = 0.05, n_samples: int = 128,
                   ws: Workspace | None = None, pair_capacity: int = 0, out=None):
    """NeDF depth+ID with marcher fallback and secant refinement.  Returns
    (depth float32 [n], id int32 [n])."""
    lib = A.load()
    n = n_rays(rays)
    dev = scene.inst_w2l.device
    if out is None:
        depth = torch.empty(n, dtype=torch.float32, device=dev)
        ident = torch.empty(n, dtype=torch.int32, device=dev)
    else:
        depth, ident = out
    sc = scene.struct()
    opts = infer_opts(dtype, p_lo, p_hi, refine_steps, refine_h, n_samples)
    ws = ws or Workspace(dev)
    nbytes = lib.nedf_workspace_size(A.OPS["infer"], C.byref(sc), C.byref(rays), ws.capacity(pair_capacity))
    buf = ws.get(nbytes)
    A.check(lib.nedf_infer_depth_id(C.byref(sc), C.byref(rays), C.byref(opts), _ptr(depth), _ptr(ident),
                                    buf.data_ptr(), int(nbytes), _stream()), "nedf_infer_depth_id")
    return depth, ident


def infer_depth_id_static(scene: SceneGPU, rays: A.Rays, dtype: str = "bf16", p_lo: float = 0.2, p_hi: float = 0.8,
                          refine_steps: int = 3, refine_h: float = 0.05, n_samples: int = 128, out=None):
    """``infer_depth_id`` through the entry point that takes no workspace and
    allocates nothing on the device (a fixed per-GPU scratch array); ``out``
    (depth, ident) lets the caller provide the outputs too."""
    lib = A.load()
    n = n_rays(rays)
    dev = scene.inst_w2l.device
    if out is None:
        depth = torch.empty(n, dtype=torch.float32, device=dev)
        ident = torch.empty(n, dtype=torch.int32, device=dev)
    else:
        depth, ident = out
    sc = scene.struct()
    opts = infer_opts(dtype, p_lo, p_hi, refine_steps, refine_h, n_samples)
    A.check(lib.nedf_infer_depth_id_static(C.byref(sc), C.byref(rays), C.byref(opts), _ptr(depth), _ptr(ident),
                                           _stream()), "nedf_infer_depth_id_static")
    return depth, ident


def subset_scene(scene: SceneGPU, idx) -> tuple[SceneGPU, torch.Tensor]:
    """The instances ``idx`` of ``scene`` as a scene of their own (same
    objects), with the int32 device tensor of their indices in ``scene`` for
    ``infer_keys``."""
    dev = scene.inst_w2l.device
    ix = torch.as_tensor(np.asarray(idx, np.int64), device=dev)
    sub = SceneGPU(scene.objects, scene.inst_object[ix].contiguous(), scene.inst_G[ix].contiguous(),
                   scene.inst_w2l[ix].contiguous())
    return sub, ix.to(torch.int32).contiguous()


def infer_keys(scene: SceneGPU, rays: A.Rays, inst_gid: torch.Tensor | None = None, dtype: str = "bf16",
               p_lo: float = 0.2, p_hi: float = 0.8, n_samples: int = 128, ws: Workspace | None = None,
               pair_capacity: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """Per-ray depth keys (int64 [n]; float bits of the depth << 32 | instance
    index in the full scene, all ones in the low word for no hit) of the
    instances of ``scene``: the part of ``infer_depth_id`` that
    ``compose_keys`` can reuse across frames."""
    lib = A.load()
    n = n_rays(rays)
    dev = scene.inst_w2l.device
    keys = out if out is not None else torch.empty(n, dtype=torch.int64, device=dev)
    sc = scene.struct()
    opts = infer_opts(dtype, p_lo, p_hi, 0, 0.05, n_samples)
    ws = ws or Workspace(dev)
    nbytes = lib.nedf_workspace_size(A.OPS["infer"], C.byref(sc), C.byref(rays), ws.capacity(pair_capacity))
    buf = ws.get(nbytes)
    A.check(lib.nedf_infer_keys(C.byref(sc), C.byref(rays), C.byref(opts), _ptr(inst_gid), _ptr(keys),
                                buf.data_ptr(), int(nbytes), _stream()), "nedf_infer_keys")
    return keys


def compose_keys(scene: SceneGPU, rays: A.Rays, key_sets, dtype: str = "bf16", refine_steps: int = 3,
                 refine_h: float = 0.05, n_samples: int = 128, ws: Workspace | None = None, out=None,
                 pair_capacity: int = 0):
    """Depth and ID of the full ``scene`` from the keys of disjoint instance
    sets (``infer_keys``), merged by their minimum and refined.  Returns
    (depth float32 [n], id int32 [n])."""
    lib = A.load()
    n = n_rays(rays)
    dev = scene.inst_w2l.device
    if out is None:
        depth = torch.empty(n, dtype=torch.float32, device=dev)
        ident = torch.empty(n, dtype=torch.int32, device=dev)
    else:
        depth, ident = out
    sets = list(key_sets)
    for k in sets:
        assert k.dtype == torch.int64 and k.is_contiguous() and k.numel() == n
    arr = (C.c_void_p * len(sets))(*[k.data_ptr() for k in sets])
    sc = scene.struct()
    opts = infer_opts(dtype, 0.2, 0.8, refine_steps, refine_h, n_samples)
    # the refinement bins at most one pair per ray
    nbytes = lib.nedf_workspace_size(A.OPS["infer"], C.byref(sc), C.byref(rays), int(pair_capacity or max(n, 1)))
    ws = ws or Workspace(dev)
    buf = ws.get(nbytes)
    A.check(lib.nedf_compose_keys(C.byref(sc), C.byref(rays), C.byref(opts), arr, len(sets), _ptr(depth),
                                  _ptr(ident), buf.data_ptr(), int(nbytes), _stream()), "nedf_compose_keys")
    return depth, ident


def shade_deferred(scene: SceneGPU, rays: A.Rays, depth: torch.Tensor, ident: torch.Tensor, K: int = 8,
                   h: float = 0.05, clear_rgb=(0.0, 0.0, 0.0), dtype: str = "bf16", ws: Workspace | None = None,
                   out: torch.Tensor | None = None, pair_capacity: int = 0, rs_sigma: float = 0.0,
                   rs_samples: int = 32) -> torch.Tensor:
    """Deferred shading of every pixel with a valid ID (pixels whose density
    stays below ``rs_sigma`` at every sample are shaded again over the
    bounding chord with ``rs_samples`` samples); returns rgb [n, 3]."""
    lib = A.load()
    n = n_rays(rays)
    dev = scene.inst_w2l.device
    rgb = out if out is not None else torch.empty((n, 3), dtype=torch.float32, device=dev)
    sc = scene.struct()
    opts = A.ShadeOpts(K=K, h=h, dtype=A.DTYPES[dtype], rs_sigma=rs_sigma, rs_samples=rs_samples)
    for i in range(3):
        opts.clear_rgb[i] = float(clear_rgb[i])
    # one (pixel, instance) pair per pixel at most
    cap = int(pair_capacity) if pair_capacity > 0 else n
    nbytes = lib.nedf_workspace_size(A.OPS["shade"], C.byref(sc), C.byref(rays), cap)
    ws = ws or Workspace(dev)
    buf = ws.get(nbytes)
    A.check(lib.nedf_shade_deferred(C.byref(sc), C.byref(rays), _ptr(depth), _ptr(ident), C.byref(opts),
                                    _ptr(rgb), buf.data_ptr(), int(nbytes), _stream()), "nedf_shade_deferred")
    return rgb


def shadow(scene: SceneGPU, rays: A.Rays, depth: torch.Tensor, ident: torch.Tensor, lights, eps: float,
           beta: float = 0.5, method: str = "nedf", dtype: str = "bf16", n_samples: int = 128,
           p_lo: float = 0.2, p_hi: float = 0.8, rgb_inout: torch.Tensor | None = None,
           ws: Workspace | None = None, out: torch.Tensor | None = None, pair_capacity: int = 0,
           directional=None, dir_distance: float = 0.0) -> torch.Tensor:
    """Shadow step of Alg. 2 for point lights (and directional lights: the
    entries of ``lights`` whose flag in ``directional`` is set are directions
    of travel, with shadow rays starting ``dir_distance`` back along them);
    returns the multiplier [n] and multiplies ``rgb_inout`` by it when given."""
    lib = A.load()
    n = n_rays(rays)
    dev = scene.inst_w2l.device
    fac = out if out is not None else torch.empty(n, dtype=torch.float32, device=dev)
    L = np.ascontiguousarray(np.asarray(lights, np.float32).reshape(-1, 3))
    sc = scene.struct()
    io = infer_opts(dtype, p_lo, p_hi, 0, 0.05, n_samples)
    mask = 0
    for i, f in enumerate(directional or []):
        if f:
            mask |= 1 << i
    opts = A.ShadowOpts(eps=eps, beta=beta, method=0 if method == "nedf" else 1, infer=io, directional_mask=mask,
                        dir_distance=dir_distance)
    # shadow rays meet other instances than the primary rays: only an explicit
    # capacity sizes their lists (the workspace's hint is the primary pass's)
    nbytes = lib.nedf_workspace_size(A.OPS["shadow"], C.byref(sc), C.byref(rays), int(pair_capacity))
    ws = ws or Workspace(dev)
    buf = ws.get(nbytes)
    A.check(lib.nedf_shadow(C.byref(sc), C.byref(rays), _ptr(depth), _ptr(ident), L.ctypes.data, L.shape[0],
                            C.byref(opts), _ptr(fac), _ptr(rgb_inout), buf.data_ptr(), int(nbytes), _stream()),
            "nedf_shadow")
    return fac


def check_status(ws: Workspace) -> int:
    lib = A.load()
    return int(lib.nedf_check_status(ws.buf.data_ptr(), _stream()))


def ws_counters(ws: Workspace) -> dict:
    """Counters of the last call on ``ws``: pairs, items, and the NeDF
    routing statistics (network-decided hits, marcher fallbacks, misses)."""
    lib = A.load()
    out = (C.c_int64 * 7)()
    A.check(lib.nedf_ws_counters(ws.buf.data_ptr(), _stream(), out), "nedf_ws_counters")
    if int(out[6]) > 0:
        ws.pair_hint = int(1.25 * int(out[6])) + (1 << 20)
    return dict(pairs=int(out[0]), items=int(out[1]), nedf_hits=int(out[2]), fallback=int(out[3]),
                nedf_misses=int(out[4]), fallback_marched=int(out[5]), culled_pairs=int(out[6]))


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


# ---------------------------------------------------------------- training
class Trainer:
    """Device training state of one intersection network (float32 master
    weights, Adam moments, gradients, bfloat16 copies) driven through
    nedf_train_step."""

    def __init__(self, W, b, enc_L: int = 8, in_kind: str = "pluecker", device=None):
        lib = A.load()
        self.dev = _device(device)
        width = W[0].shape[0]
        # classifier form: head, two layers per residual block, tail
        n_hidden = (len(W) - 2) // 2 if in_kind == "points16" else len(W) - 1
        self.shape = mlp_shape(in_kind, enc_L, width, n_hidden, W[-1].shape[0])
        self._s = A.MlpShape(**{k: int(v) for k, v in self.shape.items()})
        n = lib.nedf_train_state_bytes(C.byref(self._s))
        if n == 0:
            raise A.NedfError(2, "nedf_train_state_bytes", lib.nedf_last_error().decode())
        self.state = torch.zeros(int(n), dtype=torch.uint8, device=self.dev)
        self.dims = [(w.shape[0], w.shape[1]) for w in W]
        Wt = [torch.from_numpy(np.ascontiguousarray(w, np.float32)).to(self.dev) for w in W]
        bt = [torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(self.dev) for x in b]
        Wp = (C.c_void_p * len(Wt))(*[t.data_ptr() for t in Wt])
        bp = (C.c_void_p * len(bt))(*[t.data_ptr() for t in bt])
        A.check(lib.nedf_train_init(C.byref(self._s), Wp, bp, self.state.data_ptr(), int(n), _stream()),
                "nedf_train_init")
        torch.cuda.current_stream().synchronize()
        self.ws = Workspace(self.dev)
        self.loss = torch.zeros(4, dtype=torch.float32, device=self.dev)

    def step(self, o_l, d_l, depth_label, hit_label, lr=5e-4, beta1=0.9, beta2=0.999, eps=1e-8, w_hit=0.1,
             bound=1.0) -> torch.Tensor:
        lib = A.load()
        B = int(o_l.shape[0])
        nbytes = lib.nedf_train_workspace_size(C.byref(self._s), B)
        buf = self.ws.get(nbytes)
        opts = A.TrainOpts(lr=lr, beta1=beta1, beta2=beta2, eps=eps, w_hit=w_hit, bound=bound)
        A.check(lib.nedf_train_step(C.byref(self._s), self.state.data_ptr(), o_l.data_ptr(), d_l.data_ptr(),
                                    depth_label.data_ptr(), hit_label.data_ptr(), B, C.byref(opts),
                                    self.loss.data_ptr(), buf.data_ptr(), int(nbytes), _stream()),
                "nedf_train_step")
        return self.loss[:3]

    def export(self, which: int = 0):
        """(W list, b list) as float64 NumPy arrays: master weights (0) or the
        last step's gradients (1)."""
        lib = A.load()
        Wt = [torch.empty(d, dtype=torch.float32, device=self.dev) for d in self.dims]
        bt = [torch.empty(d[0], dtype=torch.float32, device=self.dev) for d in self.dims]
        Wp = (C.c_void_p * len(Wt))(*[t.data_ptr() for t in Wt])
        bp = (C.c_void_p * len(bt))(*[t.data_ptr() for t in bt])
        A.check(lib.nedf_train_export(C.byref(self._s), self.state.data_ptr(), which, Wp, bp, _stream()),
                "nedf_train_export")
        torch.cuda.current_stream().synchronize()
        return [t.cpu().numpy().astype(np.float64) for t in Wt], [t.cpu().numpy().astype(np.float64) for t in bt]


# ---------------------------------------------------------------- tuning
def tune_candidates(kernel: str, dtype: str) -> list:
    lib = A.load()
    out, n = (C.c_int32 * A.TUNE_MAX)(), C.c_int32(0)
    A.check(lib.nedf_tune_candidates(A.TUNE_KERNELS[kernel], A.DTYPES[dtype], out, C.byref(n)),
            "nedf_tune_candidates")
    return [int(out[i]) for i in range(n.value)]


def tune_get(kernel: str, dtype: str) -> int:
    lib = A.load()
    v = C.c_int32(0)
    A.check(lib.nedf_tune_get(A.TUNE_KERNELS[kernel], A.DTYPES[dtype], C.byref(v)), "nedf_tune_get")
    return int(v.value)


def tune_set(kernel: str, dtype: str, value: int) -> None:
    lib = A.load()
    A.check(lib.nedf_tune_set(A.TUNE_KERNELS[kernel], A.DTYPES[dtype], int(value)), "nedf_tune_set")


def autotune(kernel: str, dtype: str, scene: SceneGPU, rays: A.Rays, opts, reps: int = 2,
             ws: Workspace | None = None, pair_capacity: int = 0) -> dict:
    """Run nedf_autotune for ``kernel`` ("march" with march options, "nedf"
    with infer options) and ``dtype`` on these inputs; returns the trial
    report (candidates, ms per run, chosen value)."""
    lib = A.load()
    n = n_rays(rays)
    dev = scene.inst_w2l.device
    depth = torch.empty(n, dtype=torch.float32, device=dev)
    ident = torch.empty(n, dtype=torch.int32, device=dev)
    sc = scene.struct()
    op = A.OPS["march"] if kernel == "march" else A.OPS["infer"]  # "nedf" and "slabs" tune the infer call
    nbytes = lib.nedf_workspace_size(op, C.byref(sc), C.byref(rays), int(pair_capacity))
    ws = ws or Workspace(dev)
    buf = ws.get(nbytes)
    rep = A.TuneReport()
    A.check(lib.nedf_autotune(A.TUNE_KERNELS[kernel], A.DTYPES[dtype], C.byref(sc), C.byref(rays), C.byref(opts),
                              _ptr(depth), _ptr(ident), buf.data_ptr(), int(nbytes), int(reps), _stream(),
                              C.byref(rep)), "nedf_autotune")
    k = rep.n_candidates
    return {"kernel": kernel, "dtype": dtype, "candidates": [int(rep.candidate[i]) for i in range(k)],
            "ms": [float(rep.ms[i]) for i in range(k)], "chosen": int(rep.chosen)}


def march_opts(n_samples: int = 128, clip_to_bound: bool = True, t_near: float = 0.0, t_far: float = 0.0,
               hit_threshold: float = 0.5, dtype: str = "f32") -> A.MarchOpts:
    return A.MarchOpts(n_samples=n_samples, clip_to_bound=int(clip_to_bound), t_near=t_near, t_far=t_far,
                       hit_threshold=hit_threshold, dtype=A.DTYPES[dtype])
