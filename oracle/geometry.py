"""Rays, rigid transforms, encodings (FP64).  Test infrastructure only."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

F64 = np.float64


def camera_rays(cam, pixels=None, basis="exact"):
    """Pinhole primary rays, one per pixel (Alg. 1, NeDF generation step: a
    ray cast through each pixel).  Reading: eye ``cam.eye`` looking at
    ``cam.at``, vertical field of view ``cam.fov_y_deg``, square pixels,
    pixel (i, j) = (column, row from the top) sampled at its centre, unit
    directions.  ``basis="f32"`` takes the camera as stored in single
    precision: eye, forward axis and the right/up axes pre-scaled by the
    image-plane half extents, each rounded to float32 (nearest even), the
    rays then formed exactly from them.  Returns (o [n,3], d [n,3]) float64."""
    W, H = cam.width, cam.height
    if pixels is None:
        pixels = np.arange(W * H, dtype=np.int64)
    pixels = np.asarray(pixels, dtype=np.int64)
    eye, at, up = (np.asarray(v, F64) for v in (cam.eye, cam.at, cam.up))
    fwd = at - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    upv = np.cross(right, fwd)
    th = np.tan(np.deg2rad(cam.fov_y_deg) / 2.0)
    i = (pixels % W).astype(F64)
    j = (pixels // W).astype(F64)
    if basis == "f32":
        r32 = (right * (th * W / H)).astype(np.float32).astype(F64)
        u32 = (upv * th).astype(np.float32).astype(F64)
        f32 = fwd.astype(np.float32).astype(F64)
        eye = eye.astype(np.float32).astype(F64)
        u = (2.0 * i + 1.0 - W) / W
        v = (H - 2.0 * j - 1.0) / H
        d = u[:, None] * r32 + v[:, None] * u32 + f32
    else:
        u = (2.0 * (i + 0.5) / W - 1.0) * th * W / H
        v = (1.0 - 2.0 * (j + 0.5) / H) * th
        d = u[:, None] * right + v[:, None] * upv + fwd
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape).copy()
    return o, d


def inverse_transform(R, T, s):
    """Inverse of the rigid map G(q) = s R q + T (Sec. "Manipulating
    Objects", Eq. 7): G^{-1}(v) = R^T (v - T) / s.  Returns (M [3,3], c [3])
    with G^{-1}(v) = M v + c."""
    R = np.asarray(R, F64)
    M = R.T / s
    c = -(R.T @ np.asarray(T, F64)) / s
    return M, c


@dataclass(frozen=True)
class RecordInstance:
    """An instance seen through a single-precision world-to-local record:
    the inverse map of Eq. 7, G^{-1}(v) = R^T v / s + c with c = -R^T T / s,
    composed exactly and then rounded to float32 (nearest even) entry by
    entry, as the method's transform-preparation step stores it.  Fields hold
    those float32 values as float64; ``s`` is the rounded scale that turns a
    local depth into a world depth."""
    model: int
    R: np.ndarray       # float32-rounded rotation R (3x3), so R^T is its transpose
    inv_s: float        # float32-rounded 1 / s
    c: np.ndarray       # float32-rounded -R^T T / s
    s: float            # float32-rounded s


def _f32(x):
    return np.asarray(x, F64).astype(np.float32).astype(F64)


def f32_record(inst):
    """The single-precision record of an instance (see ``RecordInstance``)."""
    R = np.asarray(inst.R, F64)
    s = float(inst.s)
    c = -(R.T @ np.asarray(inst.T, F64)) / s
    return RecordInstance(model=inst.model, R=_f32(R), inv_s=float(_f32(1.0 / s)), c=_f32(c), s=float(_f32(s)))


def to_local(inst, o, d):
    """Map world rays to the instance's canonical space (Eq. 7: rays, not
    points, are transformed).  o_l = G^{-1}(o), d_l = R^T d (still unit);
    a world distance t along the ray is t / s along the local ray.  For a
    ``RecordInstance`` the record's rounded entries are used, with exact
    (float64) arithmetic: o_l = (R^T o) inv_s + c."""
    R = np.asarray(inst.R, F64)
    if isinstance(inst, RecordInstance):
        o_l = (np.asarray(o, F64) @ R) * inst.inv_s + inst.c
    else:
        o_l = (np.asarray(o, F64) - np.asarray(inst.T, F64)) @ R / inst.s
    d_l = np.asarray(d, F64) @ R
    return o_l, d_l


def pluecker(o_l, d_l):
    """Line coordinates (d, o x d) of a ray; independent of where the origin
    sits on the line.  Also returns t_perp = -o.d, the signed distance from o
    to the tangency point p_perp (Eq. 2, Fig. 2a) for unit d."""
    m = np.cross(o_l, d_l)
    t_perp = -np.sum(o_l * d_l, axis=-1)
    return np.concatenate([d_l, m], axis=-1), t_perp


def encode(p, L):
    """Sinusoidal encoding as in NeRF (appendix: D_i = 16 x 63 for 16 points
    with 10 levels, which includes the identity): [p, sin(2^0 pi p),
    cos(2^0 pi p), ..., sin(2^{L-1} pi p), cos(2^{L-1} pi p)], each a block
    over the components of p."""
    p = np.asarray(p, F64)
    out = [p]
    for k in range(L):
        a = (2.0 ** k) * np.pi * p
        out.append(np.sin(a))
        out.append(np.cos(a))
    return np.concatenate(out, axis=-1)


def sphere_chord(o_l, d_l, radius):
    """Interval [a, b] of a unit-direction ray inside the sphere |x| <= radius
    centred at the local origin, clipped to t >= 0.  ``valid`` is False when
    the ray misses the sphere or the sphere lies behind the origin."""
    t_perp = -np.sum(o_l * d_l, axis=-1)
    b2 = np.sum(o_l * o_l, axis=-1) - t_perp ** 2
    h2 = radius * radius - b2
    valid = h2 > 0.0
    h = np.sqrt(np.where(valid, h2, 0.0))
    a = np.maximum(t_perp - h, 0.0)
    b = t_perp + h
    valid &= b > a
    return a, b, valid
