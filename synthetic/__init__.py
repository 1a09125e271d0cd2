"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module only draws random numbers and lays them out as arrays: camera
descriptions, MLP weights, rigid-transform parameters (R, T, s), light
positions, training rays and pixel subsets.  It holds none of the rendering
method's arithmetic (no ray generation, no encoding, no network evaluation, no
compositing), so that the oracle and the GPU path stay independent.

Every generator is a NumPy PCG64 stream seeded with
``4669 + 1000 * config + stream`` so that a (config, stream) pair always gives
the same bytes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 4669


def rng(config: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * config + stream))


# --------------------------------------------------------------------------
# camera and scene descriptions (plain parameters)
# --------------------------------------------------------------------------
@dataclass
class Camera:
    eye: tuple
    at: tuple
    up: tuple
    fov_y_deg: float
    width: int
    height: int

    @property
    def n_rays(self) -> int:
        return self.width * self.height


@dataclass
class MLPWeights:
    """Fully connected layers, PyTorch convention: W[i] is [out, in] float32."""
    W: list
    b: list

    @property
    def dims(self):
        return [self.W[0].shape[1]] + [w.shape[0] for w in self.W]


@dataclass
class Model:
    """One object model.  ``kind`` names the density field family:

    * ``sphere``  analytic sigma_max * sigmoid((radius - |x|) / width)
    * ``slab``    sigma0 inside z0 <= z <= z1
    * ``mlp``     density MLP on gamma_L(x); ``sigma_mode`` is ``softplus``
                  (optionally masked to |x| <= bound) or ``sdf`` (SDF-biased)
    * ``nerf``    density trunk as ``mlp`` plus an RGB branch
    * ``nedf``    ray -> (mu_hat, hit logit) network on gamma_L(Pluecker)
    * ``nedf16``  ray -> (hit logit, coarse and fine bin logits): residual
                  network on gamma_L of points along the ray
    """
    kind: str
    bound: float = 1.0
    params: dict = field(default_factory=dict)
    trunk: MLPWeights | None = None
    rgb: MLPWeights | None = None


@dataclass
class Instance:
    model: int
    R: np.ndarray      # 3x3 float64 rotation
    T: np.ndarray      # 3 float64 translation
    s: float           # uniform scale


def normal_mlp(g: np.random.Generator, dims, head_std_fan_in: bool = True,
               hidden_gain: float = 1.0) -> MLPWeights:
    """Weights N(0, gain/fan_in) as float32, biases zero."""
    W, b = [], []
    n = len(dims) - 1
    for i in range(n):
        fan_in, fan_out = dims[i], dims[i + 1]
        gain = hidden_gain if i < n - 1 else 1.0
        w = g.standard_normal((fan_out, fan_in)) * math.sqrt(gain / fan_in)
        W.append(w.astype(np.float32))
        b.append(np.zeros(fan_out, dtype=np.float32))
    return MLPWeights(W, b)


def shoemake_rotation(g: np.random.Generator) -> np.ndarray:
    """Uniform rotation from a uniform unit quaternion (Shoemake, Graphics
    Gems III, 1992), returned as a float64 3x3 matrix."""
    u1, u2, u3 = g.random(3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    qx, qy = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    qz, qw = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)],
        [2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)],
        [2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)],
    ], dtype=np.float64)


def pixel_subset(config: int, n_pixels: int, n: int, stream: int = 7) -> np.ndarray:
    """Sorted seeded subset of pixel indices (without replacement)."""
    g = rng(config, stream)
    n = min(n, n_pixels)
    return np.sort(g.choice(n_pixels, size=n, replace=False)).astype(np.int64)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
SPHERE_A = dict(sigma_max=50.0, radius=0.5, width=0.01)


def config1_camera(width: int = 32, height: int = 32) -> Camera:
    return Camera(eye=(0.0, 0.0, 4.0), at=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
                  fov_y_deg=40.0, width=width, height=height)


def config1_models():
    """Density A (analytic sphere) and density B (gamma_6 -> 3x64 ReLU ->
    softplus, N(0, 1/fan_in) float32 weights, seed stream 1)."""
    a = Model(kind="sphere", bound=1.0, params=dict(SPHERE_A))
    g = rng(1, 1)
    trunk = normal_mlp(g, [39, 64, 64, 64, 1])
    b = Model(kind="mlp", bound=1.0, trunk=trunk,
              params=dict(enc_L=6, sigma_mode="softplus", masked=False))
    return a, b


def nerf_model(config: int, stream: int, sigma_mode: str = "softplus", sdf_shape: int = 0,
               width: int = 256, depth: int = 8, enc_L: int = 10, dir_L: int = 4,
               rgb_width: int = 128) -> Model:
    """A NeRF-shaped object: gamma_L(x) -> depth x width ReLU -> sigma head,
    plus concat(h, gamma_dirL(d)) -> rgb_width ReLU -> 3 (sigmoid).
    Hidden weights N(0, 1/fan_in), biases zero."""
    g = rng(config, stream)
    d_in = 3 * (1 + 2 * enc_L)
    trunk = normal_mlp(g, [d_in] + [width] * depth + [1])
    d_dir = 3 * (1 + 2 * dir_L)
    rgb = normal_mlp(g, [width + d_dir, rgb_width, 3])
    params = dict(enc_L=enc_L, dir_L=dir_L, sigma_mode=sigma_mode, masked=True)
    if sigma_mode == "sdf":
        params.update(sdf_shape=sdf_shape, sigma_max=50.0, width=0.01)
    return Model(kind="nerf", bound=1.0, trunk=trunk, rgb=rgb, params=params)


def config2_scene(n_objects: int = 16, width: int = 800, height: int = 800):
    """16 as-stated NeRFs (masked to |x| <= 1), random rigid placement
    (Shoemake rotation, T ~ U[-3,3]^3, s ~ U[0.5,1.5], stream 900), camera at
    (0,0,13) looking at the origin, one point light at (6,10,8)."""
    models = [nerf_model(2, k) for k in range(n_objects)]
    g = rng(2, 900)
    insts = []
    for k in range(n_objects):
        R = shoemake_rotation(g)
        T = g.uniform(-3.0, 3.0, size=3)
        s = float(g.uniform(0.5, 1.5))
        insts.append(Instance(model=k, R=R, T=T, s=s))
    cam = Camera(eye=(0.0, 0.0, 13.0), at=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
                 fov_y_deg=40.0, width=width, height=height)
    light = np.array([6.0, 10.0, 8.0])
    return models, insts, cam, [light]


def scene_extent(insts, bounds) -> float:
    """Diameter of the smallest sphere centred at the centroid of the instance
    bounding-sphere centres that contains every instance bounding sphere."""
    c = np.mean([i.T for i in insts], axis=0)
    r = max(np.linalg.norm(i.T - c) + i.s * bounds[i.model] for i in insts)
    return 2.0 * float(r)


def training_rays(config: int, stream: int, n: int, radius: float = 4.0,
                  aim_radius: float = 1.2):
    """Local-space training rays: origin uniform on the sphere of the given
    radius, aimed at a point uniform in the ball of radius ``aim_radius``.
    Returns float32 (o [n,3], d [n,3]) with unit d."""
    g = rng(config, stream)
    v = g.standard_normal((n, 3))
    o = radius * v / np.linalg.norm(v, axis=1, keepdims=True)
    w = g.standard_normal((n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    p = w * aim_radius * g.random((n, 1)) ** (1.0 / 3.0)
    d = p - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


def nedf_model(config: int, stream: int, enc_L: int = 8, width: int = 256, depth: int = 8,
               bound: float = 1.0, head_scale: float = 1.0, logit_scale: float = 1.0) -> Model:
    """An intersection network F_Phi: gamma_L(d, o x d) (6 (1 + 2L) inputs)
    -> depth x width ReLU -> (mu_hat, hit logit).  Hidden weights
    N(0, 2/fan_in) (He), head N(0, 1/fan_in) scaled by ``head_scale``
    (the hit-logit row by a further ``logit_scale``, which spreads the hit
    probabilities of an untrained network over hits, misses and the
    uncertain band without changing its depth output), biases zero: the
    training initialisation, also used untrained by the parity tests."""
    g = rng(config, stream)
    d_in = 6 * (1 + 2 * enc_L)
    trunk = normal_mlp(g, [d_in] + [width] * depth + [2], hidden_gain=2.0)
    trunk.W[-1] *= np.float32(head_scale)
    trunk.W[-1][1] *= np.float32(logit_scale)
    return Model(kind="nedf", bound=bound, trunk=trunk, params=dict(enc_L=enc_L))


def classifier_model(config: int, stream: int, enc_L: int = 10, n_points: int = 16, width: int = 256,
                     n_blocks: int = 16, n_coarse: int = 64, n_fine: int = 128, bound: float = 1.0,
                     block_scale: float = 0.25, bias_std: float = 0.0, tail_scale: float = 1.0) -> Model:
    """An intersection network in the multi-level classifier form: input
    n_points x 3 (1 + 2 enc_L) values; layers, in order: head [width, in],
    then per residual block two [width, width] layers, then the tail
    [1 + n_coarse + n_fine, width] (rows: hit logit, coarse bins, fine bins).
    Head and first block layers N(0, 2/fan_in) (He), second block layers the
    same times ``block_scale`` (keeps the residual stream's growth over the
    blocks moderate), tail N(0, 1/fan_in) times ``tail_scale``; biases
    N(0, bias_std^2) (zero: the training initialisation)."""
    g = rng(config, stream)
    d_in = n_points * 3 * (1 + 2 * enc_L)
    W, b = [], []

    def layer(n_out, n_in, std):
        W.append((g.standard_normal((n_out, n_in)) * std).astype(np.float32))
        b.append((g.standard_normal(n_out) * bias_std).astype(np.float32))

    layer(width, d_in, math.sqrt(2.0 / d_in))
    for _ in range(n_blocks):
        layer(width, width, math.sqrt(2.0 / width))
        layer(width, width, math.sqrt(2.0 / width) * block_scale)
    layer(1 + n_coarse + n_fine, width, math.sqrt(1.0 / width) * tail_scale)
    return Model(kind="nedf16", bound=bound, trunk=MLPWeights(W, b),
                 params=dict(enc_L=enc_L, n_points=n_points, n_blocks=n_blocks, n_coarse=n_coarse,
                             n_fine=n_fine))


def sdf_scene(config: int, n_inst: int, n_models: int = 4, width: int = 64, height: int = 64,
              z_range=(4.0, 8.0), spread: float = 1.2):
    """SDF-biased NeRF objects (shapes 0..n_models-1) placed in front of a
    camera at the origin looking down -z: instance k uses model k mod
    n_models, a uniform rotation, scale U[0.6, 1.2] and a centre at depth
    U[z_range] within a lateral spread.  Returns models, instances, camera."""
    models = [nerf_model(config, 100 + k, sigma_mode="sdf", sdf_shape=k % 4) for k in range(n_models)]
    g = rng(config, 901)
    insts = []
    for k in range(n_inst):
        z = g.uniform(*z_range)
        T = np.array([g.uniform(-spread, spread), g.uniform(-spread, spread), -z])
        insts.append(Instance(model=k % n_models, R=shoemake_rotation(g), T=T, s=float(g.uniform(0.6, 1.2))))
    cam = Camera(eye=(0.0, 0.0, 0.0), at=(0.0, 0.0, -1.0), up=(0.0, 1.0, 0.0), fov_y_deg=40.0,
                 width=width, height=height)
    return models, insts, cam


def _outside_all(p, insts, bounds) -> bool:
    return all(np.linalg.norm(p - i.T) > i.s * bounds[i.model] for i in insts)


def batched_scene(config: int, n_inst: int, width: int, height: int, n_models: int = 4,
                  coverage=(0.01, 0.20), z_range=(6.0, 30.0), fov_y_deg: float = 40.0,
                  lights=((20.0, 30.0, 10.0), (-25.0, 20.0, 5.0))):
    """Many instances of a few SDF-biased NeRF objects with uneven screen
    coverage.  Camera at the origin looking down -z.  Instance k uses model
    k mod n_models, a uniform rotation, a target screen coverage
    c ~ U[coverage] (fraction of the image), a depth z ~ U[z_range] and a
    screen position uniform over the image; its bounding-sphere radius is
    R = z sqrt(c W H / pi) / f_px, so s = R / l.  A light inside a bounding
    sphere is moved by seeded unit steps until it is outside every one.
    Returns models, instances, camera, lights."""
    models = [nerf_model(config, 100 + k, sigma_mode="sdf", sdf_shape=k % 4) for k in range(n_models)]
    bounds = [m.bound for m in models]
    g = rng(config, 901)
    f_px = 0.5 * height / np.tan(np.radians(0.5 * fov_y_deg))
    insts = []
    for k in range(n_inst):
        c = g.uniform(*coverage)
        z = g.uniform(*z_range)
        u, v = g.uniform(0.0, width), g.uniform(0.0, height)
        T = np.array([(u - 0.5 * width) / f_px * z, (0.5 * height - v) / f_px * z, -z])
        R_world = z * np.sqrt(c * width * height / np.pi) / f_px
        m = k % n_models
        insts.append(Instance(model=m, R=shoemake_rotation(g), T=T, s=float(R_world / bounds[m])))
    cam = Camera(eye=(0.0, 0.0, 0.0), at=(0.0, 0.0, -1.0), up=(0.0, 1.0, 0.0), fov_y_deg=fov_y_deg,
                 width=width, height=height)
    gl = rng(config, 902)
    out_lights = []
    for L in lights:
        p = np.array(L, dtype=np.float64)
        while not _outside_all(p, insts, bounds):
            w = gl.standard_normal(3)
            p = p + w / np.linalg.norm(w)
        out_lights.append(p)
    return models, insts, cam, out_lights


def config4_scene(width: int = 1920, height: int = 1080, n_inst: int = 1000):
    """The batched-composition scene: 1,000 instances of 4 models at 1080p,
    two point lights."""
    return batched_scene(4, n_inst, width, height)


def config5_scene(width: int = 3840, height: int = 2160, n_inst: int = 64):
    """The precision-stress scene: 64 instances (16 per model) at 2160p."""
    return batched_scene(5, n_inst, width, height)
