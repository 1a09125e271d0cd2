"""Pins for NeDF decode, composition, secant refinement, deferred shading
and shadows in the oracle (CPU only)."""
import math

import numpy as np

import synthetic as syn
from oracle import (camera_rays, nedf_pair, nedf_compose, secant_refine, shade_deferred,
                    shadow_factor, march_compose, nerf_eval, to_local)
from oracle.fields import sigmoid

IDENT = syn.Instance(0, np.eye(3), np.zeros(3), 1.0)


def _perfect_sphere_net(r, l):
    """Analytic stand-in for F_Phi on a sphere of radius r centred in local
    space: mu = sqrt(r^2 - |m|^2) (distance from p_perp back to the entry)."""
    def net(o_l, d_l):
        m2 = np.sum(np.cross(o_l, d_l) ** 2, axis=1)
        hit = m2 < r * r
        mu_hat = np.sqrt(np.maximum(r * r - m2, 0.0)) / l
        return mu_hat, np.where(hit, 30.0, -30.0)
    return net


def _world_sphere_entry(o, d, c, rad):
    oc = o - c
    bq = np.sum(oc * d, axis=1)
    cq = np.sum(oc * oc, axis=1) - rad * rad
    disc = bq * bq - cq
    t = -bq - np.sqrt(np.maximum(disc, 0))
    return np.where(disc > 0, t, np.nan)


def test_perfect_nedf_reproduces_ray_sphere_intersection():
    g = syn.rng(0, 21)
    model = syn.Model(kind="nedf", bound=1.0, params=dict(enc_L=8))
    for _ in range(4):
        inst = syn.Instance(0, syn.shoemake_rotation(g), g.uniform(-1, 1, 3), float(g.uniform(0.5, 1.5)))
        cam = syn.Camera(eye=(0.5, 0.2, 7.0), at=tuple(inst.T), up=(0, 1, 0), fov_y_deg=30.0,
                         width=16, height=16)
        o, d = camera_rays(cam)
        hit, D, p, path = nedf_pair(model, None, inst, o, d, net_fn=_perfect_sphere_net(0.5, 1.0),
                                    fallback=False)
        ref = _world_sphere_entry(o, d, inst.T, 0.5 * inst.s)
        assert np.array_equal(hit, np.isfinite(ref))
        assert np.allclose(D[hit], ref[hit], atol=1e-12)
        # Eq. 2 is origin-independent along the line: moving o by lambda d shifts D by -lambda
        lam = 0.7
        hit2, D2, _, _ = nedf_pair(model, None, inst, o + lam * d, d,
                                   net_fn=_perfect_sphere_net(0.5, 1.0), fallback=False)
        assert np.array_equal(hit2, hit)
        assert np.allclose(D2[hit], D[hit] - lam, atol=1e-12)


def test_nedf_band_routes_to_marcher_and_culls():
    a, _ = syn.config1_models()
    model = syn.Model(kind="nedf", bound=1.0, params=dict(enc_L=8))
    cam = syn.config1_camera(16, 16)
    o, d = camera_rays(cam)
    # a net whose hit probability is exactly 0.5 everywhere: every run ray is in the band
    band_net = lambda ol, dl: (np.zeros(len(ol)), np.zeros(len(ol)))
    hit, D, p, path = nedf_pair(model, a, IDENT, o, d, net_fn=band_net, n_samples=128)
    mnorm = np.linalg.norm(np.cross(o, d), axis=1)
    assert np.array_equal(path == 2, mnorm >= 1.0)
    assert np.all(path[mnorm < 1.0] == 1)
    dep, ident, _ = march_compose([a], [IDENT], o, d, 128)
    assert np.array_equal(hit, ident == 0)
    assert np.allclose(D[hit], dep[hit], atol=1e-12)
    # origin inside the bounding sphere always goes to the marcher
    hit3, D3, p3, path3 = nedf_pair(model, a, IDENT, np.zeros_like(o) + [0, 0, 0.9], d,
                                    net_fn=_perfect_sphere_net(0.5, 1.0))
    assert np.all(path3 == 1)


def test_nedf_compose_ties_lower_index():
    model = syn.Model(kind="nedf", bound=1.0, params=dict(enc_L=8))
    cam = syn.config1_camera(8, 8)
    o, d = camera_rays(cam)
    insts = [IDENT, IDENT]
    net = _perfect_sphere_net(0.5, 1.0)
    import oracle.render as R
    orig = R.nedf_eval
    try:
        R.nedf_eval = lambda m, ol, dl, gemm=None, scales=None: net(ol, dl)
        depth, ident = nedf_compose([model], [None], insts, o, d, fallback=False)
    finally:
        R.nedf_eval = orig
    assert np.all(ident[np.isfinite(depth)] == 0)


def test_secant_linear_exact_and_sphere_convergence():
    lin = syn.Model(kind="linear", params=dict(c0=1.0, c=[0.0, 0.0, -2.0], iso=3.0))
    o = np.array([[0.0, 0.0, 4.0]] * 3)
    d = np.array([[0.0, 0.0, -1.0]] * 3)
    # sigma(t) = 1 - 2 (4 - t) = 2t - 7, iso 3 -> root t = 5
    D_hat = np.array([4.98, 5.03, 5.0])
    out = secant_refine(lin, IDENT, o, d, D_hat)
    assert np.allclose(out, 5.0, atol=1e-12)
    # density A: iso level 25 is exactly |x| = 0.5
    a, _ = syn.config1_models()
    cam = syn.config1_camera()
    o, d = camera_rays(cam)
    tp = -np.sum(o * d, axis=1)
    b2 = np.sum(o * o, axis=1) - tp ** 2
    sel = np.nonzero(b2 < 0.4 ** 2)[0]
    t_in = tp[sel] - np.sqrt(0.25 - b2[sel])
    D_hat = t_in + 0.02
    out = secant_refine(a, IDENT, o[sel], d[sel], D_hat)
    assert np.max(np.abs(out - t_in)) < 1e-4
    # outside the bracket nothing moves
    out2 = secant_refine(a, IDENT, o[sel], d[sel], t_in - 0.2)
    assert np.array_equal(out2, t_in - 0.2)


def test_secant_scale_covariance():
    """h is in the object's units: refining on an instance scaled by s about
    the origin, seen from s times farther, gives s times the unscaled depths
    (and a guess off by 0.02 s is still inside the bracket)."""
    a, _ = syn.config1_models()
    cam = syn.config1_camera()
    o, d = camera_rays(cam)
    tp = -np.sum(o * d, axis=1)
    b2 = np.sum(o * o, axis=1) - tp ** 2
    sel = np.nonzero(b2 < 0.4 ** 2)[0]
    t_in = tp[sel] - np.sqrt(0.25 - b2[sel])
    ref = secant_refine(a, IDENT, o[sel], d[sel], t_in + 0.02)
    for sc in (0.25, 3.0):
        big = syn.Instance(0, np.eye(3), np.zeros(3), sc)
        out = secant_refine(a, big, sc * o[sel], d[sel], sc * (t_in + 0.02))
        assert np.allclose(out, sc * ref, rtol=1e-9, atol=1e-12)
        assert np.max(np.abs(out - sc * t_in)) < 1e-4 * sc


def _tiny_nerf(const_rgb=None, stream=0, sigma_mode="softplus"):
    m = syn.nerf_model(0, stream, width=16, depth=2, enc_L=2, dir_L=1, rgb_width=8,
                       sigma_mode=sigma_mode)
    if const_rgb is not None:
        m.rgb.W[-1][:] = 0
        m.rgb.b[-1][:] = np.log(np.array(const_rgb) / (1 - np.array(const_rgb)))
    return m


def test_shading_single_sample_and_constant_colour():
    m = _tiny_nerf()
    cam = syn.config1_camera(6, 6)
    o, d = camera_rays(cam)
    depth = np.full(36, 3.6)
    ident = np.zeros(36, np.int64)
    ident[::5] = -1
    rgb = shade_deferred([m], [IDENT], o, d, depth, ident, K=1, clear=(0.1, 0.2, 0.3))
    x = o + depth[:, None] * d
    sig, col = nerf_eval(m, x, d)
    hitp = ident == 0
    assert np.allclose(rgb[hitp], col[hitp], atol=1e-15)       # K = 1 is Eq. 8
    assert np.allclose(rgb[~hitp], [0.1, 0.2, 0.3])
    mc = _tiny_nerf(const_rgb=(0.25, 0.5, 0.75))
    rgb8 = shade_deferred([mc], [IDENT], o, d, depth, ident, K=8)
    assert np.allclose(rgb8[hitp], [0.25, 0.5, 0.75], atol=1e-12)
    # zero density everywhere (masked, far outside the bound): nearest-sample colour
    far = np.full(36, 20.0)
    rgb0 = shade_deferred([m], [IDENT], o, d, far, ident, K=8, h=0.05)
    t3 = far - 0.05 + 3.5 * (0.1 / 8)
    _, c3 = nerf_eval(m, o + t3[:, None] * d, d)
    assert np.allclose(rgb0[hitp], c3[hitp], atol=1e-15)


def test_shadow_two_spheres_brute_force():
    a, _ = syn.config1_models()
    models = [a]
    insts = [syn.Instance(0, np.eye(3), np.array([0.0, 0.0, 0.0]), 1.0),
             syn.Instance(0, np.eye(3), np.array([0.0, 1.2, 0.0]), 1.0)]
    light = np.array([1.0, 4.0, 1.5])
    cam = syn.Camera(eye=(3.0, 0.6, 3.0), at=(0.0, 0.6, 0.0), up=(0, 1, 0), fov_y_deg=40.0,
                     width=40, height=40)
    o, d = camera_rays(cam)
    N = 256
    depth, ident, _ = march_compose(models, insts, o, d, N)
    depth_fn = lambda oo, dd: march_compose(models, insts, oo, dd, N)[0]
    fac = shadow_factor(depth_fn, o, d, depth, ident, [light], eps=0.05, beta=0.5)
    idx = np.nonzero(ident >= 0)[0]
    assert idx.size > 50
    x = o[idx] + depth[idx, None] * d[idx]
    v = x - light
    dist = np.linalg.norm(v, axis=1)
    ds = v / dist[:, None]
    first = np.full(idx.size, np.inf)
    for inst in insts:
        t = _world_sphere_entry(np.broadcast_to(light, ds.shape), ds, inst.T, 0.5)
        first = np.fmin(first, np.where(np.isfinite(t), t, np.inf))
    # the surface normal at x decides which side faces the light
    own = np.array([insts[k].T for k in ident[idx]])
    nrm = (x - own) / np.linalg.norm(x - own, axis=1, keepdims=True)
    facing = -np.sum(ds * nrm, axis=1)
    # rays grazing a sphere's soft edge (impact parameter near the radius) are ambiguous
    graze = np.zeros(idx.size, bool)
    for inst in insts:
        oc = light - inst.T
        tp = -(ds @ oc)
        bimp = np.sqrt(np.maximum(oc @ oc - tp ** 2, 0))
        graze |= (np.abs(bimp - 0.5) < 0.08) & (tp > 0) & (tp < dist)
    clear_occl = (first < dist - 0.15) & ~graze
    clear_lit = (first > dist - 0.02) & (facing > 0.3) & ~graze
    got = fac[idx] < 1.0
    assert np.all(got[clear_occl]) and not np.any(got[clear_lit])
    assert clear_occl.sum() > 10 and clear_lit.sum() > 10
    assert np.all(fac[ident < 0] == 1.0)
    assert set(np.unique(fac)).issubset({1.0, 0.5})


def test_shadow_directional_light_two_spheres():
    """A directional light (parallel rays travelling along l) over two
    analytic spheres: a hit point is shadowed exactly when the line from it
    back towards the light meets the other sphere (closed form: distance of
    that sphere's centre from the line below its radius, centre on the
    light's side), away from grazing lines and self-shadowing sides."""
    a, _ = syn.config1_models()
    models = [a]
    insts = [syn.Instance(0, np.eye(3), np.array([0.0, 0.0, 0.0]), 1.0),
             syn.Instance(0, np.eye(3), np.array([0.0, 1.2, 0.0]), 1.0)]
    l = np.array([0.15, -1.0, 0.1])
    l /= np.linalg.norm(l)
    cam = syn.Camera(eye=(3.0, 0.6, 3.0), at=(0.0, 0.6, 0.0), up=(0, 1, 0), fov_y_deg=40.0, width=40, height=40)
    o, d = camera_rays(cam)
    N = 256
    depth, ident, _ = march_compose(models, insts, o, d, N)
    depth_fn = lambda oo, dd: march_compose(models, insts, oo, dd, N)[0]
    R = 10.0
    fac = shadow_factor(depth_fn, o, d, depth, ident, [l], eps=0.05, beta=0.5, directional=[True], dir_distance=R)
    idx = np.nonzero(ident >= 0)[0]
    x = o[idx] + depth[idx, None] * d[idx]
    occl = np.zeros(idx.size, bool)
    graze = np.zeros(idx.size, bool)
    for k, inst in enumerate(insts):
        c = inst.T
        s_ = (c - x) @ (-l)                     # along the line towards the light
        dist_c = np.linalg.norm((c - x) - s_[:, None] * (-l), axis=1)
        other = ident[idx] != k
        occl |= other & (s_ > 0) & (dist_c < 0.5)
        graze |= other & (np.abs(dist_c - 0.5) < 0.08)
    own = np.array([insts[k].T for k in ident[idx]])
    nrm = (x - own) / np.linalg.norm(x - own, axis=1, keepdims=True)
    facing = nrm @ (-l)
    got = fac[idx] < 1.0
    sure_occl = occl & ~graze
    sure_lit = ~occl & ~graze & (facing > 0.3)
    assert sure_occl.sum() > 10 and sure_lit.sum() > 10
    assert np.all(got[sure_occl]) and not np.any(got[sure_lit])
    # the same light as a point light far away along -l gives nearly the same shadows
    far = shadow_factor(depth_fn, o, d, depth, ident, [-1e4 * l], eps=0.05, beta=0.5)
    assert np.mean(far[idx] == fac[idx]) > 0.98
