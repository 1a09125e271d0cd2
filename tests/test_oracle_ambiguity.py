"""CPU pins of the oracle's single-precision records (instance transform and
camera basis) and of the rounding-ambiguity analysis used by the bfloat16
parity tests."""
import numpy as np

import synthetic as syn
from oracle import camera_rays, encode, f32_record, pluecker, round_bf16, secant_refine, to_local
from oracle.ambiguity import (_other_neighbour, encoding_error_bound, nedf_accumulation_sensitivity,
                              nedf_input_ambiguity)
from oracle.fields import mlp_forward
from oracle.rounding import bf16_rounding_margin


def _is_f32(x):
    x = np.asarray(x, np.float64)
    return np.array_equal(x, x.astype(np.float32).astype(np.float64))


def test_record_is_single_precision_and_close_to_exact():
    g = np.random.default_rng(1)
    inst = syn.Instance(0, syn.shoemake_rotation(g), np.array([1.3, -2.7, 0.4]), 0.7)
    rec = f32_record(inst)
    assert _is_f32(rec.R) and _is_f32(rec.c) and _is_f32(rec.inv_s) and _is_f32(rec.s)
    o = g.normal(size=(50, 3)) * 5
    d = g.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ol, dl = to_local(inst, o, d)
    ol2, dl2 = to_local(rec, o, d)
    scale = np.abs(o).max() / 0.7 + 5
    assert np.abs(ol2 - ol).max() <= 4 * 2.0 ** -24 * scale
    assert np.abs(dl2 - dl).max() <= 4 * 2.0 ** -24


def test_record_exact_on_representable_transform():
    """Axis permutation, power-of-two scale and a representable translation:
    the record loses nothing, so both forms agree exactly."""
    R = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    inst = syn.Instance(0, R, np.array([0.5, -1.25, 3.0]), 2.0)
    rec = f32_record(inst)
    o = np.array([[1.0, 2.0, -4.0], [0.25, 0.5, 0.75]])
    d = np.array([[0.0, 0.6, 0.8], [1.0, 0.0, 0.0]])
    ol, dl = to_local(inst, o, d)
    ol2, dl2 = to_local(rec, o, d)
    assert np.array_equal(ol, ol2) and np.array_equal(dl, dl2)
    # o_l = R^T (o - T) / s by hand for the first ray: (o - T) = (0.5, 3.25,
    # -7), and R^T picks components (z, x, y) of it
    assert np.array_equal(ol[0], np.array([(-4.0 - 3.0), (1.0 - 0.5), (2.0 + 1.25)]) / 2.0)


def test_camera_f32_basis_close_to_exact_and_unit():
    cam = syn.Camera(eye=(0.3, -0.2, 4.0), at=(0.0, 0.1, 0.0), up=(0, 1, 0), fov_y_deg=40.0, width=33, height=17)
    o, d = camera_rays(cam)
    o2, d2 = camera_rays(cam, basis="f32")
    assert np.allclose(np.linalg.norm(d2, axis=1), 1.0, atol=1e-15)
    assert np.abs(d2 - d).max() <= 8 * 2.0 ** -24
    assert _is_f32(o2)
    # the centre pixel of an odd-sized image looks along the stored forward axis
    c = (cam.height // 2) * cam.width + cam.width // 2
    fwd = np.array(cam.at) - np.array(cam.eye)
    fwd /= np.linalg.norm(fwd)
    f32 = fwd.astype(np.float32).astype(np.float64)
    assert np.allclose(d2[c], f32 / np.linalg.norm(f32), rtol=0, atol=1e-16)


def test_encoding_error_bound_brute_force():
    """Perturbing the coordinates by at most the stated error moves every
    encoded feature by at most the bound (sine error 0 here)."""
    g = np.random.default_rng(2)
    p = g.uniform(-1, 1, size=(400, 6))
    e = np.full_like(p, 1e-6)
    L = 8
    bound = encoding_error_bound(e, L, 0.0)
    assert bound.shape == encode(p, L).shape
    for _ in range(5):
        q = p + g.uniform(-1, 1, size=p.shape) * e
        assert np.all(np.abs(encode(q, L) - encode(p, L)) <= bound * (1 + 1e-9) + 1e-15)
    # the top level multiplies the coordinate error by 2^(L-1) pi
    assert np.isclose(bound[0, -1], 2.0 ** (L - 1) * np.pi * 1e-6)


def test_other_neighbour_crosses_the_nearest_boundary():
    g = np.random.default_rng(3)
    x = np.concatenate([g.uniform(-3, 3, 20000), 2.0 ** np.arange(-5, 3) * (1 + 2.0 ** -12),
                        -(2.0 ** np.arange(-5, 3)) * (1 - 2.0 ** -12)])
    q = round_bf16(x)
    m = bf16_rounding_margin(x) * np.abs(x)
    alt = _other_neighbour(x, m)
    assert np.all(alt != q)
    # adjacent: no bfloat16 value strictly between q and alt
    mid = 0.5 * (q + alt)
    assert np.all((round_bf16(mid) == q) | (round_bf16(mid) == alt) | (np.abs(mid - q) == np.abs(mid - alt)))
    # the boundary crossed is the nearest one: its distance is the margin
    assert np.allclose(np.abs(0.5 * (q + alt) - x), m, rtol=1e-9, atol=0)
    # the same for E4M3 (3 stored mantissa bits, saturating at 448)
    from oracle import round_e4m3
    from oracle.rounding import e4m3_rounding_margin
    y = g.uniform(-300, 300, 5000)
    qe = round_e4m3(y)
    me = e4m3_rounding_margin(y) * np.abs(y)
    alte = _other_neighbour(y, me, round_e4m3)
    assert np.all(alte != qe)
    assert np.allclose(np.abs(0.5 * (qe + alte) - y), me, rtol=1e-9, atol=0)


def _linear_net(w):
    """A one-hidden-layer network computing mu_hat = w . x exactly: hidden
    ReLU(x), ReLU(-x) with weights +-1 (exact in bfloat16), head [w, -w]."""
    n = w.size
    W1 = np.vstack([np.eye(n), -np.eye(n)]).astype(np.float32)
    H = np.zeros((2, 2 * n), np.float32)
    H[0, :n], H[0, n:] = w, -w
    return syn.Model(kind="nedf", bound=1.0, trunk=syn.MLPWeights(W=[W1, H], b=[np.zeros(2 * n, np.float32),
                                                                              np.zeros(2, np.float32)]),
                     params=dict(enc_L=1))


def test_input_ambiguity_closed_form_on_linear_network():
    """On mu_hat = w . round_bf16(x) the re-rounding of one close feature j
    changes mu_hat by |w_j| times the bfloat16 spacing there; a feature
    with w_j = 0 causes no ambiguity however close it is."""
    g = np.random.default_rng(4)
    o = g.uniform(-0.5, 0.5, size=(300, 3))
    d = g.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pl, _ = pluecker(o, d)
    x = encode(pl, 1)
    w = np.zeros(x.shape[1], np.float32)
    j = 7  # sin(pi m_y)
    w[j] = 0.25
    net = _linear_net(w)
    margin = bf16_rounding_margin(x[:, j]) * np.abs(x[:, j])
    # error bound flagging feature j on rays where it is within 1e-4 of a boundary
    coord_err = np.zeros_like(pl)
    amb, cnt = nedf_input_ambiguity(net, o, d, coord_err, 1e-4)
    close = margin < 1e-4
    alt = _other_neighbour(x[:, j], margin)
    expect = np.where(close, 0.25 * np.abs(alt - round_bf16(x[:, j])), 0.0)
    base = 0.25 * round_bf16(x[:, j])
    ok = np.abs(base) < 0.99  # the clamp to [-1, 1] does not bite
    assert close[ok].sum() > 5
    assert np.allclose(amb[ok], expect[ok], rtol=0, atol=1e-12)
    # zero weight: no ambiguity
    net0 = _linear_net(np.zeros_like(w))
    amb0, _ = nedf_input_ambiguity(net0, o, d, coord_err, 1e-4)
    assert np.all(amb0 == 0.0)
    # no error: nothing flagged
    amb_none, cnt_none = nedf_input_ambiguity(net, o, d, coord_err, 0.0)
    assert np.all(cnt_none == 0) and np.all(amb_none == 0.0)


def test_accumulation_sensitivity_zero_on_exact_sums():
    """Operands whose products and partial sums are exact in float32 (small
    dyadic values): float32 and float64 summation agree exactly."""
    g = np.random.default_rng(5)
    net = syn.nedf_model(3, 7, enc_L=1, width=16, depth=3)
    for i in range(len(net.trunk.W)):
        net.trunk.W[i] = (np.round(net.trunk.W[i] * 8) / 8).astype(np.float32)
    o = np.round(g.uniform(-0.5, 0.5, size=(64, 3)) * 4) / 4
    d = np.tile(np.array([[0.0, 0.0, 1.0]]), (64, 1))
    # features of these lines are not dyadic (sines), so build a direct
    # check on the forward pass with dyadic inputs instead
    x = np.round(g.uniform(-1, 1, size=(64, 18)) * 16) / 16
    a = mlp_forward(x, net.trunk, gemm="bf16")
    b = mlp_forward(x, net.trunk, gemm="bf16", acc="f32")
    assert np.array_equal(a, b)
    s = nedf_accumulation_sensitivity(net, o, d)
    assert s.shape == (64,) and np.all(s >= 0)


def test_secant_margins_on_affine_field():
    """f(t) = c0 + c . x(t) - iso along a ray is affine: the bracket margin
    is min(|f(D - e)|, |f(D + e)|) in closed form, and the guard margin of
    an exact first iterate at the root t* is min(|t* - lo|, |hi - t*|)."""
    lin = syn.Model(kind="linear", params=dict(c0=1.0, c=[0.0, 0.0, -2.0], iso=3.0))
    inst = syn.Instance(0, np.eye(3), np.zeros(3), 1.0)
    o = np.array([[0.0, 0.0, 0.0]])
    d = np.array([[0.0, 0.0, -1.0]])
    # f(t) = 1 + 2 t - 3 = 2 t - 2: root t* = 1
    D = np.array([1.02])
    out, fmin, gmin = secant_refine(lin, inst, o, d, D, h=0.05, steps=3, margins=True)
    assert np.isclose(out[0], 1.0, atol=1e-12)
    assert np.isclose(fmin[0], min(abs(2 * (1.02 - 0.05) - 2), abs(2 * (1.02 + 0.05) - 2)))
    assert np.isclose(gmin[0], min(abs(1.0 - (1.02 - 0.1)), abs((1.02 + 0.1) - 1.0)))
