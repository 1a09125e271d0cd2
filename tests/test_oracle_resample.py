"""CPU pins of the oracle's outlier processing in deferred shading (Sec.
"Deferred Shading": pixels whose density at the estimated depth is extremely
small are resampled with the volume rendering equation)."""
import numpy as np

import synthetic as syn
from oracle import camera_rays, nerf_eval, shade_deferred, sphere_chord, to_local
from tests.test_oracle_nedf import _tiny_nerf, IDENT


def _brute_chord_colour(m, inst, o, d, n):
    """Volume rendering over the bounding chord by an explicit loop over the
    samples: transmittance carried sample by sample."""
    o_l, d_l = to_local(inst, o[None], d[None])
    a, b, valid = sphere_chord(o_l, d_l, m.bound)
    assert valid[0]
    delta_l = (b[0] - a[0]) / n
    T, cw, wsum = 1.0, np.zeros(3), 0.0
    for j in range(n):
        tl = a[0] + (j + 0.5) * delta_l
        x = o_l[0] + tl * d_l[0]
        sig, col = nerf_eval(m, x[None], d_l)
        w = T * (1.0 - np.exp(-sig[0] * delta_l))
        cw += w * col[0]
        wsum += w
        T *= np.exp(-sig[0] * delta_l)
    return cw / wsum


def test_resampling_off_is_plain_deferred_shading():
    m = _tiny_nerf()
    cam = syn.config1_camera(6, 6)
    o, d = camera_rays(cam)
    depth = np.full(36, 3.6)
    ident = np.zeros(36, np.int64)
    a = shade_deferred([m], [IDENT], o, d, depth, ident, K=8)
    b, outl = shade_deferred([m], [IDENT], o, d, depth, ident, K=8, rs_sigma=0.0, return_outliers=True)
    assert np.array_equal(a, b) and not outl.any()


def test_outliers_are_volume_rendered_over_the_chord():
    """A depth far from any density (every sample below the threshold) makes
    the pixel an outlier, shaded by the chord's volume rendering (checked
    against an explicit sample loop); a depth on dense matter does not."""
    m = _tiny_nerf()
    cam = syn.config1_camera(8, 8)
    o, d = camera_rays(cam)
    ident = np.zeros(64, np.int64)
    # density along each ray over the chord: pick, per ray, the densest and
    # a sample beyond the bound (zero density: the network is masked there)
    o_l, d_l = to_local(IDENT, o, d)
    a_, b_, valid = sphere_chord(o_l, d_l, m.bound)
    keep = np.nonzero(valid)[0][:6]
    dense = np.zeros(keep.size)
    for i, r in enumerate(keep):
        ts = a_[r] + (np.arange(64) + 0.5) * (b_[r] - a_[r]) / 64
        sig, _ = nerf_eval(m, o_l[r] + ts[:, None] * d_l[r], np.repeat(d_l[r:r + 1], 64, axis=0))
        dense[i] = ts[np.argmax(sig)]
    depth_far = b_[keep] + 1.0
    thr = 1e-3
    rgb, outl = shade_deferred([m], [IDENT], o[keep], d[keep], depth_far, ident[keep], K=1, rs_sigma=thr,
                               rs_samples=16, return_outliers=True)
    assert outl.all()
    for i, r in enumerate(keep):
        assert np.allclose(rgb[i], _brute_chord_colour(m, IDENT, o[r], d[r], 16), atol=1e-12)
    sig_at, _ = nerf_eval(m, o_l[keep] + dense[:, None] * d_l[keep], d_l[keep])
    assert np.all(sig_at > thr)
    _, outl2 = shade_deferred([m], [IDENT], o[keep], d[keep], dense, ident[keep], K=1, rs_sigma=thr,
                              return_outliers=True)
    assert not outl2.any()


def test_outlier_set_grows_with_the_threshold():
    m = _tiny_nerf()
    cam = syn.config1_camera(8, 8)
    o, d = camera_rays(cam)
    ident = np.zeros(64, np.int64)
    depth = np.linspace(3.0, 5.0, 64)
    prev = None
    for thr in (1e-4, 1e-2, 1.0, 1e2):
        _, outl = shade_deferred([m], [IDENT], o, d, depth, ident, K=4, rs_sigma=thr, return_outliers=True)
        if prev is not None:
            assert np.all(outl | ~prev)
        prev = outl
