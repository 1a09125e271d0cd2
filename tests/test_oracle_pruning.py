"""Pins of the oracle's front-to-back composition with exact pruning
(Alg. 1 step 1): on tiny scenes it must return exactly the depth and id
buffers of the brute-force minimum over every instance (CPU only)."""
import numpy as np

import synthetic as syn
from oracle import (camera_rays, march_compose, march_compose_pruned, nedf_compose, nedf_compose_pruned,
                    nedf_pair, depth_lower_bound)
from oracle.render import march_instance


def _sphere_scene(n_inst=8, seed=31):
    a, _ = syn.config1_models()
    hard = syn.Model(kind="hard_sphere", bound=1.0, params=dict(sigma0=40.0, radius=0.7))
    g = syn.rng(0, seed)
    insts = []
    for k in range(n_inst):
        insts.append(syn.Instance(k % 2, syn.shoemake_rotation(g), g.uniform(-0.8, 0.8, 3) + np.array([0, 0, -5.0]),
                                  float(g.uniform(0.5, 1.3))))
    # an exact duplicate of instance 2 placed after it: every depth ties, the lower index wins
    insts.append(syn.Instance(insts[2].model, insts[2].R.copy(), insts[2].T.copy(), insts[2].s))
    cam = syn.Camera(eye=(0.0, 0.0, 0.0), at=(0.0, 0.0, -1.0), up=(0, 1, 0), fov_y_deg=40.0, width=8, height=8)
    return [a, hard], insts, cam


def test_march_pruned_equals_brute_force():
    models, insts, cam = _sphere_scene()
    o, d = camera_rays(cam)
    D0, I0, _ = march_compose(models, insts, o, d, 64)
    D1, I1, pairs = march_compose_pruned(models, insts, o, d, 64)
    assert np.array_equal(I0, I1)
    assert np.array_equal(D0, D1)
    assert (I0 >= 0).sum() > 20
    # the duplicate never wins: its twin has the lower index
    assert not np.any(I1 == len(insts) - 1)
    # fewer pairs than the brute force evaluates
    cand = sum(np.isfinite(depth_lower_bound(models[i.model].bound, i, o, d)).sum() for i in insts)
    assert pairs < cand


def test_march_pruned_permutation_invariant():
    models, insts, cam = _sphere_scene()
    insts = insts[:-1]          # no exact duplicates: no ties
    o, d = camera_rays(cam)
    D0, I0, _ = march_compose_pruned(models, insts, o, d, 64)
    perm = np.random.default_rng(2).permutation(len(insts))
    D1, I1, _ = march_compose_pruned(models, [insts[p] for p in perm], o, d, 64)
    assert np.array_equal(D0, D1)
    assert np.array_equal(I0, np.where(I1 >= 0, perm[np.maximum(I1, 0)], -1))


def test_lower_bound_never_exceeds_a_reported_depth():
    models, insts, cam = _sphere_scene()
    o, d = camera_rays(cam)
    for inst in insts:
        lb = depth_lower_bound(models[inst.model].bound, inst, o, d)
        valid, A, D = march_instance(models[inst.model], inst, o, d, 64)
        hit = valid & (A >= 0.5)
        assert np.all(np.isfinite(lb[valid]))          # every marchable pair is a candidate
        assert np.all(D[hit] >= lb[hit])


def test_nedf_pruned_equals_brute_force():
    models, insts, cam = syn.sdf_scene(3, 8, width=8, height=8, z_range=(3.0, 5.0), spread=0.6)
    nets = [syn.nedf_model(3, 200 + k, head_scale=4.0) for k in range(len(models))]
    o, d = camera_rays(cam)
    kw = dict(n_samples=32)
    D0, I0 = nedf_compose(nets, models, insts, o, d, **kw)
    D1, I1, pairs = nedf_compose_pruned(nets, models, insts, o, d, **kw)
    assert np.array_equal(I0, I1)
    # the network's matrix products run on a different batch of rows, which
    # the BLAS library may sum in another order: equal to float64 rounding
    assert np.array_equal(np.isfinite(D0), np.isfinite(D1))
    fin = np.isfinite(D0)
    assert np.allclose(D0[fin], D1[fin], rtol=0, atol=1e-12)
    assert (I0 >= 0).sum() > 10
    # every reported depth respects its pair's bound (network and fallback paths)
    paths = set()
    for inst in insts:
        hit, D, p, path = nedf_pair(nets[inst.model], models[inst.model], inst, o, d, **kw)
        lb = depth_lower_bound(nets[inst.model].bound, inst, o, d)
        assert np.all(D[hit] >= lb[hit])
        paths |= set(np.unique(path[hit]).tolist())
    assert paths == {0, 1}
