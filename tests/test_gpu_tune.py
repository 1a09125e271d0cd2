"""Autotuner: every instantiated superchunk size gives bit-identical results
(it only regroups the weight copies and barriers, not the arithmetic), and
nedf_autotune keeps one of the candidates after timing them all."""
import numpy as np
import pytest

import synthetic as syn
from tests.gpu_util import need_gpu, gpu_scene, log

pytestmark = pytest.mark.gpu


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("nedf_dtype", ["bf16", "fp8"])
def test_nedf_superchunk_variants_identical_and_autotune(nedf_dtype):
    need_gpu()
    import torch
    from paper_2308_04669_amd import api
    models, insts, cam = syn.sdf_scene(3, 6, width=64, height=64)
    nedfs = [syn.nedf_model(3, 200 + k, head_scale=4.0) for k in range(len(models))]
    scales = [None] * len(models)
    if nedf_dtype == "fp8":
        o, d = syn.training_rays(5, 2, 8192)
        scales = [api.fp8_calibrate(n.trunk.W, n.trunk.b, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
                  for n in nedfs]
    objs = [api.object_from_model(m, "bf16", nedf_model=n, nedf_dtype=nedf_dtype,
                                  nedf_scales=None if s is None else s.reshape(-1))
            for m, n, s in zip(models, nedfs, scales)]
    sc = api.make_scene(objs, insts)
    rays = api.camera_rays(cam)
    old = api.tune_get("nedf", nedf_dtype)
    outs = {}
    try:
        for v in api.tune_candidates("nedf", nedf_dtype):
            api.tune_set("nedf", nedf_dtype, v)
            dep, idn = api.infer_depth_id(sc, rays, dtype="bf16", refine_steps=0)
            outs[v] = (_np(dep), _np(idn))
        ref = next(iter(outs.values()))
        for v, (dep, idn) in outs.items():
            log(f"[tune nedf {nedf_dtype}] superchunk {v}: hits {int((idn >= 0).sum())}")
            assert np.array_equal(idn, ref[1]) and np.array_equal(dep.view(np.uint32), ref[0].view(np.uint32))
        rep = api.autotune("nedf", nedf_dtype, sc, rays, api.infer_opts("bf16", refine_steps=0), reps=2)
        log(f"[tune nedf {nedf_dtype}] {rep}")
        assert rep["chosen"] in rep["candidates"] and all(m > 0 for m in rep["ms"])
        assert api.tune_get("nedf", nedf_dtype) == rep["chosen"]
    finally:
        api.tune_set("nedf", nedf_dtype, old)


def test_march_superchunk_variants_identical_and_autotune():
    need_gpu()
    from paper_2308_04669_amd import api
    models, insts, cam, _ = syn.config2_scene(width=48, height=40)
    sc = gpu_scene(models, insts, "bf16")
    rays = api.camera_rays(cam)
    old = api.tune_get("march", "bf16")
    outs = {}
    try:
        for v in api.tune_candidates("march", "bf16"):
            api.tune_set("march", "bf16", v)
            dep, idn, opa = api.march_depth(sc, rays, n_samples=192, dtype="bf16")
            outs[v] = (_np(dep), _np(idn), _np(opa))
        ref = next(iter(outs.values()))
        for v, (dep, idn, opa) in outs.items():
            assert np.array_equal(idn, ref[1]) and np.array_equal(dep.view(np.uint32), ref[0].view(np.uint32))
            assert np.array_equal(opa.view(np.uint32), ref[2].view(np.uint32))
        rep = api.autotune("march", "bf16", sc, rays, api.march_opts(192, dtype="bf16"), reps=1)
        log(f"[tune march bf16] {rep}")
        assert rep["chosen"] in rep["candidates"]
    finally:
        api.tune_set("march", "bf16", old)


def test_depth_slabs_identical():
    """The front-to-back depth slabs skip only pairs that cannot win: depth
    and ID are bit-identical for 1 to 32 slabs, and more slabs evaluate no
    more pairs."""
    need_gpu()
    from paper_2308_04669_amd import api
    models, insts, cam, _ = syn.batched_scene(4, 200, 160, 90)
    nedfs = [syn.nedf_model(4, 200 + k, head_scale=16.0) for k in range(len(models))]
    sc = gpu_scene(models, insts, "bf16", nedf_models=nedfs)
    rays = api.camera_rays(cam)
    old = api.tune_get("slabs", "bf16")
    outs, evald = {}, {}
    try:
        for v in api.tune_candidates("slabs", "bf16"):
            api.tune_set("slabs", "bf16", v)
            ws = api.Workspace()
            dep, idn = api.infer_depth_id(sc, rays, dtype="bf16", refine_steps=0, ws=ws)
            st = api.ws_counters(ws)
            evald[v] = st["nedf_hits"] + st["fallback"] + st["nedf_misses"]
            outs[v] = (_np(dep), _np(idn))
        log(f"[slabs] evaluated pairs {evald} of {st['pairs']}")
        ref = outs[1]
        for v, (dep, idn) in outs.items():
            assert np.array_equal(idn, ref[1]) and np.array_equal(dep.view(np.uint32), ref[0].view(np.uint32))
        assert evald[1] == st["pairs"] and evald[8] <= evald[1] and evald[32] <= evald[1]
    finally:
        api.tune_set("slabs", "bf16", old)
