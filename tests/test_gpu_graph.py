"""A whole frame (NeDF depth+ID with fallback and refinement, deferred
shading, shadows and composite) captured once in a HIP graph and replayed
several times, with eager work and synchronisations between replays; every
replay must reproduce the eager frame bit for bit (through the C ABI)."""
import numpy as np
import pytest

import synthetic as syn
from tests.gpu_util import need_gpu, log

pytestmark = pytest.mark.gpu


def test_frame_graph_replays_match_eager():
    need_gpu()
    import torch
    from paper_2308_04669_amd import api
    models, insts, cam = syn.sdf_scene(3, 6, width=64, height=48)
    nedfs = [syn.nedf_model(3, 200 + k, head_scale=4.0) for k in range(len(models))]
    objs = [api.object_from_model(m, "bf16", nedf_model=n) for m, n in zip(models, nedfs)]
    sc = api.make_scene(objs, insts)
    rays = api.camera_rays(cam)
    n = cam.n_rays
    light = np.array([[3.0, 6.0, -2.0]])
    dev = "cuda"
    depth = torch.empty(n, dtype=torch.float32, device=dev)
    ident = torch.empty(n, dtype=torch.int32, device=dev)
    rgb = torch.empty((n, 3), dtype=torch.float32, device=dev)
    fac = torch.empty(n, dtype=torch.float32, device=dev)
    ws1, ws2, ws3 = api.Workspace(), api.Workspace(), api.Workspace()

    def frame():
        api.infer_depth_id(sc, rays, dtype="bf16", refine_steps=3, ws=ws1, out=(depth, ident))
        api.shade_deferred(sc, rays, depth, ident, K=8, dtype="bf16", ws=ws2, out=rgb)
        api.shadow(sc, rays, depth, ident, light, eps=0.05, method="nedf", dtype="bf16", rgb_inout=rgb, ws=ws3,
                   out=fac)

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        frame()                      # eager; also sizes every workspace
    torch.cuda.synchronize()
    ref = [t.clone() for t in (depth, ident, rgb, fac)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        frame()
    for rep in range(4):
        for t in (depth, rgb, fac):
            t.fill_(-7.0)
        ident.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        _ = torch.randn(1000, device=dev).sum().item()   # eager work between replays
        for a, b in zip((depth, ident, rgb, fac), ref):
            assert torch.equal(a, b), f"replay {rep} differs"
    log(f"[graph] {int((ref[1] >= 0).sum())} hit pixels reproduced over 4 replays")
