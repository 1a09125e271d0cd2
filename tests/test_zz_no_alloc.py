"""The fixed-memory entry point (nedf_infer_depth_id_static: no workspace
argument, a per-GPU scratch array, no device allocation) against
nedf_infer_depth_id, through the C ABI: two calls in a row, the second with
a smaller input, each bit-identical to the workspace entry point."""
import numpy as np
import pytest

import synthetic as syn
from tests.gpu_util import need_gpu, gpu_scene, log

pytestmark = pytest.mark.gpu


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_static_entry_point_matches_workspace_entry_point(dtype):
    need_gpu()
    from paper_2308_04669_amd import api, _abi as A
    lib = A.load()
    assert lib.nedf_static_scratch_bytes() == 64 << 20
    models, insts, _ = syn.sdf_scene(3, 6, width=48, height=48)
    nedfs = [syn.nedf_model(3, 200 + k, head_scale=1.0, logit_scale=4.0) for k in range(len(models))]
    sc = gpu_scene(models, insts, dtype, nedf_models=nedfs)
    for size in (48, 20):
        cam = syn.Camera(eye=(0.0, 0.0, 0.0), at=(0.0, 0.0, -1.0), up=(0.0, 1.0, 0.0), fov_y_deg=40.0,
                         width=size, height=size)
        log(f"case: static entry point {dtype} {size}x{size}, 6 instances")
        d_ws, i_ws = api.infer_depth_id(sc, api.camera_rays(cam), dtype=dtype, refine_steps=3)
        d_st, i_st = api.infer_depth_id_static(sc, api.camera_rays(cam), dtype=dtype, refine_steps=3)
        d_ws, i_ws, d_st, i_st = _np(d_ws), _np(i_ws), _np(d_st), _np(i_st)
        hits = int((i_ws >= 0).sum())
        log(f"[static {dtype} {size}] hits={hits} id_equal={np.array_equal(i_ws, i_st)} "
            f"depth_equal={np.array_equal(d_ws.view(np.uint32), d_st.view(np.uint32))}")
        assert hits > 0
        assert np.array_equal(i_ws, i_st)
        assert np.array_equal(d_ws.view(np.uint32), d_st.view(np.uint32))
