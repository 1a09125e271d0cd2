"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, and rejects bad arguments on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nedf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nedf_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported():
    from paper_2308_04669_amd import _abi as A
    lib = A.load()
    names = _declared()
    assert "nedf_march_depth" in names
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in A.SIGNATURES}
    assert set(names) <= bound, set(names) - bound


def test_version_and_status_strings():
    from paper_2308_04669_amd import _abi as A
    lib = A.load()
    assert lib.nedf_version().startswith(b"nedf-mi355x")
    for k in range(9):
        assert lib.nedf_status_string(k)


def test_pack_rejects_bad_shapes():
    from paper_2308_04669_amd import api, _abi as A
    with pytest.raises(A.NedfError):
        api.packed_bytes(api.mlp_shape("xyz", 10, 100, 8, 1), "bf16")
    with pytest.raises(A.NedfError):
        api.packed_bytes(api.mlp_shape("xyz", 10, 256, 1, 1), "bf16")
    lib = A.load()
    s = A.MlpShape(0, 6, 64, 3, 1, 0, 0)
    assert lib.nedf_pack_mlp(C.byref(s), 1, None, None, None, None, 0) == 1
    n = lib.nedf_mlp_packed_bytes(C.byref(s), 1)
    buf = np.zeros(16, np.uint8)
    W = (C.c_void_p * 4)(1, 1, 1, 1)
    assert lib.nedf_pack_mlp(C.byref(s), 1, W, W, None, buf.ctypes.data, 16) == 5
    assert n > 0


def test_host_validation_before_launch():
    """Argument errors are reported without touching the device."""
    from paper_2308_04669_amd import _abi as A
    lib = A.load()
    opts = A.MarchOpts(128, 1, 0.0, 0.0, 0.5, 0)
    r = A.Rays()
    r.kind = 0
    r.camera.width, r.camera.height, r.camera.fov_y_deg = 4, 4, 40.0
    r.camera.eye[2] = 4.0
    r.camera.up[1] = 1.0
    # NULL scene
    assert lib.nedf_march_depth(None, C.byref(r), C.byref(opts), None, None, None, None, 0, None) == 1
    obj = (A.Object * 1)()
    obj[0].field, obj[0].bound = 0, 1.0
    obj[0].param[0], obj[0].param[1], obj[0].param[2] = 50.0, 0.5, 0.01
    sc = A.Scene(1, C.cast(obj, C.POINTER(A.Object)), 1, 16, 16)
    # n_samples out of range
    bad = A.MarchOpts(0, 1, 0.0, 0.0, 0.5, 0)
    assert lib.nedf_march_depth(C.byref(sc), C.byref(r), C.byref(bad), 16, 16, None, 16, 1 << 20, None) == 2
    # fixed interval with t_far <= t_near
    bad = A.MarchOpts(64, 0, 3.0, 2.0, 0.5, 0)
    assert lib.nedf_march_depth(C.byref(sc), C.byref(r), C.byref(bad), 16, 16, None, 16, 1 << 20, None) == 2
    # misaligned output
    assert lib.nedf_march_depth(C.byref(sc), C.byref(r), C.byref(opts), 18, 16, None, 16, 1 << 20, None) == 4
    # workspace too small
    assert lib.nedf_march_depth(C.byref(sc), C.byref(r), C.byref(opts), 16, 16, None, 16, 64, None) == 5
    # MLP object without a blob
    obj[0].field = 2
    assert lib.nedf_march_depth(C.byref(sc), C.byref(r), C.byref(opts), 16, 16, None, 16, 1 << 20, None) == 1
    # workspace query
    obj[0].field = 0
    assert lib.nedf_workspace_size(0, C.byref(sc), C.byref(r), 0) >= 16 * 8 + 256
    assert b"must" in lib.nedf_last_error() or lib.nedf_last_error()


def test_tuning_table_host_logic():
    """Tuning table: candidates per (kernel, dtype), get/set with rejection of
    values that are not instantiated (host-only calls)."""
    from paper_2308_04669_amd import _abi as A
    from paper_2308_04669_amd import api
    assert api.tune_candidates("march", "f32") == [11]
    assert api.tune_candidates("march", "bf16") == [11, 12, 21, 111, 112, 1011, 1012]
    assert api.tune_candidates("nedf", "bf16") == [11, 12, 21, 111, 112, 1011, 1012]
    assert api.tune_candidates("nedf", "fp8") == [11, 12, 14, 21, 22, 1011, 1012, 1014]
    assert api.tune_candidates("slabs", "bf16") == [1, 2, 4, 8, 16, 32]
    with pytest.raises(A.NedfError):
        api.tune_candidates("march", "fp8")
    old = api.tune_get("nedf", "bf16")
    assert old in api.tune_candidates("nedf", "bf16")
    api.tune_set("nedf", "bf16", 21)
    assert api.tune_get("nedf", "bf16") == 21
    with pytest.raises(A.NedfError) as e:
        api.tune_set("nedf", "bf16", 3)
    assert e.value.status == 8
    api.tune_set("nedf", "bf16", old)
    lib = A.load()
    rep = A.TuneReport()
    # NULL arguments and a bad repetition count are rejected before any launch
    assert lib.nedf_autotune(1, 1, None, None, None, None, None, None, 0, 1, None, C.byref(rep)) == 1


def test_static_entry_point_rejects_oversized_calls_on_the_host():
    """The fixed-memory entry point rejects a call whose worst-case pair list
    (every ray meeting every instance) exceeds its 64 MiB scratch, before
    any device work (so this runs without a GPU)."""
    from paper_2308_04669_amd import _abi as A
    lib = A.load()
    assert lib.nedf_static_scratch_bytes() == 64 << 20
    sc = A.Scene()
    sc.n_objects = 1
    sc.n_inst = 1000
    rays = A.Rays()
    rays.kind = 0
    rays.camera.width, rays.camera.height = 1920, 1080
    rays.camera.fov_y_deg = 40.0
    rays.camera.at[2] = -1.0
    rays.camera.up[1] = 1.0
    opts = A.InferOpts()
    st = lib.nedf_infer_depth_id_static(C.byref(sc), C.byref(rays), C.byref(opts), None, None, None)
    assert st == 5  # NEDF_ERR_WORKSPACE
    assert b"64" in lib.nedf_last_error() or b"67108864" in lib.nedf_last_error()
