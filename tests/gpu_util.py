"""Shared helpers of the GPU parity tests (not a test module)."""
import sys

import numpy as np
import pytest

import synthetic as syn


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_04669_amd import api  # noqa: F401  (raises if the library is missing)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_scene(models, insts, dtype="f32", nedf_models=None):
    from paper_2308_04669_amd import api
    objs = []
    for i, m in enumerate(models):
        nm = None if nedf_models is None else nedf_models[i]
        objs.append(api.object_from_model(m, dtype, nedf_model=nm))
    return api.make_scene(objs, insts)


def per_instance(models, insts, o, d, n_samples, interval=None, gemm=None):
    """Oracle (A, D) of every (ray, instance) pair: arrays [n_inst, n]."""
    from oracle.render import march_instance
    As, Ds, Vs = [], [], []
    for inst in insts:
        v, A, D = march_instance(models[inst.model], inst, o, d, n_samples, interval, gemm)
        As.append(A)
        Ds.append(np.where(v & (A >= 0.5), D, np.inf))
        Vs.append(v)
    return np.array(As), np.array(Ds), np.array(Vs)


def compare_depth_id(depth_g, id_g, opac_g, As, Ds, depth_tol, thr_band, tie_tol, opac_tol=None, label=""):
    """Parity of (depth, id) against per-instance oracle values.

    A pixel is exempt from the ID check when its two smallest candidate
    depths are within ``tie_tol`` or any candidate's opacity is within
    ``thr_band`` of the 0.5 threshold (genuine near-ties).  Returns stats."""
    n = depth_g.shape[0]
    best = Ds.min(axis=0)
    id_o = np.where(np.isfinite(best), Ds.argmin(axis=0), -1)
    srt = np.sort(Ds, axis=0)
    if Ds.shape[0] > 1:
        gap = np.where(np.isfinite(srt[1]), srt[1] - np.where(np.isfinite(srt[0]), srt[0], 0.0), np.inf)
    else:
        gap = np.full(n, np.inf)
    near_thr = (np.abs(As - 0.5) <= thr_band).any(axis=0)
    exempt = near_thr | (np.isfinite(srt[0]) & (gap <= tie_tol))
    id_bad = (id_g != id_o) & ~exempt
    both = (id_g == id_o) & (id_o >= 0)
    err = np.abs(depth_g[both] - best[both])
    stats = dict(n=n, hits=int((id_o >= 0).sum()), exempt=int(exempt.sum()), id_mismatch=int(id_bad.sum()),
                 depth_max_err=float(err.max()) if err.size else 0.0,
                 depth_med_err=float(np.median(err)) if err.size else 0.0)
    if opac_g is not None:
        oerr = np.abs(opac_g - As.max(axis=0))
        stats["opac_max_err"] = float(oerr.max())
    log(f"[{label}] {stats}")
    assert stats["id_mismatch"] == 0, stats
    assert stats["depth_max_err"] <= depth_tol, stats
    if opac_tol is not None and opac_g is not None:
        assert stats["opac_max_err"] <= opac_tol, stats
    miss = id_o < 0
    assert np.all(np.isinf(depth_g[miss & ~exempt])), "miss pixels must have +inf depth"
    return stats
