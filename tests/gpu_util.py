"""Shared helpers of the GPU parity tests (not a test module)."""
import sys
from typing import NamedTuple

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


# ---- oracle-side exemption model shared by the parity tests ---------------
# Error model of the library's encoded line features: the line coordinates
# are computed in compensated arithmetic (exact to about 2^-44 |o_l|; 2^-40
# taken), the period reduction is exact, the argument in revolutions rounds
# by at most 1.5 2^-25 after it, and the hardware sine adds at most its
# measured maximum error over [-0.5, 1] revolutions (1.254e-7), doubled.
HW_SIN_ERR = 1.254e-7
SIN_ERR = 2.0 * HW_SIN_ERR + 2.0 * np.pi * 1.5 * 2.0 ** -25
COORD_REL = 2.0 ** -40


def coord_err(o_l, pl):
    return np.broadcast_to(COORD_REL * (np.linalg.norm(o_l, axis=1, keepdims=True) + 1.0), pl.shape)


class PairResult(NamedTuple):
    """Oracle of one instance on a set of rays (see ``pair_oracle``)."""
    hit: np.ndarray     # the pair reports a hit
    D: np.ndarray       # its world depth (nan where no hit)
    p: np.ndarray       # hit probability of the network (nan where not run)
    path: np.ndarray    # 0 network, 1 marcher, 2 no candidate
    A: np.ndarray       # opacity of marched pairs (nan otherwise)
    amb: np.ndarray     # depth ambiguity (world units) of network-routed pairs
    amb_p: np.ndarray   # hit-probability ambiguity of network-routed pairs
    geo: np.ndarray     # a geometric decision (candidate, inside) within its rounding band
    alt: np.ndarray     # smallest depth reported if a banded decision went the other way
    alt_miss: np.ndarray  # a banded decision could turn the pair's hit into no hit
    alt_dev: np.ndarray   # largest |alternative depth - D| of a hit under banded decisions


def near_flags(r, band):
    """Pairs with a decision inside its band: routing at p = 0.2 or 0.8
    (widened by the probability ambiguity), marched hit at opacity 0.5, or
    a geometric decision."""
    with np.errstate(invalid="ignore"):
        return ((np.abs(r.p - 0.2) <= band + r.amb_p) | (np.abs(r.p - 0.8) <= band + r.amb_p)
                | (np.abs(r.A - 0.5) <= band) | r.geo)


def pair_oracle(dens, net, rec, o, d, n_samples, dtype, scales=None, band=2e-2, mx=False):
    """Oracle of one instance (through its single-precision record) on rays
    o, d, as a ``PairResult``.  ``amb`` is the world-depth change
    s l |delta clamp(mu_hat)| and ``amb_p`` the hit-probability change that a
    reduced-precision rounding left open by the method can cause on a
    network-routed pair (input features near a rounding boundary, the
    accumulation order, and for E4M3 hidden activations near a boundary);
    0 for float32.  ``geo`` marks rays whose candidate test (line distance
    against the bounding radius, tangency point ahead) or inside test lies
    within 1e-5 (1 + |o_l|) of its boundary, where single-precision culling
    may decide the other way.  ``alt`` is the smallest depth the pair could
    report if a decision inside ``band`` (widened by amb_p) went the other
    way: the marched depth, the network depth, or for a geometric decision
    the depth lower bound (+inf where no decision is that close)."""
    from oracle import nedf_eval, nedf_pair, pluecker, to_local
    from oracle.ambiguity import nedf_accumulation_sensitivity, nedf_hidden_ambiguity, nedf_input_ambiguity
    from oracle.render import march_instance
    gemm = None if dtype == "f32" else "bf16"
    n = o.shape[0]
    net_fn = None
    if mx:
        from oracle.mx import nedf_eval_mx
        net_fn = lambda ol, dl: nedf_eval_mx(net, ol, dl)  # noqa: E731
    hit, D, p, path = nedf_pair(net, dens, rec, o, d, p_lo=0.2, p_hi=0.8, n_samples=n_samples, gemm=gemm,
                                net_scales=scales, net_fn=net_fn)
    A = np.full(n, np.nan)
    fb = np.nonzero(path == 1)[0]
    Dm = np.full(n, np.nan)
    if fb.size:
        _, A[fb], Dm[fb] = march_instance(dens, rec, o[fb], d[fb], n_samples, None, gemm)
    amb = np.zeros(n)
    amb_p = np.zeros(n)
    # every pair on which the network ran (routed to it, or to the marcher
    # by its probability)
    sel = np.nonzero(np.isfinite(p))[0]
    if mx and sel.size:
        # MX E4M3: every quantisation decision within its value's error
        # bound of the threshold, taken the other way, and (doubled) the
        # move under float32 instead of float64 summation
        from oracle.mx import nedf_eval_mx
        from oracle.fields import sigmoid
        from oracle.ambiguity import nedf_mx_ambiguity
        o_l, d_l = to_local(rec, o[sel], d[sel])
        pl, _ = pluecker(o_l, d_l)
        a_q, p_q, _ = nedf_mx_ambiguity(net, o_l, d_l, coord_err(o_l, pl), SIN_ERR)
        m0, z0 = nedf_eval_mx(net, o_l, d_l)
        m1, z1 = nedf_eval_mx(net, o_l, d_l, acc="f32")
        amb[sel] = rec.s * net.bound * np.maximum(a_q, 2.0 * np.abs(np.clip(m1, -1, 1) - np.clip(m0, -1, 1)))
        amb_p[sel] = np.maximum(p_q, 2.0 * np.abs(sigmoid(z1) - sigmoid(z0)))
    elif net.kind == "nedf16" and sel.size:
        # classifier form: argmax decisions and the hit logit near a tie
        from oracle.ambiguity import classifier_decision_ambiguity
        o_l, d_l = to_local(rec, o[sel], d[sel])
        mu_dev, p_dev = classifier_decision_ambiguity(net, o_l, d_l, gemm=gemm)
        amb[sel] = rec.s * mu_dev
        amb_p[sel] = p_dev
    elif dtype != "f32" and sel.size:
        o_l, d_l = to_local(rec, o[sel], d[sel])
        pl, _ = pluecker(o_l, d_l)
        a_in, _, p_in = nedf_input_ambiguity(net, o_l, d_l, coord_err(o_l, pl), SIN_ERR, scales=scales,
                                             with_p=True)
        a_acc, p_acc = nedf_accumulation_sensitivity(net, o_l, d_l, scales=scales, with_p=True)
        a_mu, a_p = np.maximum(a_in, a_acc), np.maximum(p_in, p_acc)
        if scales is not None:
            h_mu, h_p, _ = nedf_hidden_ambiguity(net, o_l, d_l, scales)
            a_mu, a_p = np.maximum(a_mu, h_mu), np.maximum(a_p, h_p)
        amb[sel] = rec.s * net.bound * a_mu
        amb_p[sel] = a_p
    # geometric decisions
    o_l, d_l = to_local(rec, o, d)
    l = net.bound
    scale = 1e-5 * (1.0 + np.linalg.norm(o_l, axis=1))
    mnorm = np.linalg.norm(np.cross(o_l, d_l), axis=1)
    t_perp = -np.sum(o_l * d_l, axis=1)
    geo = (np.abs(mnorm - l) <= scale) | ((np.abs(t_perp) <= scale) & (mnorm < l + scale))
    geo |= np.abs(np.linalg.norm(o_l, axis=1) - l) <= scale
    res = PairResult(hit, D, p, path, A, amb, amb_p, geo, np.full(n, np.inf), np.zeros(n, bool), np.zeros(n))
    # alternative depths of banded decisions
    with np.errstate(invalid="ignore"):
        lo_b = np.abs(p - 0.2) <= band + amb_p
        hi_b = np.abs(p - 0.8) <= band + amb_p
        a_b = np.abs(A - 0.5) <= band
    alt = np.where(a_b, Dm, np.inf)
    dev = np.zeros(n)
    idx = np.nonzero(lo_b | hi_b)[0]
    if idx.size:
        o_i, d_i = o_l[idx], d_l[idx]
        if mx:
            from oracle.mx import nedf_eval_mx
            mu, _ = nedf_eval_mx(net, o_i, d_i)
        else:
            mu, _ = nedf_eval(net, o_i, d_i, gemm=gemm, scales=scales)
        Dn = rec.s * (t_perp[idx] - l * np.clip(mu, -1.0, 1.0))
        _, Am, Dmi = march_instance(dens, rec, o[idx], d[idx], n_samples, None, gemm)
        march_alt = np.where(Am >= 0.5 - band, Dmi, np.inf)
        net_alt = np.where(hi_b[idx] & (Dn > 0), Dn, np.inf)
        alt[idx] = np.minimum(alt[idx], np.minimum(march_alt, net_alt))
        Di = D[idx]
        with np.errstate(invalid="ignore"):
            dev[idx] = np.maximum(np.where(np.isfinite(march_alt), np.abs(march_alt - Di), 0.0),
                                  np.where(np.isfinite(net_alt), np.abs(net_alt - Di), 0.0))
        dev = np.where(np.isnan(dev), 0.0, dev)
    alt = np.where(geo, np.minimum(alt, rec.s * (t_perp - l)), alt)
    # a hit that a banded decision could lose: routing at 0.2 (a marched
    # hit could become a miss), routing at 0.8 (a network hit could go to
    # the marcher, which may miss), the marched opacity, or geometry
    alt_miss = hit & (lo_b | hi_b | a_b | geo)
    return res._replace(alt=alt, alt_miss=alt_miss, alt_dev=np.where(hit, dev, 0.0))


def refine_with_stability(models, recs, ids, o, d, start, unc, dtype="bf16"):
    """Oracle refinement (3 secant steps, h = 0.05) of each hit from
    ``start``.  The library starts from its own unrefined depth, which may
    lie anywhere within ``unc`` of the oracle's, so the refinement is also
    run from start -+ unc: a pixel is unstable when the three runs disagree
    on whether the seeds bracket the surface (or the guard stops them), or
    all three refine but end more than ``unc_out`` apart.  Returns (refined
    depth, refined at all, unstable, largest spread of refined runs)."""
    from oracle import secant_refine
    gemm = None if dtype == "f32" else "bf16"
    ref = start.copy()
    moved = np.zeros(start.shape, bool)
    unstable = np.zeros(start.shape, bool)
    spread = np.zeros(start.shape)
    for k in np.unique(ids[ids >= 0]):
        sel = np.nonzero(ids == k)[0]
        rec = recs[k]
        u = unc[sel]
        starts = [start[sel] + s_ * u for s_ in (0.0, -1.0, 1.0)]
        outs = [secant_refine(models[rec.model], rec, o[sel], d[sel], st, h=0.05, steps=3, gemm=gemm)
                for st in starts]
        mv = [out != st for out, st in zip(outs, starts)]
        ref[sel] = outs[0]
        moved[sel] = mv[0]
        unstable[sel] = (mv[0] != mv[1]) | (mv[0] != mv[2])
        spread[sel] = np.where(mv[0], np.maximum(np.abs(outs[1] - outs[0]), np.abs(outs[2] - outs[0])), 0.0)
    return ref, moved, unstable, spread
