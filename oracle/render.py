"""Volume-rendering marcher, NeDF decode, composition, refinement, deferred
shading and shadows (FP64).  Test infrastructure only."""
from __future__ import annotations

import numpy as np

from .geometry import to_local, pluecker, sphere_chord
from .fields import density, nerf_eval, nedf_eval, sigmoid, surface_value

F64 = np.float64
CHUNK_SAMPLES = 1 << 18


def march(sigma_fn, o_l, d_l, a, b, n_samples):
    """Volume-rendered depth along local rays (Eq. 5).

    Reading: N midpoint samples t_i = a + (i + 1/2) delta, delta = (b - a)/N,
    no terminal interval; optical depth tau_i = sum_{j<i} sigma_j delta;
    w_i = exp(-tau_i) (1 - exp(-sigma_i delta)).  Returns the opacity
    A = sum w_i, the normalised depth sum w_i t_i / A (NaN where A = 0) and
    the raw Eq. 5 depth sum w_i t_i, all in local units (|d_l| = 1)."""
    o_l = np.asarray(o_l, F64)
    d_l = np.asarray(d_l, F64)
    a = np.asarray(a, F64)
    b = np.asarray(b, F64)
    n = o_l.shape[0]
    A = np.zeros(n)
    raw = np.zeros(n)
    per = max(1, CHUNK_SAMPLES // n_samples)
    for s0 in range(0, n, per):
        sl = slice(s0, min(n, s0 + per))
        delta = (b[sl] - a[sl]) / n_samples
        t = a[sl, None] + (np.arange(n_samples) + 0.5)[None, :] * delta[:, None]
        x = o_l[sl, None, :] + t[..., None] * d_l[sl, None, :]
        sig = np.asarray(sigma_fn(x.reshape(-1, 3)), F64).reshape(t.shape)
        sd = sig * delta[:, None]
        tau = np.cumsum(sd, axis=1) - sd
        w = np.exp(-tau) * (-np.expm1(-sd))
        A[sl] = w.sum(axis=1)
        raw[sl] = (w * t).sum(axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        D = np.where(A > 0, raw / np.where(A > 0, A, 1.0), np.nan)
    return A, D, raw


def march_instance(model, inst, o, d, n_samples, interval=None, gemm=None):
    """March one instance for world rays.  ``interval`` None marches the
    chord of the local bounding sphere (radius ``model.bound``); a pair
    (t_n, t_f) marches that fixed world interval.  World depth is s times the
    local depth (Eq. 7: only depth is scaled).  Returns (valid, A, D_world)."""
    o_l, d_l = to_local(inst, o, d)
    n = o_l.shape[0]
    if interval is None:
        a, b, valid = sphere_chord(o_l, d_l, model.bound)
    else:
        a = np.full(n, interval[0] / inst.s)
        b = np.full(n, interval[1] / inst.s)
        valid = np.ones(n, bool)
    A = np.zeros(n)
    D = np.full(n, np.nan)
    idx = np.nonzero(valid)[0]
    if idx.size:
        Ai, Di, _ = march(lambda x: density(model, x, gemm=gemm), o_l[idx], d_l[idx],
                          a[idx], b[idx], n_samples)
        A[idx] = Ai
        D[idx] = inst.s * Di
    return valid, A, D


def march_compose(models, insts, o, d, n_samples, interval=None, hit_thr=0.5, gemm=None):
    """Step 1 of Alg. 1 with the plain marcher as the per-model depth: for
    each instance in increasing index and each ray, write (D, id) when the
    ray hits (A >= hit_thr) and D is strictly below the buffer (ties keep the
    lower index).  Buffers start at (+inf, -1).  Also returns the opacity
    buffer max_k A_k."""
    n = np.asarray(o).shape[0]
    depth = np.full(n, np.inf)
    ident = np.full(n, -1, np.int64)
    opac = np.zeros(n)
    for k, inst in enumerate(insts):
        valid, A, D = march_instance(models[inst.model], inst, o, d, n_samples, interval, gemm)
        hit = valid & (A >= hit_thr)
        better = hit & (D < depth)
        depth[better] = D[better]
        ident[better] = k
        opac = np.maximum(opac, A)
    return depth, ident, opac


def nedf_pair(nedf_model, dens_model, inst, o, d, p_lo=0.2, p_hi=0.8, n_samples=128,
              hit_thr=0.5, gemm=None, fallback=True, net_fn=None, net_scales=None):
    """NeDF depth of one instance for world rays (Eq. 1, 2, 7), with the
    plain marcher as fallback for uncertain rays.

    Reading: mu = l * clamp(mu_hat, -1, 1) with l the local bounding radius,
    t_perp = -o_l . d_l (signed), D = s (t_perp - mu) (Eq. 2 and Eq. 7);
    p = sigmoid(z).  A ray whose line misses the bounding sphere, or whose
    tangency point lies behind an outside origin, is a miss without running
    the network.  p > p_hi: hit at D if D > 0; p < p_lo: miss; otherwise
    (inclusive band), or when the origin is inside the bounding sphere, the
    marcher decides.  ``fallback=False`` classifies by p >= 0.5 instead.

    ``net_fn(o_l, d_l) -> (mu_hat, z)`` replaces the network (used to plug
    in analytic stand-ins); ``net_scales`` evaluates the network with E4M3
    inputs at those per-layer (w_scale, a_scale) pairs.  Returns (hit, D, p, path) with path 0 = network,
    1 = marcher, 2 = no network evaluation needed (miss)."""
    o_l, d_l = to_local(inst, o, d)
    l = nedf_model.bound
    n = o_l.shape[0]
    _, t_perp = pluecker(o_l, d_l)
    mnorm = np.linalg.norm(np.cross(o_l, d_l), axis=-1)
    inside = np.linalg.norm(o_l, axis=-1) < l
    run = ~inside & (mnorm < l) & (t_perp > 0)
    hit = np.zeros(n, bool)
    D = np.full(n, np.nan)
    p = np.full(n, np.nan)
    path = np.full(n, 2, np.int64)
    idx = np.nonzero(run)[0]
    if idx.size:
        if net_fn is None:
            mu_hat, z = nedf_eval(nedf_model, o_l[idx], d_l[idx], gemm=gemm, scales=net_scales)
        else:
            mu_hat, z = net_fn(o_l[idx], d_l[idx])
        pi = sigmoid(z)
        p[idx] = pi
        Di = inst.s * (t_perp[idx] - l * np.clip(mu_hat, -1.0, 1.0))
        path[idx] = 0
        if fallback:
            conf = (pi > p_hi) & (Di > 0)
            hit[idx[conf]] = True
            D[idx[conf]] = Di[conf]
            band = (pi >= p_lo) & (pi <= p_hi)
            path[idx[band]] = 1
        else:
            conf = (pi >= 0.5) & (Di > 0)
            hit[idx[conf]] = True
            D[idx[conf]] = Di[conf]
    if fallback:
        fb = np.nonzero(inside | (path == 1))[0]
        path[fb] = 1
        if fb.size:
            valid, A, Dm = march_instance(dens_model, inst, o[fb], d[fb], n_samples, None, gemm)
            h = valid & (A >= hit_thr)
            hit[fb] = h
            D[fb] = np.where(h, Dm, np.nan)
    return hit, D, p, path


def nedf_compose(nedf_models, dens_models, insts, o, d, **kw):
    """Alg. 1 step 1 with NeDF depths (and marcher fallback): per-pixel
    minimum over instances, ties to the lower index."""
    n = np.asarray(o).shape[0]
    depth = np.full(n, np.inf)
    ident = np.full(n, -1, np.int64)
    for k, inst in enumerate(insts):
        hit, D, _, _ = nedf_pair(nedf_models[inst.model], dens_models[inst.model], inst, o, d, **kw)
        better = hit & (D < depth)
        depth[better] = D[better]
        ident[better] = k
    return depth, ident


def secant_refine(dens_model, inst, o, d, D_hat, h=0.05, steps=3, gemm=None, margins=False):
    """Secant refinement of a hit depth on the density field near the
    predicted depth.

    Reading: the iteration runs on f(t) = q(G^{-1}(o + t d)) in world t,
    where q is the field's surface function (``surface_value``: the logit of
    sigma / sigma_max, zero on the iso-surface sigma = sigma_max / 2, nearly
    affine across a sharp surface).  h is a distance in the object's own
    (canonical) units, so the world offset is e = h s for an instance of
    scale s.  Seeds t0 = D - e, t1 = D + e, used only when
    f(t0) < 0 <= f(t1).  Each step t+ = t1 - f1 (t1 - t0) / (f1 - f0), then
    (t0, t1) <- (t1, t+).  It stops when the denominator is 0 or an iterate
    leaves [D - 2e, D + 2e]; the last accepted iterate (initially D) is
    returned.  ``steps`` updates need steps + 1 field evaluations.

    ``margins=True`` also returns, per ray, how close its decisions came to
    going the other way: the smaller |f| of the two seeds (the bracket test)
    and the smallest distance of an iterate to the guard interval's ends
    (+inf where no iterate was tested)."""
    o = np.asarray(o, F64)
    d = np.asarray(d, F64)
    D_hat = np.asarray(D_hat, F64)
    n = o.shape[0]

    def f(t, sel):
        o_l, _ = to_local(inst, o[sel] + t[sel, None] * d[sel], d[sel])
        return surface_value(dens_model, o_l, gemm=gemm)

    out = D_hat.copy()
    fmin = np.full(n, np.inf)
    gmin = np.full(n, np.inf)
    if n == 0:
        return (out, fmin, gmin) if margins else out
    allr = np.arange(n)
    e = h * float(inst.s)
    t0, t1 = D_hat - e, D_hat + e
    f0, f1 = f(t0, allr), f(t1, allr)
    fmin = np.minimum(np.abs(f0), np.abs(f1))
    active = (f0 < 0) & (f1 >= 0)
    lo, hi = D_hat - 2 * e, D_hat + 2 * e
    for it in range(steps):
        den = f1 - f0
        ok = active & (den != 0)
        with np.errstate(invalid="ignore", divide="ignore"):
            tn = t1 - f1 * (t1 - t0) / np.where(den != 0, den, 1.0)
        gmin = np.where(ok, np.minimum(gmin, np.minimum(np.abs(tn - lo), np.abs(hi - tn))), gmin)
        ok &= (tn >= lo) & (tn <= hi)
        out = np.where(ok, tn, out)
        active = ok
        if it < steps - 1 and active.any():
            fn = np.zeros(n)
            ia = np.nonzero(active)[0]
            fn[ia] = f(tn, ia)
            t0, f0 = np.where(active, t1, t0), np.where(active, f1, f0)
            t1, f1 = np.where(active, tn, t1), np.where(active, fn, f1)
    return (out, fmin, gmin) if margins else out


def _shade_window(model, inst, o, d, t_lo, step, K, gemm):
    """Local compositing of K samples t_j = t_lo + (j + 1/2) step (world
    units, per ray) of one instance's NeRF: colour sum w_j c_j / sum w_j, or
    c at the sample nearest the window's centre (lower j on a tie) when
    sum w < 1e-6; also the largest density among the samples."""
    t = t_lo[:, None] + (np.arange(K) + 0.5)[None, :] * step[:, None]
    x = o[:, None, :] + t[..., None] * d[:, None, :]
    o_l, d_l = to_local(inst, x.reshape(-1, 3), np.repeat(d, K, axis=0))
    sig, col = nerf_eval(model, o_l, d_l, gemm=gemm)
    sig = sig.reshape(-1, K)
    col = col.reshape(-1, K, 3)
    sd = sig * (step / inst.s)[:, None]
    tau = np.cumsum(sd, axis=1) - sd
    w = np.exp(-tau) * (-np.expm1(-sd))
    ws = w.sum(axis=1)
    near = (K - 1) // 2
    with np.errstate(invalid="ignore", divide="ignore"):
        c = (w[..., None] * col).sum(axis=1) / np.where(ws > 0, ws, 1.0)[:, None]
    c = np.where((ws < 1e-6)[:, None], col[:, near, :], c)
    return c, sig.max(axis=1)


def shade_deferred(models, insts, o, d, depth, ident, K=8, h=0.05, clear=(0.0, 0.0, 0.0),
                   gemm=None, rs_sigma=0.0, rs_samples=32, return_outliers=False):
    """Deferred shading (Eq. 8, Alg. 1 step 2): each pixel with a valid ID is
    shaded by that instance's NeRF near its depth.  Reading (K samples):
    t_j = D - h + (j + 1/2) 2h/K in world units, evaluated in local space
    with local direction; weights from local compositing with step
    (2h/K)/s; rgb = sum w_j c_j / sum w_j, or c at the sample nearest D
    (lower j on a tie) when sum w < 1e-6.  K = 1 is the single evaluation of
    Eq. 8.  Pixels without an ID get the clear colour.

    Outlier processing (Sec. "Deferred Shading": a density that is extremely
    small at the estimated depth means it missed the surface, and such
    pixels can be resampled with the volume rendering equation).  Reading:
    with rs_sigma > 0 a pixel whose density is below rs_sigma at every one
    of its K samples (for K = 1, at D itself) is shaded again by the same
    compositing over the whole chord of the instance's bounding sphere with
    rs_samples midpoint samples.  ``return_outliers`` also returns the mask
    of such pixels."""
    o = np.asarray(o, F64)
    d = np.asarray(d, F64)
    n = o.shape[0]
    rgb = np.tile(np.asarray(clear, F64), (n, 1))
    outl = np.zeros(n, bool)
    for k, inst in enumerate(insts):
        idx = np.nonzero(ident == k)[0]
        if idx.size == 0:
            continue
        model = models[inst.model]
        step = np.full(idx.size, 2.0 * h / K)
        c, smax = _shade_window(model, inst, o[idx], d[idx], depth[idx] - h, step, K, gemm)
        if rs_sigma > 0:
            r = np.nonzero(smax < rs_sigma)[0]
            if r.size:
                o_l, d_l = to_local(inst, o[idx[r]], d[idx[r]])
                a_, b_, valid = sphere_chord(o_l, d_l, model.bound)
                r, a_, b_ = r[valid], a_[valid], b_[valid]
                if r.size:
                    c[r], _ = _shade_window(model, inst, o[idx[r]], d[idx[r]], inst.s * a_,
                                            inst.s * (b_ - a_) / rs_samples, rs_samples, gemm)
                    outl[idx[r]] = True
        rgb[idx] = c
    return (rgb, outl) if return_outliers else rgb


def shadow_factor(depth_fn, o, d, depth, ident, lights, eps, beta=0.5, directional=None, dir_distance=0.0):
    """Shadow step (Alg. 2): for each pixel with a valid ID, x = o + D d; for
    each point light L cast a ray from L towards x and get its depth D_L as
    in step 1 (``depth_fn(origins, dirs) -> depth``, all instances).  The
    pixel is shadowed by L when D_L + eps < |L - x|; each shadowing light
    multiplies the factor by beta (reading for several lights).

    Directional lights (Introduction: parallel light as well as point
    lights): where ``directional[m]`` is set, lights[m] is the direction of
    travel l (normalised here); the shadow ray starts at x - R l with
    R = ``dir_distance`` (beyond every bounding sphere) and runs along l,
    the orthographic counterpart of the point light's ray; shadowed when
    D_L + eps < R."""
    o = np.asarray(o, F64)
    d = np.asarray(d, F64)
    n = o.shape[0]
    fac = np.ones(n)
    idx = np.nonzero(ident >= 0)[0]
    if idx.size == 0:
        return fac
    x = o[idx] + depth[idx, None] * d[idx]
    for m, L in enumerate(lights):
        L = np.asarray(L, F64)
        if directional is not None and directional[m]:
            lv = L / np.linalg.norm(L)
            ds = np.broadcast_to(lv, x.shape).copy()
            DL = depth_fn(x - dir_distance * lv, ds)
            occl = DL + eps < dir_distance
            fac[idx] = np.where(occl, fac[idx] * beta, fac[idx])
            continue
        v = x - L
        dist = np.linalg.norm(v, axis=1)
        ds = v / dist[:, None]
        DL = depth_fn(np.broadcast_to(L, ds.shape).copy(), ds)
        occl = DL + eps < dist
        fac[idx] = np.where(occl, fac[idx] * beta, fac[idx])
    return fac


def composite(rgb, factor):
    """Final image: colour buffer times shadow buffer (Fig. 1 data flow)."""
    return np.asarray(rgb, F64) * np.asarray(factor, F64)[:, None]


def depth_lower_bound(bound, inst, o, d):
    """Lowest world depth any method can report for a (ray, instance) pair,
    or +inf when the pair is no candidate: s (t_perp - l) when the ray's line
    passes within the local bounding radius l and the sphere is not behind an
    outside origin.  The intersection network reports s (t_perp - l clamp(mu_hat))
    and the marcher a depth inside the chord, both at least this bound."""
    o_l, d_l = to_local(inst, o, d)
    _, t_perp = pluecker(o_l, d_l)
    mnorm = np.linalg.norm(np.cross(o_l, d_l), axis=-1)
    inside = np.linalg.norm(o_l, axis=-1) < bound
    cand = (mnorm < bound) & ((t_perp > 0) | inside)
    return np.where(cand, inst.s * (t_perp - bound), np.inf)


def compose_pruned(pair_fn, lower_bounds):
    """Alg. 1 step 1 with exact pruning (front to back).

    ``lower_bounds`` is [n_inst, n]: for each instance and ray a lower bound
    on any depth the pair can report (+inf: no candidate).  Each ray visits
    its candidates in increasing bound order and stops once the next bound
    exceeds the best depth so far; since no skipped pair could report a
    depth below its bound, the result equals the full minimum over all
    instances in increasing index with ties to the lower index.
    ``pair_fn(k, idx) -> (hit [m], D [m])`` evaluates instance k on the rays
    ``idx``.  Returns (depth, id, pairs evaluated)."""
    lb = np.asarray(lower_bounds, F64)
    n_inst, n = lb.shape
    depth = np.full(n, np.inf)
    ident = np.full(n, -1, np.int64)
    order = np.argsort(lb, axis=0, kind="stable")
    cols = np.arange(n)
    evaluated = 0
    for r in range(n_inst):
        k_r = order[r]
        b_r = lb[k_r, cols]
        need = np.isfinite(b_r) & (b_r <= depth)
        if not need.any():
            break
        for k in np.unique(k_r[need]):
            idx = np.nonzero(need & (k_r == k))[0]
            hit, D = pair_fn(int(k), idx)
            evaluated += idx.size
            cur, cid = depth[idx], ident[idx]
            better = hit & ((D < cur) | ((D == cur) & (k < cid)))
            depth[idx[better]] = D[better]
            ident[idx[better]] = k
    return depth, ident, evaluated


def march_compose_pruned(models, insts, o, d, n_samples, hit_thr=0.5, gemm=None):
    """``march_compose`` on the bounding chords with exact pruning: same
    depth and id buffers, fewer marched pairs.  Returns (depth, id, pairs)."""
    o = np.asarray(o, F64)
    d = np.asarray(d, F64)
    lb = np.array([depth_lower_bound(models[i.model].bound, i, o, d) for i in insts])

    def pair(k, idx):
        inst = insts[k]
        valid, A, D = march_instance(models[inst.model], inst, o[idx], d[idx], n_samples, None, gemm)
        return valid & (A >= hit_thr), D

    return compose_pruned(pair, lb)


def nedf_compose_pruned(nedf_models, dens_models, insts, o, d, **kw):
    """``nedf_compose`` with exact pruning: same depth and id buffers.
    Returns (depth, id, pairs)."""
    o = np.asarray(o, F64)
    d = np.asarray(d, F64)
    lb = np.array([depth_lower_bound(nedf_models[i.model].bound, i, o, d) for i in insts])

    def pair(k, idx):
        inst = insts[k]
        hit, D, _, _ = nedf_pair(nedf_models[inst.model], dens_models[inst.model], inst, o[idx], d[idx], **kw)
        return hit, D

    return compose_pruned(pair, lb)
