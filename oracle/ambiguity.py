"""Where a reduced-precision result is not fixed by the method alone (FP64;
test infrastructure only).

A bfloat16 network rounds every operand of its matrix products to 8
significant bits.  An implementation computes the first layer's operands (the
encoded line coordinates) in single precision, so a feature whose exact value
lies closer to a rounding boundary than that computation's error can round to
either neighbour; and the single-precision accumulation of each matrix product
has no prescribed summation order.  Both are left open by the method, so two
correct implementations can differ on such rays by more than the bfloat16
depth tolerance.  The functions here find those rays from the oracle's own
arithmetic; a parity test exempts exactly them and holds every other ray to
the tolerance.
"""
from __future__ import annotations

import numpy as np

from .fields import mlp_forward, sigmoid
from .geometry import encode, pluecker
from .rounding import bf16_rounding_margin, e4m3_rounding_margin, round_bf16, round_e4m3

F64 = np.float64


def f32_ulp(x):
    """Spacing of float32 values at |x| (one unit in the last place)."""
    return np.spacing(np.abs(np.asarray(x, F64)).astype(np.float32)).astype(F64)


def encoding_error_bound(coord_err, L, sin_err):
    """Absolute error bound of each encoded feature [p, sin(2^0 pi p),
    cos(2^0 pi p), ..., sin(2^{L-1} pi p), cos(2^{L-1} pi p)] (the layout of
    ``encode``) when the coordinates p carry absolute error ``coord_err``
    [n, c] and each sine or cosine adds at most ``sin_err``: the k-th level
    multiplies the coordinate error by its frequency 2^k pi."""
    e = np.asarray(coord_err, F64)
    parts = [e]
    for k in range(L):
        ek = (2.0 ** k) * np.pi * e + sin_err
        parts += [ek, ek]
    return np.concatenate(parts, axis=-1)


def _other_neighbour(x, margin_abs, rnd=round_bf16):
    """The value of the format rounded to by ``rnd`` on the far side of the
    rounding boundary nearest to x, whose distance from x is ``margin_abs``:
    x moved just past that distance toward the boundary rounds to it, and
    moved the other way by the same amount it still rounds to x's own
    value (the other boundary is at least as far)."""
    x = np.asarray(x, F64)
    m = np.asarray(margin_abs, F64)
    q = rnd(x)
    step = m * (1.0 + 1e-6) + np.abs(x) * 1e-15 + 1e-300
    up = rnd(x + step)
    return np.where(up != q, up, rnd(x - step))


def _features(model, o_l, d_l):
    pl, _ = pluecker(np.asarray(o_l, F64), np.asarray(d_l, F64))
    return encode(pl, model.params["enc_L"])


def _head_delta(out, base):
    """|change| of clamp(mu_hat, -1, 1) and of the hit probability
    sigmoid(z) between two head outputs [m, 2]."""
    dmu = np.abs(np.clip(out[:, 0], -1.0, 1.0) - np.clip(base[:, 0], -1.0, 1.0))
    dp = np.abs(sigmoid(out[:, 1]) - sigmoid(base[:, 1]))
    return dmu, dp


def nedf_input_ambiguity(model, o_l, d_l, coord_err, sin_err, max_alternatives=64, scales=None, with_p=False):
    """For each ray, the largest change of the clamped network depth output
    clamp(mu_hat, -1, 1) when encoded input features whose exact value lies
    within its error bound (``encoding_error_bound``) of a rounding boundary
    of the first layer's operand format are rounded to the other neighbour:
    each such feature alone, and all of them together.  The format is
    bfloat16, or E4M3 of the feature divided by the first layer's activation
    scale when per-layer ``scales`` are given.  0 where no feature is that
    close.  Returns (ambiguity [n], number of such features [n]), and with
    ``with_p`` also the largest change of the hit probability sigmoid(z)."""
    L = model.params["enc_L"]
    x = _features(model, o_l, d_l)
    err = encoding_error_bound(coord_err, L, sin_err)
    if scales is None:
        a0, rnd, marg = 1.0, round_bf16, bf16_rounding_margin
        fwd = lambda xx: mlp_forward(xx, model.trunk, gemm="bf16")
    else:
        a0, rnd, marg = float(scales[0][1]), round_e4m3, e4m3_rounding_margin
        fwd = lambda xx: mlp_forward(xx, model.trunk, scales=scales)
    y = x / a0
    margin = marg(y) * np.abs(y)
    close = margin < err / a0
    count = close.sum(axis=1)
    amb = np.zeros(x.shape[0])
    amb_p = np.zeros(x.shape[0])
    rows = np.nonzero(count > 0)[0]
    if rows.size == 0:
        return (amb, count, amb_p) if with_p else (amb, count)
    base = fwd(x[rows])
    alts, owner = [], []
    for j, r in enumerate(rows):
        feats = np.nonzero(close[r])[0][:max_alternatives]
        alt_vals = _other_neighbour(y[r, feats], margin[r, feats], rnd) * a0
        for f, v in zip(feats, alt_vals):
            xa = x[r].copy()
            xa[f] = v
            alts.append(xa)
            owner.append(j)
        if feats.size > 1:
            xa = x[r].copy()
            xa[feats] = alt_vals
            alts.append(xa)
            owner.append(j)
    owner = np.array(owner)
    dmu, dp = _head_delta(fwd(np.array(alts)), base[owner])
    per, per_p = np.zeros(rows.size), np.zeros(rows.size)
    np.maximum.at(per, owner, dmu)
    np.maximum.at(per_p, owner, dp)
    amb[rows] = per
    amb_p[rows] = per_p
    return (amb, count, amb_p) if with_p else (amb, count)


def nedf_hidden_ambiguity(model, o_l, d_l, scales, max_alternatives=32):
    """E4M3 networks: for each ray, the largest change of clamp(mu_hat) and
    of sigmoid(z) when one hidden layer's quantised input is rounded to the
    other E4M3 neighbour because its exact value lies within the
    single-precision accumulation error of the layer before of a rounding
    boundary (or of the ReLU kink).  That error is bounded by
    gamma_K sum |a w| (gamma_K = K u / (1 - K u), u = 2^-24, K the fan-in)
    plus a few units of the result for the scale and bias.  Each such value
    is flipped alone and the network re-evaluated from that layer on.
    Returns (ambiguity of clamp(mu_hat) [n], of sigmoid(z) [n], number of
    such values [n])."""
    x = _features(model, o_l, d_l)
    n = x.shape[0]
    W = [np.asarray(w, F64) for w in model.trunk.W]
    b = [np.asarray(v, F64) for v in model.trunk.b]
    nh = len(W) - 1
    u = 2.0 ** -24

    def run_from(i, q_in):
        """Forward from hidden layer i given its quantised input q_in
        (E4M3 codes of input / a_i), to the head output [m, 2]."""
        h = None
        q = q_in
        for j in range(i, nh):
            ws, as_ = scales[j]
            z = (q @ round_e4m3(W[j] / ws).T) * (as_ * ws) + b[j]
            h = np.maximum(z, 0.0)
            if j + 1 < nh:
                q = round_e4m3(h / scales[j + 1][1])
        return h @ W[-1].T + b[-1]

    # forward keeping each hidden layer's quantised input and the bound on
    # the accumulation error of the pre-activation that produced it
    qs = [round_e4m3(x / scales[0][1])]
    flags = []
    for j in range(nh - 1):
        ws, as_ = scales[j]
        qw = round_e4m3(W[j] / ws)
        z = (qs[j] @ qw.T) * (as_ * ws) + b[j]
        K = qw.shape[1]
        gam = K * u / (1.0 - K * u)
        err = gam * (np.abs(qs[j]) @ np.abs(qw).T) * (as_ * ws) + 4 * u * (np.abs(z) + np.abs(b[j]))
        a_next = scales[j + 1][1]
        y = np.maximum(z, 0.0) / a_next
        with np.errstate(invalid="ignore"):
            marg = np.where(y > 0, e4m3_rounding_margin(y) * np.abs(y), np.inf)
        close = (marg < err / a_next) | (np.abs(z) <= err)
        qs.append(round_e4m3(y))
        flags.append((close, y, marg, err / a_next, z))
    base = run_from(0, qs[0])
    amb = np.zeros(n)
    amb_p = np.zeros(n)
    count = np.zeros(n, np.int64)
    for j, (close, y, marg, e, z) in enumerate(flags):
        rows, units = np.nonzero(close)
        if rows.size == 0:
            continue
        count += np.bincount(rows, minlength=n)
        # at most max_alternatives per ray and layer
        keep = np.concatenate([np.nonzero(rows == r)[0][:max_alternatives] for r in np.unique(rows)])
        rows, units = rows[keep], units[keep]
        q_alt = qs[j + 1][rows].copy()
        yv = y[rows, units]
        kink = np.abs(z[rows, units]) <= e[rows, units] * scales[j + 1][1]
        alt = np.where(kink & (q_alt[np.arange(rows.size), units] == 0.0),
                       round_e4m3(np.abs(e[rows, units])),   # ReLU output could be positive
                       _other_neighbour(yv, marg[rows, units], round_e4m3))
        q_alt[np.arange(rows.size), units] = alt
        dmu, dp = _head_delta(run_from(j + 1, q_alt), base[rows])
        np.maximum.at(amb, rows, dmu)
        np.maximum.at(amb_p, rows, dp)
        # all of a ray's close values of this layer flipped together
        ur = np.unique(rows)
        q_all = qs[j + 1][ur].copy()
        pos = np.searchsorted(ur, rows)
        q_all[pos, units] = alt
        dmu, dp = _head_delta(run_from(j + 1, q_all), base[ur])
        np.maximum.at(amb, ur, dmu)
        np.maximum.at(amb_p, ur, dp)
    return amb, amb_p, count


def nedf_accumulation_sensitivity(model, o_l, d_l, scales=None, with_p=False):
    """For each ray, |clamp(mu_hat)| under float32 summation of the hidden
    layers' products minus the same under float64 summation (bfloat16
    operands, or E4M3 operands at the per-layer ``scales``): how far the
    result moves with the accumulator's precision and summation order alone
    (the operands are identical).  With ``with_p`` also the change of the
    hit probability sigmoid(z)."""
    x = _features(model, o_l, d_l)
    kw = dict(gemm="bf16") if scales is None else dict(scales=scales)
    dmu, dp = _head_delta(mlp_forward(x, model.trunk, acc="f32", **kw), mlp_forward(x, model.trunk, **kw))
    return (dmu, dp) if with_p else dmu


def classifier_decision_ambiguity(model, o_l, d_l, gemm=None, margin=2.0):
    """How far the decoded mu (local units) and the hit probability of the
    classifier-form network may move when its argmax decisions or its hit
    logit are taken with another summation order (Eq. 4 decodes by argmax, a
    decision the logits' rounding can flip on a near-tie).  The logits are
    computed with float64 and with float32 accumulation; eps is ``margin``
    times the larger of the pair's largest logit difference and a batch-wide
    floor: the 90th percentile of it in float32 (unrounded activations: the
    difference is a smooth function of the summation order), its maximum
    with ``gemm="bf16"``, where a summation difference can move one of the
    ~8,000 rounded activations of a pair across a rounding boundary, a jump
    of one bfloat16 step that the other order may take at another pair (in
    the batch's measured tail).  A coarse bin j with v_c* - v_j <= eps moves mu by
    |j - c*| 2l / N_c, a fine bin by |f - f*| 2l / (N_c N_f); the returned
    mu deviation is the largest coarse move plus the largest fine move.
    Returns (mu_dev [n], p_dev [n])."""
    from .classifier import classifier_forward, encode_points, line_points
    from .fields import sigmoid
    l = model.bound
    nc, nf = model.params["n_coarse"], model.params["n_fine"]
    feats = encode_points(line_points(o_l, d_l, l, model.params["n_points"]), model.params["enc_L"])
    a0, c0, f0 = classifier_forward(model, feats, gemm=gemm)
    a1, c1, f1 = classifier_forward(model, feats, gemm=gemm, acc="f32")
    dl = np.maximum(np.abs(c1 - c0).max(axis=1), np.abs(f1 - f0).max(axis=1))
    da = np.abs(a1 - a0)
    if dl.size == 0:
        return np.zeros(0), np.zeros(0)
    q = 0.9 if gemm is None else 1.0
    eps = margin * np.maximum(dl, np.quantile(dl, q))
    eps_a = margin * np.maximum(da, np.quantile(da, q))

    def largest_move(v, step):
        best = np.argmax(v, axis=1)
        top = v[np.arange(v.shape[0]), best]
        near = (top[:, None] - v) <= eps[:, None]
        dist = np.abs(np.arange(v.shape[1])[None, :] - best[:, None]) * near
        return dist.max(axis=1) * step

    mu_dev = largest_move(c0, 2.0 * l / nc) + largest_move(f0, 2.0 * l / (nc * nf))
    p_dev = np.maximum(np.abs(sigmoid(a0 + eps_a) - sigmoid(a0)), np.abs(sigmoid(a0 - eps_a) - sigmoid(a0)))
    return mu_dev, p_dev


def nedf_mx_ambiguity(model, o_l, d_l, coord_err, sin_err, max_alternatives=32):
    """MX block-scaled E4M3 networks (``oracle.mx``): for each ray, the
    largest change of clamp(mu_hat) and of sigmoid(z) when a quantisation
    decision of some layer's input lies within that value's error bound of
    its threshold, decided the other way and the network re-run from that
    layer.  Values: the encoded features (bound ``encoding_error_bound``) and
    each hidden layer's output (single-precision accumulation bound
    gamma_K sum |a w| plus a few units of the result).  Decisions: the E4M3
    rounding of a value in its block's scaled units; the ReLU kink; and a
    block's shared exponent, when amax lies within its bound of a step of it
    (the whole block re-quantised one exponent up or
    down; the exponent steps where amax crosses 448 times a power of two).
    Each decision alone, and all of a layer's together, the ambiguity being
    the larger of the largest such change and the sum over layers of the
    all-together changes (first-order effect of several layers).  Returns
    (ambiguity of clamp(mu_hat) [n], of sigmoid(z) [n], decisions [n])."""
    from .mx import mx_quantize, hidden_blocks, encoded_blocks, mx_exponent
    x = _features(model, o_l, d_l)
    n = x.shape[0]
    L = model.params["enc_L"]
    W = [np.asarray(w, F64) for w in model.trunk.W]
    b = [np.asarray(v, F64) for v in model.trunk.b]
    nh = len(W) - 1
    u = 2.0 ** -24
    blocks = [encoded_blocks(6, L)] + [hidden_blocks(W[j].shape[1]) for j in range(1, nh)]
    Wq = [mx_quantize(W[j], blocks[j])[0] for j in range(nh)]

    def run_from(j, hq):
        h = None
        for jj in range(j, nh):
            h = np.maximum(hq @ Wq[jj].T + b[jj], 0.0)
            if jj + 1 < nh:
                hq = mx_quantize(h, blocks[jj + 1])[0]
        return h @ W[-1].T + b[-1]

    # each layer's value before quantisation, its error bound, and (hidden)
    # its pre-activation
    vals = [x]
    errs = [encoding_error_bound(coord_err, L, sin_err)]
    pre = [None]
    hq = mx_quantize(x, blocks[0])[0]
    hqs = [hq]
    for j in range(nh - 1):
        z = hq @ Wq[j].T + b[j]
        K = Wq[j].shape[1]
        gam = K * u / (1.0 - K * u)
        err = gam * (np.abs(hq) @ np.abs(Wq[j]).T) + 4 * u * (np.abs(z) + np.abs(b[j]))
        y = np.maximum(z, 0.0)
        vals.append(y)
        errs.append(err)
        pre.append(z)
        hq = mx_quantize(y, blocks[j + 1])[0]
        hqs.append(hq)
    base = run_from(0, hqs[0])
    amb = np.zeros(n)
    amb_p = np.zeros(n)
    sum_mu = np.zeros(n)
    sum_p = np.zeros(n)
    count = np.zeros(n, np.int64)

    def apply(j, rows, alts):
        """Re-run from layer j with per-row altered quantised inputs."""
        dmu, dp = _head_delta(run_from(j, alts), base[rows])
        np.maximum.at(amb, rows, dmu)
        np.maximum.at(amb_p, rows, dp)

    for j in range(nh):
        y, e, hq = vals[j], errs[j], hqs[j]
        cand = []   # (row, column indices, their alternative dequantised values)
        for blk in blocks[j]:
            if blk.size == 0:
                continue
            v = y[:, blk]
            ev = e[:, blk]
            amax = np.max(np.abs(v), axis=1)
            ex = mx_exponent(amax)
            X = np.exp2(ex)[:, None]
            r = v / X
            # element roundings
            with np.errstate(invalid="ignore"):
                marg = np.where(r != 0, e4m3_rounding_margin(r) * np.abs(r), np.inf)
            close = marg < ev / X
            if pre[j] is not None:
                close |= (np.abs(pre[j][:, blk]) <= ev) & (v == 0)
            for row, col in zip(*np.nonzero(close)):
                if v[row, col] == 0:
                    alt = round_e4m3(ev[row, col] / X[row, 0]) * X[row, 0]
                else:
                    alt = _other_neighbour(r[row, col], marg[row, col], round_e4m3) * X[row, 0]
                cand.append((row, blk[col:col + 1], np.array([alt])))
            # shared exponent: it steps where amax crosses 448 2^e, i.e.
            # 1.75 times a power of two; amax within its bound of such a point
            k = np.floor(np.log2(np.where(amax > 0, amax, 1.0) / 1.75))
            emax = ev[np.arange(v.shape[0]), np.argmax(np.abs(v), axis=1)]
            lo, hi = amax - 1.75 * np.exp2(k), 1.75 * np.exp2(k + 1) - amax
            for row in np.nonzero((amax > 0) & (np.minimum(lo, hi) <= emax))[0]:
                ex2 = ex[row] + (-1.0 if lo[row] <= hi[row] else 1.0)
                X2 = np.exp2(ex2)
                cand.append((row, blk, round_e4m3(v[row] / X2) * X2))
        if not cand:
            continue
        rows = np.array([c[0] for c in cand])
        count += np.bincount(rows, minlength=n)
        # each decision alone (at most max_alternatives per ray and layer)
        seen = {}
        sel = []
        for i, c in enumerate(cand):
            seen[c[0]] = seen.get(c[0], 0) + 1
            if seen[c[0]] <= max_alternatives:
                sel.append(i)
        alts = hq[rows[sel]].copy()
        for a, i in enumerate(sel):
            alts[a, cand[i][1]] = cand[i][2]
        apply(j, rows[sel], alts)
        # all of a ray's decisions of this layer together; the layers'
        # effects add up (to first order) when several layers have one
        ur = np.unique(rows)
        pos = {r_: i for i, r_ in enumerate(ur)}
        alls = hq[ur].copy()
        for c in cand:
            alls[pos[c[0]], c[1]] = c[2]
        dmu, dp = _head_delta(run_from(j, alls), base[ur])
        np.maximum.at(amb, ur, dmu)
        np.maximum.at(amb_p, ur, dp)
        np.add.at(sum_mu, ur, dmu)
        np.add.at(sum_p, ur, dp)
    return np.maximum(amb, sum_mu), np.maximum(amb_p, sum_p), count
