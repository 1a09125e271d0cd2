"""Throughput benchmark of the NeDF composition hot path on one MI355X.

Default workload (``--workload frame``): the batched composition scene, 1,000
instances of 4 SDF-biased NeRF objects (gamma_10(x) -> 8 x 256 ReLU -> sigma,
colour branch (256 + 27) -> 128 -> 3) at 1920 x 1080, uneven screen coverage
(1-20 % per instance), two point lights.  Each object gets an intersection
network (gamma_8 of the Pluecker ray -> 8 x 256 ReLU -> (depth, hit logit))
trained before the timed region by the library's own kernels on labels from
its own FP32 marcher.  A step is one frame through the library: FP64
transform composition, in-kernel camera rays, culling/binning, the BF16
intersection network with marcher fallback for uncertain pairs, the per-pixel
min-reduce, 3-step secant refinement, K = 8 deferred shading, shadow rays to
both lights and the composite.  ``value`` is pixels per second of whole
frames.  Beside it: the depth+ID stage alone, the plain FP32 marcher on a
seeded pixel subset of the same scene (rays/s and the NeDF path's depth error
and hit agreement against it), the roofline of the dominant kernel from
library-side HIP events, and the FP64 oracle timed on a bounded pixel sample.

``--workload marcher``: the plain-marcher composition scene (16 random NeRF
objects, 800 x 800, 192 samples per pair), BF16 with an FP32 run beside it.

``--workload train``: the intersection network's Adam step alone (Eq. 6),
65,536 synthetic rays per step, the regression form (the frame's networks)
and the classifier form beside it, with the step's HBM roofline.

``--workload precision``: 64 instances at 3840 x 2160; the depth+ID path
with the intersection network in FP32, BF16 and FP8 (per-layer scales from
the library's calibration pass), each with 3-step refinement on the density
field (FP8 also without), timed, with depth error and hit agreement against
the FP32 marcher on a seeded pixel subset.

Inputs are seeded synthetic weights and placements (no trained models or
datasets).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/s depth+ID (NeDF vs plain marcher, ≤1% depth err); MFMA util"
PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3, "fp8": 5000.0}
# density trunk multiply-adds per sample: 63x256 + 7 x 256x256 + 256 (sigma head)
MAC_PER_SAMPLE = 63 * 256 + 7 * 256 * 256 + 256
# colour branch per sample: (256 + 27) x 128 + 128 x 3
MAC_RGB = (256 + 27) * 128 + 128 * 3
# intersection network per pair: 102 x 256 + 7 x 256x256 + 256 x 2
MAC_NEDF = 102 * 256 + 7 * 256 * 256 + 256 * 2
# classifier-form network per pair: head 1,008 -> 256, 16 residual blocks of
# two 256 x 256 layers, tail 256 -> 193
MAC_CLS = 1008 * 256 + 32 * 256 * 256 + 256 * 193


# HBM bytes per launch of a matrix-core kernel in the timed frames, from the
# hardware byte counters of a profiled run of this benchmark (FETCH_SIZE and
# WRITE_SIZE, each scaled by what it reads for a plain device copy of known
# size).  Each record keeps a hash of the kernels' sources; the figure is
# reported only while they are unchanged.
NET_SOURCES = ["include/nedf.h"] + ["paper_2308_04669_amd/csrc/" + f for f in (
    "k_depth.hip", "pipeline.h", "mlp_engine.h", "device_common.h", "launch.h", "runtime.h", "blob_layout.h")]
TRAFFIC_RECORDS = {
    "infer.nedf/net": os.path.join(ROOT, "profiles", "nedf_net_bf16_batched_1000inst_1920x1080.md"),
    "fallback.mlp": os.path.join(ROOT, "profiles", "fallback_march_bf16_batched_1000inst_1920x1080.md"),
    "train.step": os.path.join(ROOT, "profiles", "train_step_bf16_65536rays.md"),
}
TRAIN_SOURCES = ["include/nedf.h"] + ["paper_2308_04669_amd/csrc/" + f for f in ("k_train.hip", "train_layout.h")]


def sources_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(record: str, files):
    """(bytes per launch, note) from a counter record, or (None, reason)."""
    try:
        with open(record) as fh:
            kv = dict(re.findall(r"^- ([a-z_0-9]+): `([^`]*)`", fh.read(), re.M))
    except OSError:
        return None, "no counter record"
    if kv.get("sources_sha256") != sources_hash(files):
        return None, "kernel sources changed since the counters were taken"
    try:
        return float(kv["hbm_bytes_per_launch"]), os.path.relpath(record, ROOT)
    except (KeyError, ValueError):
        return None, "counter record without hbm_bytes_per_launch"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None, help="timed steps (default 5; 200 for --workload train)")
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="frame", choices=["frame", "marcher", "precision", "nedf", "ablation",
                                                            "train"])
    p.add_argument("--dtype", default="bf16", choices=["bf16", "f32"])
    # frame workload
    p.add_argument("--width", type=int, default=1920)
    p.add_argument("--height", type=int, default=1080)
    p.add_argument("--instances", type=int, default=1000)
    p.add_argument("--train-steps", type=int, default=None,
                   help="Adam steps per object (default 1500 for the frame, 20000 for --workload nedf)")
    p.add_argument("--train-batch", type=int, default=65536)
    p.add_argument("--label-batches", type=int, default=153, help="labels per object = batches x batch (10 M)")
    p.add_argument("--fallback-samples", type=int, default=128)
    p.add_argument("--marcher-pixels", type=int, default=2048)
    p.add_argument("--no-shading", action="store_true", help="depth+ID only in the timed frame")
    p.add_argument("--rs-sigma", type=float, default=0.5,
                   help="frame: outlier threshold of the rs / wo rs shading comparison (1 %% of sigma_max)")
    p.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing beside the eager frames")
    p.add_argument("--no-manip", action="store_true",
                   help="skip the buffer-reuse timing (one instance moved, the others' keys kept)")
    p.add_argument("--no-precision", action="store_true",
                   help="skip the per-dtype leg (FP32 / BF16 / FP8 networks at 3840x2160, 64 instances)")
    # marcher workload
    p.add_argument("--samples", type=int, default=192)
    p.add_argument("--size", type=int, default=800)
    p.add_argument("--f32-steps", type=int, default=2)
    # intersection-network workload
    p.add_argument("--labels", type=int, default=10_000_000)
    p.add_argument("--quality-pixels", type=int, default=4096)
    p.add_argument("--fp64-pixels", type=int, default=256,
                   help="frame: seeded pixels judged by the FP64 oracle marcher (inside the CPU-baseline leg)")
    # regression-vs-classifier workload
    p.add_argument("--ablation-steps", type=int, default=4000, help="Adam steps per network and object")
    p.add_argument("--ablation-size", type=int, default=384, help="side of each object's evaluation view")
    # oracle baseline and counters
    p.add_argument("--cpu-pixels", type=int, default=0, help="0: the workload's default sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--sources-hash", action="store_true",
                   help="print the hash of the network kernel's sources (kept with its counter record) and exit")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="after the timed region, copy a tensor of this size (device to device) so that "
                        "hardware byte counters can be scaled against a copy of known size")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return 1


def stage_table(stages):
    return {k: v[0] / max(v[1], 1) for k, v in stages.items()}


# ---------------------------------------------------------------------------
# frame workload
# ---------------------------------------------------------------------------

def train_nedfs(models, config, args):
    """Label generation (FP32 marcher on random local rays) and training of
    one intersection network per object, all through the library."""
    import torch
    import synthetic as syn
    from paper_2308_04669_amd import api

    ident = syn.Instance(model=0, R=np.eye(3), T=np.zeros(3), s=1.0)
    nets, info = [], []
    B, nb = args.train_batch, args.label_batches
    for k, m in enumerate(models):
        sc = api.make_scene([api.object_from_model(m, "f32")], [ident])
        o, d = syn.training_rays(config, 300 + k, nb * B)
        ot, dt = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        depth, idn, _ = api.march_depth(sc, api.array_rays(ot, dt), n_samples=128, dtype="f32", opacity=False,
                                        ws=api.Workspace())
        hit = (idn >= 0).to(torch.uint8)
        depth = torch.where(idn >= 0, depth, torch.zeros_like(depth))
        torch.cuda.synchronize()
        t_label = time.perf_counter() - t0
        init = syn.nedf_model(config, 200 + k)
        tr = api.Trainer(init.trunk.W, init.trunk.b, enc_L=init.params["enc_L"])
        first = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(args.train_steps):
            j = it % nb
            lr = 5e-5 + 0.5 * (5e-4 - 5e-5) * (1.0 + math.cos(math.pi * it / max(args.train_steps, 1)))
            loss = tr.step(ot[j * B:(j + 1) * B], dt[j * B:(j + 1) * B], depth[j * B:(j + 1) * B],
                           hit[j * B:(j + 1) * B], lr=lr, bound=m.bound)
            if it == 0:
                first = loss.clone()
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        W, b = tr.export(0)
        nets.append(syn.Model(kind="nedf", bound=m.bound, params=dict(enc_L=init.params["enc_L"]),
                              trunk=syn.MLPWeights([w.astype(np.float32) for w in W],
                                                   [x.astype(np.float32) for x in b])))
        info.append({"label_rays": nb * B, "label_s": t_label, "hit_frac": float(hit.float().mean()),
                     "steps": args.train_steps, "train_s": t_train,
                     "loss_first": float(first[0]), "loss_last": float(loss[0])})
        log(f"nedf {k}: labels {t_label:.2f} s, train {t_train:.2f} s, loss {info[-1]['loss_first']:.4f} -> "
            f"{info[-1]['loss_last']:.4f}")
    ms_step = 1e3 * sum(i["train_s"] for i in info) / max(sum(i["steps"] for i in info), 1)
    summary = {"ms_per_step": ms_step, "rays_per_s": args.train_batch / (ms_step * 1e-3),
               "batch": args.train_batch,
               "tflops": 3.0 * 2.0 * MAC_NEDF * args.train_batch / (ms_step * 1e-3) / 1e12,
               "per_object": info}
    return nets, summary


def frame_bench(args):
    import torch
    import synthetic as syn
    from paper_2308_04669_amd import api

    config = 4
    W, H = args.width, args.height
    models, insts, cam, lights = syn.batched_scene(config, args.instances, W, H)
    n = W * H
    t0 = time.perf_counter()
    nets, train = train_nedfs(models, config, args)
    setup_train_s = time.perf_counter() - t0
    objs = [api.object_from_model(m, args.dtype, nedf_model=nn, nedf_dtype=args.dtype) for m, nn in zip(models, nets)]
    sc = api.make_scene(objs, insts)
    rays = api.camera_rays(cam)
    extent = syn.scene_extent(insts, [m.bound for m in models])
    eps = 0.01 * extent
    ws = api.Workspace()
    dev = "cuda"
    depth = torch.empty(n, dtype=torch.float32, device=dev)
    ident = torch.empty(n, dtype=torch.int32, device=dev)
    rgb = torch.empty((n, 3), dtype=torch.float32, device=dev)
    fac = torch.empty(n, dtype=torch.float32, device=dev)

    def depth_id():
        sc.inst_w2l = api.compose_transforms(sc.inst_G)
        api.infer_depth_id(sc, rays, dtype=args.dtype, refine_steps=3, n_samples=args.fallback_samples, ws=ws,
                           out=(depth, ident))

    def frame():
        depth_id()
        if not args.no_shading:
            api.shade_deferred(sc, rays, depth, ident, K=8, h=0.05, dtype=args.dtype, ws=ws, out=rgb)
            api.shadow(sc, rays, depth, ident, lights, eps, beta=0.5, method="nedf", dtype=args.dtype,
                       n_samples=args.fallback_samples, rgb_inout=rgb, ws=ws, out=fac)

    # superchunk sizes of the matrix-core kernels from the library's autotuner:
    # the intersection network on this frame, the marcher on a pixel subset
    g = np.random.default_rng(4669 + 1000 * config + 78)
    tpix = np.sort(g.choice(n, size=min(4096, n), replace=False))
    to_, td_ = subset_rays(cam, tpix % W, tpix // W)
    trays = api.array_rays(torch.from_numpy(to_).cuda(), torch.from_numpy(td_).cuda())
    tune = {"nedf": api.autotune("nedf", args.dtype, sc, rays,
                                 api.infer_opts(args.dtype, refine_steps=3, n_samples=args.fallback_samples),
                                 reps=1, ws=ws),
            "march": api.autotune("march", args.dtype, sc, trays,
                                  api.march_opts(args.fallback_samples, dtype=args.dtype), reps=1)}
    tune["slabs"] = api.autotune("slabs", args.dtype, sc, rays,
                                 api.infer_opts(args.dtype, refine_steps=3, n_samples=args.fallback_samples),
                                 reps=1, ws=ws)
    log(f"autotune {tune}")
    for _ in range(args.warmup):
        frame()
    torch.cuda.synchronize()
    # routing counters of the primary pass (read before shading reuses the workspace)
    depth_id()
    torch.cuda.synchronize()
    st = api.ws_counters(ws)
    assert api.check_status(ws) == 0, "frame reported a device status error"
    api.profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        frame()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    stages = api.profile_read()
    api.profile_enable(False)
    assert api.check_status(ws) == 0, "frame reported a device status error"
    per = stage_table(stages)
    depth_ms = sum(v for k, v in per.items() if "/" not in k and k not in ("shade", "shadow"))

    # the same frame captured once in a HIP graph and replayed (launch-side
    # cost of the ~240 kernels per frame removed); reported beside `value`
    graph = None
    if not args.no_graph:
        gs = torch.cuda.Stream()
        gs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(gs):
            frame()
        gs.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=gs):
            frame()
        with torch.cuda.stream(gs):
            for _ in range(args.warmup):
                g.replay()
            gs.synchronize()
            g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            g0.record(gs)
            for _ in range(args.steps):
                g.replay()
            g1.record(gs)
        gs.synchronize()
        gms = g0.elapsed_time(g1) / args.steps
        graph = {"ms_per_step": gms, "rays_per_s": n / (gms * 1e-3), "replays": args.steps}
        assert api.check_status(ws) == 0, "graph replay reported a device status error"

    # outlier processing in deferred shading (the paper's "rs" / "wo rs"):
    # shading alone, timed with and without resampling of the pixels whose
    # density stays below rs_sigma at all K samples
    rs = None
    if not args.no_shading:
        depth_id()
        torch.cuda.synchronize()
        rgb_rs = torch.empty_like(rgb)
        ws_rs = api.Workspace()
        times = {}
        for name, thr in (("wo_rs", 0.0), ("rs", args.rs_sigma)):
            out = rgb if thr == 0.0 else rgb_rs
            api.shade_deferred(sc, rays, depth, ident, K=8, h=0.05, dtype=args.dtype, ws=ws_rs, out=out,
                               rs_sigma=thr, rs_samples=32)
            torch.cuda.synchronize()
            r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            r0.record()
            for _ in range(args.steps):
                api.shade_deferred(sc, rays, depth, ident, K=8, h=0.05, dtype=args.dtype, ws=ws_rs, out=out,
                                   rs_sigma=thr, rs_samples=32)
            r1.record()
            torch.cuda.synchronize()
            times[name] = r0.elapsed_time(r1) / args.steps
        n_rs = api.ws_counters(ws_rs)["fallback"]
        hits = int((ident >= 0).sum())
        diff = (rgb_rs - rgb).abs().max(dim=1).values
        rs = {"rs_sigma": args.rs_sigma, "rs_samples": 32, "shade_ms_wo_rs": times["wo_rs"],
              "shade_ms_rs": times["rs"], "resampled_pixels": int(n_rs),
              "resampled_frac_of_hits": n_rs / max(hits, 1),
              "mean_abs_rgb_change_resampled": float(diff[diff > 0].mean()) if bool((diff > 0).any()) else 0.0}
        log(f"outlier resampling {rs}")

    # buffer reuse while one object is manipulated: the keys of the other
    # instances are computed once and kept; a manipulation frame recomputes
    # the moving instance's keys, min-merges and refines, against the full
    # depth+ID pass on the same moved scene (results must be bit-identical)
    manip = None
    if not args.no_manip:
        depth_id()
        torch.cuda.synchronize()
        cnt = torch.bincount(ident[ident >= 0].long(), minlength=len(insts))
        mover = int(cnt.argmax())
        static_idx = [k for k in range(len(insts)) if k != mover]
        G = sc.inst_G.clone()
        G[mover, 9] += 0.03 * extent
        G[mover, 10] -= 0.02 * extent
        sc_m = api.SceneGPU(sc.objects, sc.inst_object, G, api.compose_transforms(G))
        sub_s, gid_s = api.subset_scene(sc_m, static_idx)
        sub_m, gid_m = api.subset_scene(sc_m, [mover])
        ws_s, ws_m, ws_c, ws_f = (api.Workspace() for _ in range(4))
        keys_s = torch.empty(n, dtype=torch.int64, device=dev)
        keys_m = torch.empty(n, dtype=torch.int64, device=dev)
        d_m = torch.empty(n, dtype=torch.float32, device=dev)
        i_m = torch.empty(n, dtype=torch.int32, device=dev)
        d_f = torch.empty(n, dtype=torch.float32, device=dev)
        i_f = torch.empty(n, dtype=torch.int32, device=dev)
        kw = dict(dtype=args.dtype, n_samples=args.fallback_samples)

        # pair lists sized from this frame's culled pairs, not rays x instances
        cap = int(st["culled_pairs"] * 1.25) + (1 << 20)

        def static_pass():
            api.infer_keys(sub_s, rays, gid_s, ws=ws_s, out=keys_s, pair_capacity=cap, **kw)

        def manip_frame():
            sc_m.inst_w2l = api.compose_transforms(sc_m.inst_G)
            sub_m.inst_w2l = sc_m.inst_w2l[mover:mover + 1]
            api.infer_keys(sub_m, rays, gid_m, ws=ws_m, out=keys_m, **kw)
            api.compose_keys(sc_m, rays, [keys_s, keys_m], refine_steps=3, ws=ws_c, out=(d_m, i_m), **kw)

        def full_frame():
            sc_m.inst_w2l = api.compose_transforms(sc_m.inst_G)
            api.infer_depth_id(sc_m, rays, refine_steps=3, ws=ws_f, out=(d_f, i_f), pair_capacity=cap, **kw)

        res = {}
        for name, fn in (("static_keys_once", static_pass), ("manipulation_frame", manip_frame),
                         ("full_depth_id", full_frame)):
            fn()
            torch.cuda.synchronize()
            m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            m0.record()
            for _ in range(args.steps):
                fn()
            m1.record()
            torch.cuda.synchronize()
            res[name] = m0.elapsed_time(m1) / args.steps
        for w_ in (ws_s, ws_m, ws_c, ws_f):
            assert api.check_status(w_) == 0, "buffer-reuse leg reported a device status error"
        same = bool(torch.equal(i_m, i_f) and torch.equal(d_m.view(torch.int32), d_f.view(torch.int32)))
        manip = {"moved_instance": mover, "moved_instance_pixels": int(cnt[mover]),
                 "ms_static_keys_once": res["static_keys_once"], "ms_manipulation_frame": res["manipulation_frame"],
                 "ms_full_depth_id": res["full_depth_id"],
                 "speedup": res["full_depth_id"] / max(res["manipulation_frame"], 1e-9),
                 "bit_identical_to_full": same}
        log(f"buffer reuse {manip}")
        assert same, "buffer-reuse depth/ID differ from the full pass"
        del ws_s, ws_m, ws_c, ws_f, keys_s, keys_m
        torch.cuda.empty_cache()

    # precision leg: the same four objects and trained networks, 64 instances
    # at 3840 x 2160 (the precision-stress placement), depth+ID per network
    # dtype (FP32, BF16, FP8 with and without refinement)
    precision = None
    if not args.no_precision:
        _, insts5, cam5, _ = syn.batched_scene(5, 64, 3840, 2160)
        runs5, extent5, npix5 = precision_runs(models, nets, insts5, cam5, 5, args)
        precision = {"workload": "64 instances of the frame's 4 objects, 3840x2160 (placement of the precision "
                                 "stress scene), depth+ID", "extent": extent5, "judge_pixels": npix5,
                     "per_dtype": runs5}

    # plain FP32 marcher on a seeded pixel subset of the same scene
    g = np.random.default_rng(4669 + 1000 * config + 77)
    pix = np.sort(g.choice(n, size=min(args.marcher_pixels, n), replace=False))
    px, py = pix % W, pix // W
    o_s, d_s = subset_rays(cam, px, py)
    ot, dt = torch.from_numpy(o_s).cuda(), torch.from_numpy(d_s).cuda()
    sub = api.array_rays(ot, dt)
    wsm = api.Workspace()
    sc32 = api.make_scene([api.object_from_model(m, "f32") for m in models], insts)
    api.march_depth(sc32, sub, n_samples=192, dtype="f32", opacity=False, ws=wsm)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dm, im, _ = api.march_depth(sc32, sub, n_samples=192, dtype="f32", opacity=False, ws=wsm)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    marcher_rps = len(pix) / t_m
    pix_t = torch.from_numpy(pix).cuda()
    dn, idn_ = depth[pix_t].cpu().numpy().astype(np.float64), ident[pix_t].cpu().numpy()
    dm, im = dm.cpu().numpy().astype(np.float64), im.cpu().numpy()
    agree = float(np.mean((dn < np.inf) == (im >= 0)))
    both = (idn_ == im) & (im >= 0)
    med = float(np.median(np.abs(dn[both] - dm[both]))) if both.any() else float("inf")
    quality = {"pixels": int(len(pix)), "hit_agreement": agree, "id_agreement": float(np.mean(idn_ == im)),
               "median_depth_err": med, "median_depth_err_frac_extent": med / extent, "extent": extent,
               "depth_err_over": "pixels with the same ID",
               "reference": "library FP32 marcher, 192 samples per pair"}

    # dominant kernel of the timed frames, per launch: the network runs once
    # per depth slab, so a launch's algorithmic work is the frame's evaluated
    # pairs over the launches per frame
    ev = st["nedf_hits"] + st["fallback"] + st["nedf_misses"]
    net_ms, net_n = stages.get("infer.nedf/net", (0.0, 1))
    launches = max(net_n // max(args.steps, 1), 1)
    cand = {
        "infer.nedf/net": (net_ms / max(net_n, 1), 2.0 * MAC_NEDF * ev / launches, args.dtype),
        "fallback.mlp": (per.get("fallback.mlp", 0.0), 2.0 * MAC_PER_SAMPLE * args.fallback_samples *
                         st.get("fallback_marched", st["fallback"]), args.dtype),
    }
    kname = max(cand, key=lambda k: cand[k][0] * (launches if k == "infer.nedf/net" else 1))
    k_ms, k_flops, k_dt = cand[kname]
    achieved = k_flops / (k_ms * 1e-3) / 1e12 if k_ms > 0 else 0.0
    peak = PEAK_TFLOPS[k_dt]
    traffic, traffic_src = recorded_traffic(TRAFFIC_RECORDS[kname], NET_SOURCES)
    line = {
        "metric": METRIC,
        "value": n / (ms * 1e-3),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded SDF-biased NeRF objects and placements; intersection networks trained in setup "
                "on the library's own FP32 marcher labels)",
        "config": {"workload": f"batched composition: {args.instances} instances of 4 SDF-biased NeRF objects "
                               f"(gamma10 xyz, 8x256 ReLU, sigma + colour), {W}x{H}, BF16 NeDF + fallback "
                               f"({args.fallback_samples} samples) + 3-step refine, "
                               + ("depth+ID only" if args.no_shading else
                                  "K=8 deferred shading, 2 point lights with shadow rays"),
                   "pairs_per_frame": int(st["culled_pairs"]), "network_pairs_evaluated": int(ev),
                   "nedf_hits": int(st["nedf_hits"]), "fallback_pairs_marched": int(st["fallback_marched"]),
                   "fallback_pairs": int(st["fallback"]), "fallback_frac": st["fallback"] / max(ev, 1)},
        "depth_id": {"rays_per_s": n / (depth_ms * 1e-3) if depth_ms > 0 else None, "ms": depth_ms,
                     "vs_fp32_marcher": (n / (depth_ms * 1e-3)) / marcher_rps if depth_ms > 0 else None},
        "fp32_marcher": {"rays_per_s": marcher_rps, "pixels": int(len(pix)), "samples_per_pair": 192},
        "quality": quality,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic, "traffic_unit": "bytes per launch",
                     "traffic_source": traffic_src, "kernel": kname, "avg_launch_ms": k_ms,
                     "flop_per_launch": k_flops, "launches_per_frame": launches if kname.endswith("net") else 1},
        "stages_ms_per_step": per,
        "autotune": tune,
        "graph": graph,
        "outlier_resampling": rs,
        "buffer_reuse": manip,
        "precision": precision,
        "training": train,
        "setup_train_s": setup_train_s,
    }
    depth_np, ident_np = depth.cpu().numpy(), ident.cpu().numpy()
    return line, (models, nets, insts, cam, config, depth_np, ident_np, extent)


def subset_rays(cam, px, py):
    """Pinhole rays through pixel centres (px, py) in float32 (the same
    convention as the library's in-kernel camera rays)."""
    eye = np.asarray(cam.eye, np.float64)
    fwd = np.asarray(cam.at, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(cam.up, np.float64))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(0.5 * cam.fov_y_deg))
    aspect = cam.width / cam.height
    u = (2.0 * (px + 0.5) / cam.width - 1.0) * th * aspect
    v = (1.0 - 2.0 * (py + 0.5) / cam.height) * th
    d = fwd[None] + u[:, None] * right[None] + v[:, None] * up[None]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape)
    return np.ascontiguousarray(o, np.float32), np.ascontiguousarray(d, np.float32)


def frame_cpu_baseline(ctx, n_pixels, quality_pixels):
    """FP64 oracle of the depth+ID path (intersection network, marcher
    fallback) timed on a seeded pixel sample of the same frame; and, on a
    second seeded sample, the FP64 oracle marcher (192 samples per pair,
    front to back with exact pruning) as the judge of the frame's depth and
    ID buffers, with every ID disagreement classified."""
    import synthetic as syn
    from oracle import camera_rays, f32_record, nedf_compose, nedf_pair, march_compose_pruned
    from oracle.render import march_instance
    models, nets, insts, cam, config, depth_g, ident_g, extent = ctx
    pix = syn.pixel_subset(config, cam.n_rays, n_pixels)
    o, d = camera_rays(cam, pix)
    t0 = time.perf_counter()
    nedf_compose(nets, models, insts, o, d, n_samples=128)
    dt = time.perf_counter() - t0
    base = {"value": n_pixels / dt, "unit": "rays/s", "cores": int(host_threads()), "kind": "oracle",
            "sample": f"{n_pixels} seeded pixels of the same {cam.width}x{cam.height} frame, depth+ID "
                      f"(intersection network, marcher fallback), FP64 NumPy, {dt:.1f} s"}
    # the same oracle on one host thread (BLAS limited to one thread), on the
    # first tenth of the sample
    try:
        from threadpoolctl import threadpool_limits
        n1 = max(n_pixels // 10, 1)
        o1, d1 = camera_rays(cam, pix[:n1])
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            nedf_compose(nets, models, insts, o1, d1, n_samples=128)
            dt1 = time.perf_counter() - t0
        base["value_1core"] = n1 / dt1
        base["sample_1core"] = f"first {n1} pixels of the sample, one thread, {dt1:.1f} s"
    except ImportError:
        pass
    # the FP64 oracle marcher as the judge (rays of the single-precision camera)
    qp = syn.pixel_subset(config, cam.n_rays, quality_pixels, stream=13)
    oq, dq = camera_rays(cam, qp, basis="f32")
    recs = [f32_record(i) for i in insts]
    t0 = time.perf_counter()
    ref_d, ref_id, n_pairs = march_compose_pruned(models, recs, oq, dq, 192)
    t_ref = time.perf_counter() - t0
    g_d, g_id = depth_g[qp].astype(np.float64), ident_g[qp].astype(np.int64)
    same = (g_id == ref_id) & (ref_id >= 0)
    err = np.abs(g_d[same] - ref_d[same])
    tol = 0.01 * extent
    mism = np.nonzero((g_id != ref_id) & (g_id >= 0) & (ref_id >= 0))[0]
    near_tie, routes = 0, {"network_miss": 0, "fallback_band": 0, "network_hit_deeper": 0, "inside": 0}
    for i in mism:
        # the oracle marcher's depth of the instance the frame chose: a near-tie
        # when it lies within 1 % of the extent of the winner's
        kg = int(g_id[i])
        v, A, D = march_instance(models[recs[kg].model], recs[kg], oq[i:i + 1], dq[i:i + 1], 192)
        if v[0] and A[0] >= 0.5 and abs(D[0] - ref_d[i]) <= tol:
            near_tie += 1
            continue
        # how the intersection network (bfloat16 emulation) routed the marcher's winner
        kr = int(ref_id[i])
        hit, Dn, pr, path = nedf_pair(nets[recs[kr].model], models[recs[kr].model], recs[kr], oq[i:i + 1],
                                      dq[i:i + 1], n_samples=128, gemm="bf16")
        if path[0] == 1 and not np.isfinite(pr[0]):
            routes["inside"] += 1
        elif path[0] == 1:
            routes["fallback_band"] += 1
        elif not hit[0]:
            routes["network_miss"] += 1
        else:
            routes["network_hit_deeper"] += 1
    base["quality_fp64"] = {
        "pixels": int(len(qp)), "reference": "FP64 oracle marcher, 192 samples per pair, exact pruning",
        "oracle_s": t_ref, "pairs_marched": int(n_pairs),
        "hit_agreement": float(np.mean((g_id >= 0) == (ref_id >= 0))),
        "id_agreement": float(np.mean(g_id == ref_id)),
        "median_depth_err_frac_extent": float(np.median(err)) / extent if err.size else None,
        "p90_depth_err_frac_extent": float(np.quantile(err, 0.9)) / extent if err.size else None,
        "depth_err_over": "pixels with the same ID",
        "id_mismatch": {"total": int(len(mism)), "near_tie_within_1pct_extent": near_tie,
                        "other_by_network_route_of_the_marcher_winner": routes},
    }
    return base


# ---------------------------------------------------------------------------
# precision workload
# ---------------------------------------------------------------------------

def precision_runs(models, nets, insts, cam, config, args):
    """Depth+ID of one scene with the intersection networks in FP32, BF16,
    FP8 (+ refinement) and FP8: rays/s, the network stage's per-frame time
    and matrix-core rate against its dtype's dense peak, and depth/ID quality
    against the FP32 marcher on seeded pixels."""
    import torch
    import synthetic as syn
    from paper_2308_04669_amd import api

    W, H = cam.width, cam.height
    n = W * H
    scales = []
    for k, net in enumerate(nets):
        o, d = syn.training_rays(config, 500 + k, 65536)
        scales.append(api.fp8_calibrate(net.trunk.W, net.trunk.b, torch.from_numpy(o).cuda(),
                                        torch.from_numpy(d).cuda()))
    extent = syn.scene_extent(insts, [m.bound for m in models])
    rays = api.camera_rays(cam)
    # judge: the FP32 marcher on a seeded pixel subset
    g = np.random.default_rng(4669 + 1000 * config + 77)
    pix = np.sort(g.choice(n, size=min(args.marcher_pixels, n), replace=False))
    o_s, d_s = subset_rays(cam, pix % W, pix // W)
    sc32 = api.make_scene([api.object_from_model(m, "f32") for m in models], insts)
    dm, im, _ = api.march_depth(sc32, api.array_rays(torch.from_numpy(o_s).cuda(), torch.from_numpy(d_s).cuda()),
                                n_samples=192, dtype="f32", opacity=False, ws=api.Workspace())
    dm, im = dm.cpu().numpy().astype(np.float64), im.cpu().numpy()
    pix_t = torch.from_numpy(pix).cuda()
    runs = {}
    ws = api.Workspace()
    peak = {"f32": PEAK_TFLOPS["f32"], "bf16": PEAK_TFLOPS["bf16"], "fp8": PEAK_TFLOPS["fp8"],
            "fp8mx": PEAK_TFLOPS["fp8"]}
    for name, dens_dt, nedf_dt, refine in (("f32", "f32", "f32", 3), ("bf16", "bf16", "bf16", 3),
                                           ("fp8+refine", "bf16", "fp8", 3), ("fp8", "bf16", "fp8", 0),
                                           ("fp8mx+refine", "bf16", "fp8mx", 3), ("fp8mx", "bf16", "fp8mx", 0)):
        objs = [api.object_from_model(m, dens_dt, nedf_model=nn, nedf_dtype=nedf_dt,
                                      nedf_scales=sc.reshape(-1) if nedf_dt == "fp8" else None)
                for m, nn, sc in zip(models, nets, scales)]
        scn = api.make_scene(objs, insts)
        depth = torch.empty(n, dtype=torch.float32, device="cuda")
        ident = torch.empty(n, dtype=torch.int32, device="cuda")
        io = api.infer_opts(dens_dt, refine_steps=refine, n_samples=args.fallback_samples)
        if nedf_dt != "fp8mx":  # MX runs its one launch shape and the FP8 slab count
            api.autotune("nedf", nedf_dt, scn, rays, io, reps=1, ws=ws)
            api.autotune("slabs", nedf_dt, scn, rays, io, reps=1, ws=ws)

        def step():
            scn.inst_w2l = api.compose_transforms(scn.inst_G)
            api.infer_depth_id(scn, rays, dtype=dens_dt, refine_steps=refine, n_samples=args.fallback_samples,
                               ws=ws, out=(depth, ident))

        step()
        torch.cuda.synchronize()
        st = api.ws_counters(ws)
        api.profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        stages = api.profile_read()
        api.profile_enable(False)
        assert api.check_status(ws) == 0
        ms = e0.elapsed_time(e1) / args.steps
        ev = st["nedf_hits"] + st["fallback"] + st["nedf_misses"]
        net_ms, net_n = stages.get("infer.nedf/net", (0.0, 1))
        net_ms /= args.steps
        tflops = 2.0 * MAC_NEDF * ev / (net_ms * 1e-3) / 1e12 if net_ms > 0 else 0.0
        dn, idn = depth[pix_t].cpu().numpy().astype(np.float64), ident[pix_t].cpu().numpy()
        both = (idn >= 0) & (im >= 0)
        err = np.abs(dn[both] - dm[both])
        runs[name] = {"rays_per_s": n / (ms * 1e-3), "ms": ms,
                      "network_ms_per_frame": net_ms, "network_launches_per_frame": net_n // max(args.steps, 1),
                      "network_pairs": int(ev), "network_tflops": tflops,
                      "network_frac_of_peak": tflops / peak[nedf_dt], "network_peak_tflops": peak[nedf_dt],
                      "hit_agreement": float(np.mean((idn >= 0) == (im >= 0))),
                      "id_agreement": float(np.mean(idn == im)),
                      "median_depth_err_frac_extent": float(np.median(err)) / extent if err.size else None,
                      "p90_depth_err_frac_extent": float(np.quantile(err, 0.9)) / extent if err.size else None,
                      "fallback_frac": st["fallback"] / max(ev, 1)}
        log(f"precision {name}: {runs[name]}")
    return runs, extent, len(pix)


def precision_bench(args):
    import synthetic as syn

    config = 5
    W, H = (args.width, args.height) if args.width != 1920 else (3840, 2160)
    n_inst = args.instances if args.instances != 1000 else 64
    models, insts, cam, _ = syn.batched_scene(config, n_inst, W, H)
    nets, train = train_nedfs(models, config, args)
    runs, extent, n_pix = precision_runs(models, nets, insts, cam, config, args)
    fp8 = runs["fp8+refine"]
    line = {
        "metric": METRIC,
        "value": fp8["rays_per_s"],
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": fp8["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp8",
        "data": "synthetic (seeded SDF-biased NeRF objects; intersection networks trained in setup)",
        "config": {"workload": f"precision stress: {n_inst} instances of 4 SDF-biased NeRF objects, {W}x{H}, "
                               f"depth+ID per intersection-network dtype",
                   "extent": extent, "judge": f"library FP32 marcher, 192 samples, {n_pix} seeded pixels"},
        "roofline": {"bound": "mfma", "achieved": fp8["network_tflops"], "peak": PEAK_TFLOPS["fp8"],
                     "unit": "TFLOP/s", "frac": fp8["network_frac_of_peak"], "traffic": None,
                     "kernel": "infer.nedf/net (FP8)"},
        "per_dtype": runs,
        "training": train,
    }
    return line


# ---------------------------------------------------------------------------
# plain-marcher workload
# ---------------------------------------------------------------------------

def marcher_bench(args):
    import torch
    import synthetic as syn
    from paper_2308_04669_amd import api

    models, insts, cam, _ = syn.config2_scene(width=args.size, height=args.size)
    rays = api.camera_rays(cam)
    n = cam.n_rays

    def run(dtype, steps, warmup):
        sc = api.make_scene([api.object_from_model(m, dtype) for m in models], insts)
        ws = api.Workspace()
        out = (torch.empty(n, dtype=torch.float32, device="cuda"), torch.empty(n, dtype=torch.int32, device="cuda"),
               None)

        def step():
            sc.inst_w2l = api.compose_transforms(sc.inst_G)
            api.march_depth(sc, rays, n_samples=args.samples, dtype=dtype, opacity=False, ws=ws, out=out)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        api.profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        stages = api.profile_read()
        api.profile_enable(False)
        pairs = api.ws_counters(ws)["pairs"]
        assert api.check_status(ws) == 0
        return ms, stages, pairs

    # launch shape of the marcher from the library's autotuner, on this frame
    tsc = api.make_scene([api.object_from_model(m, args.dtype) for m in models], insts)
    tune = api.autotune("march", args.dtype, tsc, rays, api.march_opts(args.samples, dtype=args.dtype), reps=1)
    log(f"autotune {tune}")
    ms, stages, pairs = run(args.dtype, args.steps, args.warmup)
    mlp_ms, mlp_cnt = stages.get("march.mlp", (0.0, 1))
    avg_mlp = mlp_ms / max(mlp_cnt, 1)
    flops = 2.0 * MAC_PER_SAMPLE * args.samples * pairs
    achieved = flops / (avg_mlp * 1e-3) / 1e12 if avg_mlp > 0 else 0.0
    peak = PEAK_TFLOPS[args.dtype]
    line = {
        "metric": METRIC,
        "value": n / (ms * 1e-3),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded random-init NeRF-shaped MLPs and placements)",
        "config": {"workload": f"plain-marcher composition: 16 NeRF objects (gamma10 xyz, 8x256 ReLU, sigma head), "
                               f"{args.size}x{args.size} rays, {args.samples} samples per pair, depth+ID",
                   "pairs_per_frame": pairs, "samples_per_pair": args.samples, "path": "plain marcher"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "march.mlp", "avg_launch_ms": avg_mlp,
                     "flop_per_launch": flops},
        "stages_ms_per_step": stage_table(stages),
        "autotune": tune,
    }
    if args.dtype != "f32" and args.f32_steps > 0:
        ms32, st32, _ = run("f32", args.f32_steps, 1)
        m32, c32 = st32.get("march.mlp", (0.0, 1))
        a32 = flops / (m32 / max(c32, 1) * 1e-3) / 1e12 if m32 > 0 else 0.0
        line["f32_marcher"] = {"rays_per_s": n / (ms32 * 1e-3), "ms_per_step": ms32,
                               "mlp_tflops": a32, "mlp_frac_of_f32_peak": a32 / PEAK_TFLOPS["f32"]}
    return line


# ---------------------------------------------------------------------------
# intersection-network workload (one object at a time)
# ---------------------------------------------------------------------------

def nedf_bench(args):
    """Density A (analytic sphere) and B' (density B masked to |x| <= 1), one
    at a time: 10 M labels per object from the library's FP32 marcher (128
    samples on the bounding chord; origins on the sphere of radius 4 aimed
    into the ball of radius 1.2), training of the intersection network
    (batch 65,536, bfloat16 matrix cores, float32 master weights, Adam with a
    cosine learning rate), then the 800 x 800 view of the config-1 camera:
    BF16 network + marcher fallback for p in [0.2, 0.8] + 3-step refinement
    (A; B' has no surface to refine) against the plain FP32 marcher on the
    same view, and the depth quality against the FP64 oracle marcher on a
    seeded pixel subset (hit agreement, median depth error / scene extent)."""
    import torch
    import synthetic as syn
    from oracle import camera_rays, march_compose
    from paper_2308_04669_amd import api

    a, b = syn.config1_models()
    bp = syn.Model(kind=b.kind, bound=1.0, trunk=b.trunk, params=dict(b.params, masked=True))
    ident = syn.Instance(model=0, R=np.eye(3), T=np.zeros(3), s=1.0)
    cam = syn.config1_camera(args.size, args.size)
    n = cam.n_rays
    extent = syn.scene_extent([ident], [1.0])
    B = args.train_batch
    per, tot_px, tot_s, tot_m = {}, 0, 0.0, 0.0
    train_ms, train_steps = 0.0, 0
    for k, (name, m) in enumerate((("A", a), ("B'", bp))):
        sc_l = api.make_scene([api.object_from_model(m, "f32")], [ident])
        n_lab = args.labels // B * B
        o, d = syn.training_rays(3, 300 + k, n_lab)
        ot, dt = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
        del o, d
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        depth, idn, _ = api.march_depth(sc_l, api.array_rays(ot, dt), n_samples=128, dtype="f32", opacity=False,
                                        ws=api.Workspace())
        hit = (idn >= 0).to(torch.uint8)
        depth = torch.where(idn >= 0, depth, torch.zeros_like(depth))
        torch.cuda.synchronize()
        t_label = time.perf_counter() - t0
        init = syn.nedf_model(3, 200 + k)
        tr = api.Trainer(init.trunk.W, init.trunk.b, enc_L=init.params["enc_L"])
        nb = n_lab // B
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for it in range(args.train_steps):
            j = it % nb
            lr = 5e-5 + 0.5 * (5e-4 - 5e-5) * (1.0 + math.cos(math.pi * it / max(args.train_steps, 1)))
            loss = tr.step(ot[j * B:(j + 1) * B], dt[j * B:(j + 1) * B], depth[j * B:(j + 1) * B],
                           hit[j * B:(j + 1) * B], lr=lr, bound=m.bound)
        e1.record()
        torch.cuda.synchronize()
        ms_train = e0.elapsed_time(e1)
        train_ms += ms_train
        train_steps += args.train_steps
        W_, b_ = tr.export(0)
        net = syn.Model(kind="nedf", bound=1.0, params=dict(enc_L=init.params["enc_L"]),
                        trunk=syn.MLPWeights([w.astype(np.float32) for w in W_], [x.astype(np.float32) for x in b_]))
        del ot, dt, depth, idn, hit
        # the view: intersection network path and the plain FP32 marcher
        sc = api.make_scene([api.object_from_model(m, "bf16", nedf_model=net)], [ident])
        sc32 = api.make_scene([api.object_from_model(m, "f32")], [ident])
        rays = api.camera_rays(cam)
        ws = api.Workspace()
        dep = torch.empty(n, dtype=torch.float32, device="cuda")
        idt = torch.empty(n, dtype=torch.int32, device="cuda")
        for _ in range(args.warmup):
            api.infer_depth_id(sc, rays, dtype="bf16", refine_steps=3, ws=ws, out=(dep, idt))
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            api.infer_depth_id(sc, rays, dtype="bf16", refine_steps=3, ws=ws, out=(dep, idt))
        e1.record()
        torch.cuda.synchronize()
        ms_nedf = e0.elapsed_time(e1) / args.steps
        st = api.ws_counters(ws)
        ws32 = api.Workspace()
        api.march_depth(sc32, rays, n_samples=128, dtype="f32", ws=ws32)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.f32_steps):
            api.march_depth(sc32, rays, n_samples=128, dtype="f32", ws=ws32)
        e1.record()
        torch.cuda.synchronize()
        ms_march = e0.elapsed_time(e1) / args.f32_steps
        # quality against the FP64 oracle marcher
        pix = syn.pixel_subset(3, n, args.quality_pixels, stream=11 + k)
        o_q, d_q = camera_rays(cam, pix)
        ref_d, ref_id, _ = march_compose([m], [ident], o_q, d_q, 128)
        g_d = dep.cpu().numpy()[pix].astype(np.float64)
        g_id = idt.cpu().numpy()[pix]
        both = (g_id >= 0) & (ref_id >= 0)
        err = np.abs(g_d[both] - ref_d[both])
        evald = max(st["nedf_hits"] + st["fallback"] + st["nedf_misses"], 1)
        per[name] = {
            "label_rays": n_lab, "label_s": t_label, "train_steps": args.train_steps,
            "train_ms_per_step": ms_train / args.train_steps, "loss_last": float(loss[0]),
            "nedf_ms": ms_nedf, "nedf_rays_per_s": n / (ms_nedf * 1e-3),
            "fp32_marcher_ms": ms_march, "fp32_marcher_rays_per_s": n / (ms_march * 1e-3),
            "vs_fp32_marcher": ms_march / ms_nedf,
            "fallback_frac": st["fallback"] / evald,
            "quality": {"pixels": int(len(pix)), "reference": "FP64 oracle marcher, 128 samples on the chord",
                        "hit_agreement": float(np.mean((g_id >= 0) == (ref_id >= 0))),
                        "median_depth_err_frac_extent": float(np.median(err)) / extent if err.size else 0.0,
                        "p99_depth_err_frac_extent": float(np.quantile(err, 0.99)) / extent if err.size else 0.0,
                        "extent": extent}}
        log(f"nedf {name}: {per[name]}")
        tot_px += n
        tot_s += ms_nedf * 1e-3
        tot_m += ms_march * 1e-3
    ms_step = train_ms / max(train_steps, 1)
    flop_step = 3.0 * 2.0 * MAC_NEDF * B
    return {
        "metric": METRIC, "value": tot_px / tot_s, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * tot_s / 2, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (config-1 densities; intersection networks trained in setup on the library's own "
                "FP32 marcher labels)",
        "config": {"workload": f"intersection networks of density A and B' (masked), one object each, "
                               f"{args.size}x{args.size} config-1 view, BF16 network + fallback [0.2, 0.8] + "
                               f"3-step refinement; {args.labels} labels per object, {args.train_steps} Adam "
                               f"steps of {B}"},
        "vs_fp32_marcher": tot_m / tot_s,
        "training": {"ms_per_step": ms_step, "batch": B, "tflops": flop_step / (ms_step * 1e-3) / 1e12,
                     "roofline_frac": flop_step / (ms_step * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"]},
        "objects": per,
    }


# --------------------------------------------------------------------------
# regression vs multi-level classifier (the paper's Fig. 3 ablation)
# --------------------------------------------------------------------------
def ablation_bench(args):
    """Both intersection-network forms trained through the library on the
    same marcher labels of each config-4 object, then judged against the
    FP32 marcher on a held-out view of the object: depth error over pixels
    where both hit, split into pixels at a depth discontinuity (a 4-neighbour
    misses, or its depth differs by more than 5 % of the bounding radius) and
    the others, and the share of pixels off by more than 10 % of the radius
    (floaters).  The networks decide every pair themselves (p_lo = p_hi =
    0.5, no refinement).  Then the classifier networks replace the regression
    ones in the 1920 x 1080, 1,000-instance frame, whose depth+ID pass is
    timed with each form."""
    import torch
    import synthetic as syn
    from paper_2308_04669_amd import api

    config = 4
    models, insts, cam, _ = syn.batched_scene(config, args.instances, args.width, args.height)
    ident = syn.Instance(model=0, R=np.eye(3), T=np.zeros(3), s=1.0)
    B, nb, T = args.train_batch, args.label_batches, args.ablation_steps
    out = {"objects": []}
    reg_nets, cls_nets = [], []
    times = {"regression": 0.0, "classifier": 0.0}
    for k, m in enumerate(models):
        sc = api.make_scene([api.object_from_model(m, "f32")], [ident])
        o, d = syn.training_rays(config, 300 + k, nb * B)
        ot, dt = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
        depth, idn, _ = api.march_depth(sc, api.array_rays(ot, dt), n_samples=128, dtype="f32", opacity=False,
                                        ws=api.Workspace())
        hit = (idn >= 0).to(torch.uint8)
        depth = torch.where(idn >= 0, depth, torch.zeros_like(depth))
        forms = {"regression": (syn.nedf_model(config, 200 + k), "pluecker", 8),
                 "classifier": (syn.classifier_model(config, 500 + k), "points16", 10)}
        res = {}
        for name, (init, kind, L) in forms.items():
            tr = api.Trainer(init.trunk.W, init.trunk.b, enc_L=L, in_kind=kind)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for it in range(T):
                j = it % nb
                lr = 5e-5 + 0.5 * (5e-4 - 5e-5) * (1.0 + math.cos(math.pi * it / max(T, 1)))
                loss = tr.step(ot[j * B:(j + 1) * B], dt[j * B:(j + 1) * B], depth[j * B:(j + 1) * B],
                               hit[j * B:(j + 1) * B], lr=lr, bound=m.bound)
            torch.cuda.synchronize()
            dt_s = time.perf_counter() - t0
            times[name] += dt_s
            W, bb = tr.export(0)
            net = syn.Model(kind=init.kind, bound=m.bound, params=dict(init.params),
                            trunk=syn.MLPWeights([w.astype(np.float32) for w in W], [x.astype(np.float32) for x in bb]))
            (reg_nets if name == "regression" else cls_nets).append(net)
            res[name] = {"train_s": dt_s, "loss_last": float(loss[0])}
            log(f"object {k} {name}: {T} steps in {dt_s:.1f} s, loss {float(loss[0]):.4f}")
        # held-out view: the object alone, seen from a seeded direction
        g = np.random.default_rng(4669 + 1000 * config + 600 + k)
        v = g.standard_normal(3)
        v /= np.linalg.norm(v)
        view = syn.Camera(eye=tuple(3.2 * m.bound * v), at=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0) if abs(v[1]) < 0.9
                          else (1.0, 0.0, 0.0), fov_y_deg=45.0, width=args.ablation_size, height=args.ablation_size)
        rays = api.camera_rays(view)
        dm, im, _ = api.march_depth(sc, rays, n_samples=192, dtype="f32", opacity=False)
        dm, im = dm.cpu().numpy().astype(np.float64), im.cpu().numpy()
        S = args.ablation_size
        Dm = np.where(im >= 0, dm, np.inf).reshape(S, S)
        edge = np.zeros((S, S), bool)
        for sh in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            nb_ = np.roll(Dm, sh, axis=(0, 1))
            edge |= ~np.isfinite(nb_) | (np.abs(nb_ - Dm) > 0.05 * m.bound)
        edge = edge.reshape(-1)
        for name, net in (("regression", reg_nets[-1]), ("classifier", cls_nets[-1])):
            spec = api.object_from_model(m, "bf16", nedf_model=net, nedf_dtype="bf16")
            scn = api.make_scene([spec], [ident])
            dn, idn_ = api.infer_depth_id(scn, rays, dtype="bf16", p_lo=0.5, p_hi=0.5, refine_steps=0)
            dn, idn_ = dn.cpu().numpy().astype(np.float64), idn_.cpu().numpy()
            both = (im >= 0) & (idn_ >= 0)
            err = np.abs(dn - dm)
            e_edge, e_in = err[both & edge], err[both & ~edge]
            res[name].update({
                "hit_agreement": float(np.mean((im >= 0) == (idn_ >= 0))),
                "median_err_interior": float(np.median(e_in)) / m.bound if e_in.size else None,
                "median_err_edge": float(np.median(e_edge)) / m.bound if e_edge.size else None,
                "p90_err_edge": float(np.quantile(e_edge, 0.9)) / m.bound if e_edge.size else None,
                "floater_frac": float(np.mean(err[both] > 0.1 * m.bound)) if both.any() else None,
                "floater_frac_edge": float(np.mean(e_edge > 0.1 * m.bound)) if e_edge.size else None})
        res["pixels_hit"] = int((im >= 0).sum())
        res["edge_pixels_hit"] = int(((im >= 0) & edge).sum())
        out["objects"].append(res)
        log(f"object {k}: {json.dumps(res)}")
    # the frame's depth+ID pass with each form
    frame = {}
    rays = api.camera_rays(cam)
    n = args.width * args.height
    for name, nets in (("regression", reg_nets), ("classifier", cls_nets)):
        objs = [api.object_from_model(m, "bf16", nedf_model=nn, nedf_dtype="bf16") for m, nn in zip(models, nets)]
        scn = api.make_scene(objs, insts)
        ws = api.Workspace()
        for _ in range(max(args.warmup, 1)):
            api.infer_depth_id(scn, rays, dtype="bf16", refine_steps=3, n_samples=args.fallback_samples, ws=ws)
        torch.cuda.synchronize()
        st = api.ws_counters(ws)
        api.profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            api.infer_depth_id(scn, rays, dtype="bf16", refine_steps=3, n_samples=args.fallback_samples, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        stages = api.profile_read()
        api.profile_enable(False)
        ms = e0.elapsed_time(e1) / args.steps
        ev = st["nedf_hits"] + st["fallback"] + st["nedf_misses"]
        net_ms = stages.get("infer.nedf/net", (0.0, 1))[0] / args.steps
        mac = MAC_CLS if name == "classifier" else MAC_NEDF
        tflops = 2.0 * mac * ev / (net_ms * 1e-3) / 1e12 if net_ms > 0 else 0.0
        frame[name] = {"depth_id_ms": ms, "rays_per_s": n / (ms * 1e-3), "network_pairs": int(ev),
                       "fallback_pairs": int(st["fallback"]), "network_ms": net_ms, "network_tflops": tflops,
                       "network_frac_of_bf16_peak": tflops / PEAK_TFLOPS["bf16"]}
        log(f"frame {name}: {json.dumps(frame[name])}")
    cls = frame["classifier"]
    keys = ("median_err_interior", "median_err_edge", "p90_err_edge", "floater_frac", "floater_frac_edge")
    mean = {nm: {k: float(np.mean([o[nm][k] for o in out["objects"] if o[nm][k] is not None])) for k in keys}
            for nm in ("regression", "classifier")}
    return {
        "metric": "classifier-form NeDF depth+ID rays/s (1920x1080, 1000 instances) and regression-vs-classifier "
                  "depth error at discontinuities",
        "value": cls["rays_per_s"], "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": cls["depth_id_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic (seeded SDF-biased NeRF objects; both network forms trained in setup "
                                  "on the library's FP32 marcher labels)",
        "config": {"workload": f"regression (Pluecker gamma8, 8x256) vs classifier (16 points gamma10, 16 residual "
                               f"blocks, 64 x 128 bins) NeDF, {T} Adam steps of {B} rays per object and form; "
                               f"frame {args.width}x{args.height}, {args.instances} instances"},
        "roofline": {"bound": "mfma", "achieved": cls["network_tflops"], "peak": PEAK_TFLOPS["bf16"],
                     "unit": "TFLOP/s", "frac": cls["network_frac_of_bf16_peak"], "traffic": None,
                     "kernel": "infer.nedf/net (classifier form)", "flop_per_pair": 2 * MAC_CLS},
        "mean_over_objects": mean, "objects": out["objects"], "frame": frame,
        "train_ms_per_step": {k: 1e3 * v / (T * len(models)) for k, v in times.items()},
    }


def marcher_cpu_baseline(n_pixels: int, n_samples: int, size: int):
    """FP64 oracle marcher on a seeded pixel subset of the same frame."""
    import synthetic as syn
    from oracle import camera_rays, march_compose
    models, insts, cam, _ = syn.config2_scene(width=size, height=size)
    pix = syn.pixel_subset(2, cam.n_rays, n_pixels)
    o, d = camera_rays(cam, pix)
    t0 = time.perf_counter()
    march_compose(models, insts, o, d, n_samples)
    dt = time.perf_counter() - t0
    return {"value": n_pixels / dt, "unit": "rays/s", "cores": int(host_threads()), "kind": "oracle",
            "sample": f"{n_pixels} seeded pixels of the same {size}x{size} frame, {n_samples} samples/pair, "
                      f"FP64 NumPy, {dt:.1f} s"}


# ---------------------------------------------------------------------------
# training workload (the Adam step alone)
# ---------------------------------------------------------------------------

def sphere_labels(o, d, r=0.5):
    """Synthetic labels: depth of a radius-r sphere at the origin along each
    local ray, and whether the ray hits it."""
    tp = -np.sum(o * d, axis=1)
    b2 = np.sum(o * o, axis=1) - tp ** 2
    hit = b2 < r * r
    return np.where(hit, tp - np.sqrt(np.maximum(r * r - b2, 0.0)), 0.0), hit


def train_step_bytes(B, k0=128, width=256, n_hidden=8, n_params=0, splits=16):
    """Algorithmic HBM bytes of one regression-form step as the library runs
    it: every bfloat16 activation and gradient written once and read by each
    consumer (next layer, data gradient, weight gradient), ReLU masks as bits,
    split-K weight-gradient partials written and summed, Adam over float32
    state (read p, m, v, g; write p, m, v and two bfloat16 copies)."""
    act, x = B * width * 2, B * k0 * 2
    bits = B * width // 8
    encode = B * (2 * 12 + 5) + x + B * 8
    fwd = (x + (n_hidden - 1) * act) + (n_hidden - 1) * (act + bits) + act + B * 8
    dgrad = (n_hidden - 1) * (act + bits + act)
    wgrad = n_hidden * act + (n_hidden - 1) * act + x
    partials = 2 * splits * width * ((k0 + 1) + (n_hidden - 1) * (width + 1)) * 4
    adam = n_params * (4 * 4 + 3 * 4 + 2 * 2)
    return encode + fwd + dgrad + wgrad + partials + adam


def train_bench(args):
    """Adam steps of the intersection network (Eq. 6) on one batch of
    synthetic rays: local rays through the unit ball, sphere labels.  The
    regression form is the frame's network; the classifier form (16 residual
    blocks, 193 outputs) runs beside it."""
    import torch
    from paper_2308_04669_amd import api
    import synthetic as syn
    B = args.train_batch
    o, d = syn.training_rays(3, 7, B)
    D, hit = sphere_labels(o.astype(np.float64), d.astype(np.float64))
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ot, dt, Dt, ht = t(o), t(d), t(D.astype(np.float32)), t(hit.astype(np.uint8))

    def run(model, L, kind, steps, warmup):
        tr = api.Trainer(model.trunk.W, model.trunk.b, enc_L=L, in_kind=kind)
        for _ in range(warmup):
            loss = tr.step(ot, dt, Dt, ht, lr=5e-4)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            loss = tr.step(ot, dt, Dt, ht, lr=5e-4)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, loss.cpu().numpy()

    steps = args.steps
    reg = syn.nedf_model(3, 200)
    ms, loss = run(reg, 8, "pluecker", steps, max(args.warmup, 20))
    n_params = sum(w.size + b.size for w, b in zip(reg.trunk.W, reg.trunk.b))
    nbytes = train_step_bytes(B, n_params=n_params)
    gbs = nbytes / (ms * 1e-3) / 1e9
    flops = 3.0 * 2.0 * MAC_NEDF * B
    traffic, traffic_src = recorded_traffic(TRAFFIC_RECORDS["train.step"], TRAIN_SOURCES)
    cls = syn.classifier_model(3, 500)
    cls_steps = max(steps // 10, 5)
    ms_c, loss_c = run(cls, 10, "points16", cls_steps, 3)
    return {
        "metric": "training rays/s (Adam steps of the intersection network, Eq. 6)",
        "value": B / (ms * 1e-3),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(args.warmup, 20),
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded local rays through the unit ball, radius-0.5 sphere labels; He-initialised "
                "networks)",
        "config": {"workload": f"regression-form intersection network (gamma8 Pluecker -> 8 x 256 -> 2), "
                               f"{B} rays per step, BF16 matrix cores, FP32 master weights, Adam",
                   "batch": B, "loss_last": [float(x) for x in loss]},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                     "traffic": traffic, "traffic_unit": "bytes per step", "traffic_source": traffic_src,
                     "kernel": "train.step (all kernels of one step)", "algorithmic_bytes_per_step": nbytes,
                     "mfma_tflops": flops / (ms * 1e-3) / 1e12,
                     "mfma_frac_of_bf16_peak": flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"]},
        "classifier_form": {"ms_per_step": ms_c, "rays_per_s": B / (ms_c * 1e-3), "steps": cls_steps,
                            "tflops": 3.0 * 2.0 * MAC_CLS * B / (ms_c * 1e-3) / 1e12,
                            "loss_last": [float(x) for x in loss_c]},
    }


def train_cpu_baseline(n_rays):
    """The FP64 oracle's loss and gradients (Eq. 6, regression form) on
    n_rays of the same synthetic rays and labels, one step (no update)."""
    import synthetic as syn
    from oracle import nedf_loss_and_grads
    o, d = syn.training_rays(3, 7, n_rays)
    o, d = o.astype(np.float64), d.astype(np.float64)
    D, hit = sphere_labels(o, d)
    tp = -np.sum(o * d, axis=1)
    mu = np.where(hit, tp - D, 0.0)
    t0 = time.perf_counter()
    nedf_loss_and_grads(syn.nedf_model(3, 200), o, d, mu, hit.astype(np.float64))
    dt = time.perf_counter() - t0
    return {"value": n_rays / dt, "unit": "rays/s", "cores": int(host_threads()), "kind": "oracle",
            "sample": f"{n_rays} of the same synthetic rays, loss and all gradients in FP64 NumPy (no update), "
                      f"{dt:.1f} s"}


def main():
    args = parse()
    if args.sources_hash:
        print(sources_hash(TRAIN_SOURCES if args.workload == "train" else NET_SOURCES))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding is a "
              f"design note, not a build target", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.train_steps is None:
        args.train_steps = 20000 if args.workload == "nedf" else 6000
    if args.steps is None:
        args.steps = 200 if args.workload == "train" else 5
    if args.workload == "frame":
        line, ctx = frame_bench(args)
    elif args.workload == "precision":
        line, ctx = precision_bench(args), None
        args.no_cpu_baseline = True
    elif args.workload == "nedf":
        line, ctx = nedf_bench(args), None
        args.no_cpu_baseline = True
    elif args.workload == "ablation":
        line, ctx = ablation_bench(args), None
        args.no_cpu_baseline = True
    elif args.workload == "train":
        line, ctx = train_bench(args), None
    else:
        line, ctx = marcher_bench(args), None
    if args.copy_mib > 0:
        x = torch.ones(args.copy_mib * (1 << 18), dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = args.copy_mib << 20
    if not args.no_cpu_baseline:
        if args.workload == "frame":
            line["cpu_baseline"] = frame_cpu_baseline(ctx, args.cpu_pixels or 2000, args.fp64_pixels)
            line["quality_fp64"] = line["cpu_baseline"].pop("quality_fp64")
        elif args.workload == "train":
            line["cpu_baseline"] = train_cpu_baseline(args.cpu_pixels or args.train_batch)
        else:
            line["cpu_baseline"] = marcher_cpu_baseline(args.cpu_pixels or 6000, args.samples, args.size)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
