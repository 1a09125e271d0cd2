"""GPU parity of the classifier-form intersection network (16 points on the
line, gamma_10, ReLU head, residual blocks, two-level classifier decoded by
argmax; Sec. "Intersection network", Eq. 3-4, appendix architecture) inside
nedf_infer_depth_id, through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest

import synthetic as syn
from tests.gpu_util import need_gpu, gpu_scene, log, pair_oracle

pytestmark = pytest.mark.gpu


def _classifier_nets(models, insts, o, d, n_blocks=16, hit_spread=3.0):
    """Random classifier networks, one per object, whose hit logit is centred
    and spread on this scene's rays: the untrained network's logit carries a
    common offset (its inputs are non-negative), which would send every pair
    the same way.  The centring uses the oracle's forward pass on the rays
    of the object's first instance."""
    from oracle import classifier_eval, f32_record, to_local
    nets = []
    for k in range(len(models)):
        net = syn.classifier_model(3, 400 + k, n_blocks=n_blocks, bias_std=0.05)
        inst = next((i for i in insts if i.model == k), None)
        if inst is None:  # an object without instances
            nets.append(net)
            continue
        o_l, d_l = to_local(f32_record(inst), o, d)
        hitting = np.linalg.norm(np.cross(o_l, d_l), axis=1) < net.bound
        _, a = classifier_eval(net, o_l[hitting][:400], d_l[hitting][:400])
        med = float(np.median(a))
        net.trunk.W[-1][0] *= np.float32(hit_spread)
        net.trunk.b[-1][0] = np.float32(-hit_spread * med)
        nets.append(net)
    return nets


def _setup(n_inst=6, size=48, n_blocks=16):
    from oracle import camera_rays
    models, insts, cam = syn.sdf_scene(3, n_inst, width=size, height=size)
    o, d = camera_rays(cam)
    o32, d32 = o.astype(np.float32), d.astype(np.float32)
    nets = _classifier_nets(models, insts, o32.astype(np.float64), d32.astype(np.float64), n_blocks)
    return models, insts, nets, o32, d32


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_classifier_network_parity(dtype):
    need_gpu()
    import torch
    from paper_2308_04669_amd import api
    from oracle import f32_record
    from tests.test_gpu_pipeline import _infer_compare
    models, insts, nets, o32, d32 = _setup()
    log(f"case: classifier NeDF {dtype} 48x48, 6 instances, 16 residual blocks, float32 ray arrays")
    sc = gpu_scene(models, insts, dtype, nedf_models=nets)
    rays = api.array_rays(torch.from_numpy(o32).cuda(), torch.from_numpy(d32).cuda())
    ws = api.Workspace()
    depth, ident = api.infer_depth_id(sc, rays, dtype=dtype, refine_steps=0, n_samples=128, ws=ws)
    stats = api.ws_counters(ws)
    assert api.check_status(ws) == 0
    torch.cuda.synchronize()
    depth, ident = depth.cpu().numpy().astype(np.float64), ident.cpu().numpy()
    o, d = o32.astype(np.float64), d32.astype(np.float64)
    res = []
    for inst in insts:
        rec = f32_record(inst)
        res.append(pair_oracle(models[rec.model], nets[rec.model], rec, o, d, 128, dtype))
    # BF16: the argmax decoding turns the rare single-step jumps of rounded
    # activations into bin changes on near-ties; the exemption bound is twice
    # the largest logit jump measured between two summation orders over the
    # batch, which exempts about a quarter of the hits from the depth check
    st = _infer_compare(depth, ident, res, dtype, f"classifier {dtype}", cap=0.05 if dtype == "f32" else 0.3,
                        route_depth=True)
    log(f"routing {stats}")
    net_pairs = stats["nedf_hits"] + stats["fallback"] + stats["nedf_misses"]
    n_amb = int(sum((r.amb > 0).sum() for r in res))
    log(f"pairs with a near-tie decision: {n_amb} of {net_pairs}")
    # the network decided a good share of the pairs itself, over several
    # 128-pair work items per object
    assert stats["nedf_hits"] > 100 and stats["nedf_misses"] > 100, stats
    assert st["checked"] > 300, st


def test_classifier_edge_cases():
    """One residual block (the smallest instantiated depth), an empty frame
    of rays, and a ray count that leaves a ragged last work item."""
    need_gpu()
    import torch
    from paper_2308_04669_amd import api
    from oracle import f32_record
    from tests.test_gpu_pipeline import _infer_compare
    models, insts, nets, o32, d32 = _setup(n_inst=3, size=40, n_blocks=1)
    log("case: classifier NeDF f32, 1 block, 3 instances, 1,597 rays; empty ray set")
    sc = gpu_scene(models, insts, "f32", nedf_models=nets)
    n = 1597
    rays = api.array_rays(torch.from_numpy(o32[:n]).cuda(), torch.from_numpy(d32[:n]).cuda())
    depth, ident = api.infer_depth_id(sc, rays, dtype="f32", refine_steps=0)
    torch.cuda.synchronize()
    o, d = o32[:n].astype(np.float64), d32[:n].astype(np.float64)
    res = [pair_oracle(models[f32_record(i).model], nets[i.model], f32_record(i), o, d, 128, "f32") for i in insts]
    _infer_compare(depth.cpu().numpy().astype(np.float64), ident.cpu().numpy(), res, "f32", "classifier 1 block",
                   route_depth=True)
    empty = api.array_rays(torch.zeros((0, 3), device="cuda"), torch.zeros((0, 3), device="cuda"))
    d0, i0 = api.infer_depth_id(sc, empty, dtype="f32", refine_steps=0)
    assert d0.numel() == 0 and i0.numel() == 0


def _bin_centre_labels(o, d, g, l=1.0, hit_frac=0.5):
    """Labels whose mu sits at the centre of a fine bin (so that the bins of
    S are the same whatever the precision of mu): random bins, depth
    t_perp - mu, about ``hit_frac`` of the rays hits."""
    from oracle import segment_inverse
    n = o.shape[0]
    c = g.integers(0, 64, n)
    f = g.integers(0, 128, n)
    mu = segment_inverse(c, f, l) + l / 8192.0
    tp = -np.sum(o * d, axis=1)
    hit = g.random(n) < hit_frac
    return np.where(hit, tp - mu, 0.0), hit, mu


def test_classifier_training_step_matches_oracle():
    """Loss of Eq. 6 and every layer's gradients of one training step of the
    16-block classifier network against the FP64 oracle (and its bfloat16
    emulation), then the first Adam update against its closed form."""
    need_gpu()
    import torch
    from paper_2308_04669_amd import api
    from oracle import classifier_loss_and_grads
    model = syn.classifier_model(3, 450, bias_std=0.05)
    B = 1024
    o, d = syn.training_rays(3, 451, B)
    o64, d64 = o.astype(np.float64), d.astype(np.float64)
    D, hit, _ = _bin_centre_labels(o64, d64, np.random.default_rng(452))
    D32 = D.astype(np.float32)
    log("case: classifier training step, 16 blocks, B = 1024, labels at fine-bin centres")
    tr = api.Trainer(model.trunk.W, model.trunk.b, enc_L=10, in_kind="points16")
    t = lambda x, dt=None: torch.from_numpy(np.ascontiguousarray(x if dt is None else x.astype(dt))).cuda()
    loss = tr.step(t(o), t(d), t(D32), t(hit, np.uint8), lr=0.0)
    torch.cuda.synchronize()
    loss = loss.cpu().numpy().astype(np.float64)
    gW, gb = tr.export(1)
    tp = -np.sum(o64 * d64, axis=1)
    mu = np.where(hit, tp - D32.astype(np.float64), 0.0)
    ref = classifier_loss_and_grads(model, o64, d64, mu, hit.astype(np.float64))
    em = classifier_loss_and_grads(model, o64, d64, mu, hit.astype(np.float64), gemm="bf16")
    log(f"loss gpu {loss} oracle {ref[:3]} bf16-emulated {em[:3]}")
    for i in range(3):
        assert abs(loss[i] - em[i]) <= 2e-3 * abs(em[i]) + 1e-7, (i, loss, em[:3])
        assert abs(loss[i] - ref[i]) <= 2e-2 * abs(ref[i]) + 1e-7, (i, loss, ref[:3])
    worst_em = 0.0
    for i, ((dw, db), (ew_, eb_)) in enumerate(zip(ref[3], em[3])):
        ew = np.linalg.norm(gW[i] - dw) / max(np.linalg.norm(dw), 1e-30)
        e2w = np.linalg.norm(gW[i] - ew_) / max(np.linalg.norm(ew_), 1e-30)
        e2b = np.linalg.norm(gb[i] - eb_) / max(np.linalg.norm(eb_), 1e-30)
        if i in (0, 1, 2, 16, 31, 32, 33):
            log(f"layer {i}: rel err vs float64 W {ew:.3e}; vs bf16-emulated W {e2w:.3e} b {e2b:.3e}")
        worst_em = max(worst_em, e2w, e2b)
        assert ew <= 0.25, (i, ew)
    log(f"worst relative gradient error against the bf16 emulation: {worst_em:.3e}")
    assert worst_em <= 3e-2
    W0, _ = tr.export(0)
    tr.step(t(o), t(d), t(D32), t(hit, np.uint8), lr=5e-4)
    W1, _ = tr.export(0)
    gW2, _ = tr.export(1)
    for i in (0, 1, 33):
        m = 0.9 * 0.1 * gW[i] + 0.1 * gW2[i]
        v = 0.999 * 0.001 * gW[i] ** 2 + 0.001 * gW2[i] ** 2
        upd = -5e-4 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
        assert np.allclose(W1[i] - W0[i], upd, atol=2e-6 * 5e-4 + 1e-9, rtol=2e-3), i
    assert W1[33].shape == (193, 256)
