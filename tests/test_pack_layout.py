"""CPU emulation of the matrix-core dataflow over a packed network blob.

The GPU kernels never see the network in natural order: weights are packed
in MFMA fragment order with permuted K columns, biases and heads in
accumulator order.  This test replays, lane by lane in NumPy, exactly the
register dataflow the kernels use (32x32 MFMA operand/accumulator layouts,
first-layer encoding slots, accumulator -> next-layer operand reuse, narrow
head) on the host-packed blob and compares with the oracle's forward pass.
No GPU needed."""
import struct

import numpy as np
import pytest

import synthetic as syn
from oracle import mlp_forward, encode, round_bf16

api = pytest.importorskip("paper_2308_04669_amd.api")

HDR = "<16I16I2I16Q5Q"


def header(blob):
    f = struct.unpack_from(HDR, blob.tobytes(), 0)
    keys = ["magic", "version", "dtype", "in_kind", "enc_L", "width", "n_hidden", "n_out", "rgb_width",
            "dir_L", "n_in", "n_dir", "ks_in", "ks_hidden", "ks_rgb", "frag_bytes"]
    h = dict(zip(keys, f[:16]))
    h["chunk_bytes"] = list(f[16:32])
    h["rgb_chunk_bytes"] = f[32]
    h["off_layer"] = list(f[34:50])
    h["off_head_b"], h["off_rgb"], h["off_rgbh_b"], h["off_scales"], h["total"] = f[50:55]
    return h


def bf16_to_f64(u16):
    return (u16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def enc_slot(p, a, half, L):
    n = p.shape[-1]
    if a < n * L:
        level, comp = a // n, a % n
        return np.sin(np.pi * (2.0 ** level * p[..., comp] + 0.5 * half))
    i = a - n * L
    if i >= (n + 1) // 2:
        return np.zeros(p.shape[:-1])
    c = 2 * i + half
    return p[..., c] if c < n else np.zeros(p.shape[:-1])


def a_frag(blob, h, base, fb, ks, chunk):
    """A operand of K-step ks of block fb: [32 rows, K-per-step] (float64)."""
    if h["dtype"] == 1:
        off = base + fb * chunk + ks * 1024
        lanes = np.frombuffer(blob[off:off + 1024].tobytes(), dtype=np.uint16).reshape(64, 8)
        A = np.zeros((32, 16))
        for l in range(64):
            A[l % 32, 8 * (l // 32):8 * (l // 32) + 8] = bf16_to_f64(lanes[l])
        return A
    off = base + fb * chunk + (ks // 4) * 1024
    words = np.frombuffer(blob[off:off + 1024].tobytes(), dtype=np.float32).reshape(64, 4)
    A = np.zeros((32, 2))
    for l in range(64):
        A[l % 32, l // 32] = words[l, ks % 4]
    return A


def emulate(blob, h, pts):
    """Replay the kernel dataflow for 32 samples; returns head outputs [32, n_out]."""
    bf = h["dtype"] == 1
    kps = 16 if bf else 2
    L = h["enc_L"]
    W = h["width"]
    # per-lane B operand: B[ks] is [K-per-step, 32 samples]; lane half h holds rows (8h..8h+7) or (h)
    def first_B():
        Bs = []
        for ks in range(h["ks_in"]):
            Bm = np.zeros((kps, 32))
            for half in range(2):
                if bf:
                    for j in range(8):
                        Bm[8 * half + j] = enc_slot(pts, 8 * ks + j, half, L)
                else:
                    Bm[half] = enc_slot(pts, ks, half, L)
            if bf:
                Bm = round_bf16(Bm)
            Bs.append(Bm)
        return Bs
    B = first_B()
    out = np.zeros((32, h["n_out"]))
    for layer in range(h["n_hidden"]):
        ks_n = h["ks_in"] if layer == 0 else h["ks_hidden"]
        chunk = h["chunk_bytes"][layer]
        base = h["off_layer"][layer]
        newB = [np.zeros((kps, 32)) for _ in range(W // kps)]
        for fb in range(W // 32):
            bias = np.frombuffer(blob[base + fb * chunk + ks_n * h["frag_bytes"]:][:128].tobytes(), np.float32)
            C = np.zeros((32, 32))   # [row i, sample]
            for ks in range(ks_n):
                C += a_frag(blob, h, base, fb, ks, chunk) @ B[ks]
            for l in range(64):
                half = l // 32
                for r in range(16):
                    row = 8 * (r // 4) + 4 * half + (r % 4)
                    v = max(C[row, l % 32] + bias[half * 16 + r], 0.0)
                    if bf:
                        newB[2 * fb + r // 8][8 * half + (r % 8), l % 32] = v
                    else:
                        newB[16 * fb + r][half, l % 32] = v
                    if layer == h["n_hidden"] - 1:
                        for o in range(h["n_out"]):
                            hw = np.frombuffer(blob[base + fb * chunk + ks_n * h["frag_bytes"] + 128 * (1 + o):][:128]
                                               .tobytes(), np.float32)
                            out[l % 32, o] += hw[half * 16 + r] * v
        B = [round_bf16(x) for x in newB] if bf else newB
    hb = np.frombuffer(blob[h["off_head_b"]:][:8].tobytes(), np.float32)
    return out + hb[:h["n_out"]]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_density_b_blob_dataflow(dtype):
    _, b = syn.config1_models()
    shape = api.mlp_shape("xyz", 6, 64, 3, 1)
    blob = api.pack_host(b.trunk.W, b.trunk.b, shape, dtype)
    h = header(blob)
    assert h["magic"] == 0x4644454E and h["total"] == blob.size
    pts = syn.rng(0, 60).uniform(-1, 1, (32, 3))
    got = emulate(blob, h, pts)
    ref = mlp_forward(encode(pts, 6), b.trunk, gemm="bf16" if dtype == "bf16" else None)
    tol = 1e-9 if dtype == "f32" else 1e-9
    assert np.allclose(got, ref, atol=tol * 10, rtol=1e-6), np.abs(got - ref).max()


def test_wide_blob_dataflow_bf16():
    # 256-wide, random biases so that the bias/head tables are exercised
    g = syn.rng(0, 61)
    t = syn.normal_mlp(g, [63, 256, 256, 256, 2])
    for bb in t.b:
        bb[:] = (g.standard_normal(bb.shape) * 0.1).astype(np.float32)
    shape = api.mlp_shape("xyz", 10, 256, 3, 2)
    blob = api.pack_host(t.W, t.b, shape, "bf16")
    h = header(blob)
    pts = g.uniform(-1, 1, (32, 3))
    got = emulate(blob, h, pts)
    ref = mlp_forward(encode(pts, 10), t, gemm="bf16")
    assert np.allclose(got, ref, atol=1e-6, rtol=1e-5), np.abs(got - ref).max()


def e4m3_decode(codes):
    codes = np.asarray(codes, np.int64)
    s = np.where(codes & 0x80, -1.0, 1.0)
    e = (codes >> 3) & 15
    m = codes & 7
    v = np.where(e == 0, np.ldexp(m / 8.0, -6), np.ldexp(1.0 + m / 8.0, e - 7))
    return s * v


def emulate_fp8(blob, h, pts6, L):
    """Replay of the FP8 dataflow (K-steps of 64, 32 bytes per lane, per-layer
    scales folded into bias and epilogue) for 32 Pluecker inputs."""
    from oracle import round_e4m3
    sc = np.frombuffer(blob[h["off_scales"]:][:4 * 33].tobytes(), np.float32).astype(np.float64)
    W = h["width"]

    def frag(base, fb, ks, chunk):
        off = base + fb * chunk + ks * 2048
        A = np.zeros((32, 64))
        for l in range(64):
            for jj in range(32):
                byte = blob[off + (jj // 16) * 1024 + l * 16 + (jj % 16)]
                A[l % 32, 32 * (l // 32) + jj] = e4m3_decode(byte)
        return A

    B = []
    for ks in range(h["ks_in"]):
        Bm = np.zeros((64, 32))
        for half in range(2):
            for j in range(32):
                Bm[32 * half + j] = round_e4m3(enc_slot(pts6, 32 * ks + j, half, L) * sc[0])
        B.append(Bm)
    out = np.zeros((32, h["n_out"]))
    for layer in range(h["n_hidden"]):
        ks_n = h["ks_in"] if layer == 0 else h["ks_hidden"]
        chunk = h["chunk_bytes"][layer]
        base = h["off_layer"][layer]
        to_real, inv_next = sc[1 + 2 * layer], sc[2 + 2 * layer]
        newB = [np.zeros((64, 32)) for _ in range(W // 64)]
        for fb in range(W // 32):
            bias = np.frombuffer(blob[base + fb * chunk + ks_n * 2048:][:128].tobytes(), np.float32)
            C = np.zeros((32, 32))
            for ks in range(ks_n):
                C += frag(base, fb, ks, chunk) @ B[ks]
            for l in range(64):
                half = l // 32
                for r in range(16):
                    row = 8 * (r // 4) + 4 * half + (r % 4)
                    real = max((C[row, l % 32] + bias[half * 16 + r]) * to_real, 0.0)
                    j = (fb % 2) * 16 + r
                    newB[fb // 2][32 * half + j, l % 32] = round_e4m3(real * inv_next)
                    if layer == h["n_hidden"] - 1:
                        for o in range(h["n_out"]):
                            hw = np.frombuffer(blob[base + fb * chunk + ks_n * 2048 + 128 * (1 + o):][:128].tobytes(),
                                               np.float32)
                            out[l % 32, o] += hw[half * 16 + r] * real
        B = newB
    hb = np.frombuffer(blob[h["off_head_b"]:][:8].tobytes(), np.float32)
    return out + hb[:h["n_out"]]


def test_fp8_blob_dataflow():
    g = syn.rng(0, 62)
    t = syn.normal_mlp(g, [102, 256, 256, 2], hidden_gain=2.0)
    for bb in t.b:
        bb[:] = (g.standard_normal(bb.shape) * 0.05).astype(np.float32)
    pts6 = np.concatenate([g.standard_normal((32, 3)), g.uniform(-0.8, 0.8, (32, 3))], axis=1)
    pts6[:, :3] /= np.linalg.norm(pts6[:, :3], axis=1, keepdims=True)
    # scales {w_scale, a_scale} per hidden layer from the float64 forward
    x = encode(pts6, 8)
    acts = [x]
    hcur = x
    for i in range(2):
        hcur = np.maximum(hcur @ t.W[i].astype(np.float64).T + t.b[i], 0)
        acts.append(hcur)
    scales = np.array([[np.abs(t.W[i]).max() / 448, np.abs(acts[i]).max() / 448] for i in range(2)])
    shape = api.mlp_shape("pluecker", 8, 256, 2, 2)
    blob = api.pack_host(t.W, t.b, shape, "fp8", fp8_scales=scales.reshape(-1))
    h = header(blob)
    assert h["dtype"] == 2 and h["ks_in"] == 2 and h["ks_hidden"] == 4
    got = emulate_fp8(blob, h, pts6, 8)
    ref = mlp_forward(x, t, scales=[tuple(s) for s in scales])
    assert np.allclose(got, ref, atol=1e-4, rtol=1e-4), np.abs(got - ref).max()
