// Training of an intersection network (Eq. 6 in regression form, training
// details of the paper: Adam, lr 5e-4): input encoding and label conversion
// (inverse of Eq. 2), bfloat16 matrix-core GEMMs with fused epilogues for the
// forward pass, the ReLU-masked data gradients and split-K weight gradients,
// the head + loss kernel and Adam on float32 master weights.
#include <cstring>

#include "device_common.h"
#include "runtime.h"
#include "train_layout.h"

namespace nedf {
namespace {

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));
}
__device__ __forceinline__ float bf16_val(uint16_t u) { return __uint_as_float(uint32_t(u) << 16); }

// ---- input encoding and labels ------------------------------------------------
// Features in natural order [p, sin(2^0 pi p), cos(2^0 pi p), ...] of the
// Pluecker (d, o x d) or xyz input, zero padded to Kpad; labels
// mu* = (t_perp - D) / l and alpha = hit.
__global__ void k_train_encode(const float* o_l, const float* d_l, const float* depth, const uint8_t* hit,
                               int B, int in_kind, int L, int Kpad, float bound, uint16_t* H, float* mu,
                               float* alpha) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const float o[3] = {o_l[3 * s], o_l[3 * s + 1], o_l[3 * s + 2]};
  const float d[3] = {d_l[3 * s], d_l[3 * s + 1], d_l[3 * s + 2]};
  float p[6], plo[6] = {0, 0, 0, 0, 0, 0};
  int n;
  if (in_kind == NEDF_IN_PLUECKER) {
    n = 6;
    float tp;
    line_of_local(o, d, p, plo, tp);
  } else {
    n = 3;
    p[0] = o[0]; p[1] = o[1]; p[2] = o[2];
  }
  uint16_t* row = H + size_t(s) * Kpad;
  for (int f = 0; f < Kpad; ++f) {
    float v = 0.0f;
    if (f < n) {
      v = p[f];
    } else if (f < n * (1 + 2 * L)) {
      const int q = f - n, level = q / (2 * n), w = q % (2 * n), c = w % n;
      v = sinpi_hw(float(1 << level) * p[c], float(1 << level) * plo[c], w >= n ? 1 : 0);
    }
    row[f] = bf16_bits(v);
  }
  if (!depth) return;  // calibration: no labels
  float pl[6], pllo[6], tperp;
  line_of_local(o, d, pl, pllo, tperp);
  const bool h = hit[s] != 0;
  alpha[s] = h ? 1.0f : 0.0f;
  mu[s] = h ? (tperp - depth[s]) / bound : 0.0f;
}

// amax of |x| over n bfloat16 values (non-negative float bits order as
// unsigned integers).
__global__ void k_amax16(const uint16_t* x, size_t n, uint32_t* out) {
  float m = 0.f;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    m = fmaxf(m, fabsf(bf16_val(x[i])));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void k_amax32(const float* x, size_t n, uint32_t* out) {
  float m = 0.f;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    m = fmaxf(m, fabsf(x[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// Scales {w_scale, a_scale} = amax / 448 per hidden layer (E4M3 largest finite).
__global__ void k_fp8_scales(const uint32_t* amax_w, const uint32_t* amax_a, int n_hidden, float* scales) {
  const int i = threadIdx.x;
  if (i >= n_hidden) return;
  const float w = __uint_as_float(amax_w[i]), a = __uint_as_float(amax_a[i]);
  scales[2 * i] = w > 0.f ? w / 448.0f : 1.0f;
  scales[2 * i + 1] = a > 0.f ? a / 448.0f : 1.0f;
}

// ---- GEMM ---------------------------------------------------------------------
// C[M][N] = A[M][K] B[K][N] on 32x32x16 bf16 matrix cores, 64x64 tile per
// workgroup (4 waves, 32x32 each), K tiles of 32 staged in LDS with K
// contiguous.  AT: 0 A stored [M][K], 1 stored [K][M].  BT: 0 B stored
// [K][N], 1 stored [N][K].  Split-K over blockIdx.z.
struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  int M, N, K, lda, ldb;
  int k_per_split;
  // epilogue
  const float* bias;     // EPI 0
  const uint16_t* mask;  // EPI 1 ([M][ldm] bf16, > 0 keeps)
  int ldm;
  uint16_t* out16;       // EPI 0/1 [M][ldo]
  float* out32;          // EPI 2 [M][ldo] (atomic add), columns < n_valid
  int ldo, n_valid;
};

constexpr int GT_BM = 64, GT_BN = 64, GT_BK = 32, GT_LD = 40;  // LDS row stride (bf16), 80 bytes

template <int AT, int BT, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GT_BM * GT_LD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GT_BN * GT_LD];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * GT_BM, n0 = blockIdx.y * GT_BN;
  const int kb = blockIdx.z * g.k_per_split;
  const int ke = min(g.K, kb + g.k_per_split);
  f32x16_t acc = {};
  for (int k0 = kb; k0 < ke; k0 += GT_BK) {
    // A tile -> As[m][k]
    if (AT == 0) {
      const int m = t >> 2, kk = (t & 3) * 8;
      const uint4 v = *reinterpret_cast<const uint4*>(g.A + size_t(m0 + m) * g.lda + k0 + kk);
      *reinterpret_cast<uint4*>(As + m * GT_LD + kk) = v;
    } else {
      const int k = t >> 3, mm = (t & 7) * 8;
      const uint4 v = *reinterpret_cast<const uint4*>(g.A + size_t(k0 + k) * g.lda + m0 + mm);
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int i = 0; i < 8; ++i) As[(mm + i) * GT_LD + k] = e[i];
    }
    // B tile -> Bs[n][k]
    if (BT == 1) {
      const int n = t >> 2, kk = (t & 3) * 8;
      const uint4 v = *reinterpret_cast<const uint4*>(g.B + size_t(n0 + n) * g.ldb + k0 + kk);
      *reinterpret_cast<uint4*>(Bs + n * GT_LD + kk) = v;
    } else {
      const int k = t >> 3, nn = (t & 7) * 8;
      const uint4 v = *reinterpret_cast<const uint4*>(g.B + size_t(k0 + k) * g.ldb + n0 + nn);
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs[(nn + i) * GT_LD + k] = e[i];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GT_BK / 16; ++ks) {
      const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(As + (wm * 32 + (lane & 31)) * GT_LD + ks * 16 + 8 * (lane >> 5));
      const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(Bs + (wn * 32 + (lane & 31)) * GT_LD + ks * 16 + 8 * (lane >> 5));
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator (row i, col j) of the 32x32 block: lane holds col = lane % 32
  const int col = n0 + wn * 32 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wm * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
    const float v = acc[r];
    if (EPI == 0) {
      g.out16[size_t(row) * g.ldo + col] = bf16_bits(fmaxf(v + g.bias[col], 0.0f));
    } else if (EPI == 1) {
      const bool keep = bf16_val(g.mask[size_t(row) * g.ldm + col]) > 0.0f;
      g.out16[size_t(row) * g.ldo + col] = bf16_bits(keep ? v : 0.0f);
    } else {
      if (col < g.n_valid) atomicAdd(&g.out32[size_t(row) * g.ldo + col], v);
    }
  }
}

// ---- head and loss ------------------------------------------------------------
// One block of 256 threads per 256 samples; width must be 256.  Phase 1: the
// (mu_hat, z) head and the loss terms per sample; phase 2: per feature, the
// head gradients and G = (g_mu W_h0 + g_z W_h1) * (H > 0).
__global__ __launch_bounds__(256) void k_head_loss(const uint16_t* H, const float* Wh, const float* bh,
                                                   const float* mu, const float* alpha, int B, float w_hit,
                                                   float* loss, uint16_t* G, float* gWh, float* gbh) {
  __shared__ float sW[2][256];
  __shared__ float sg[2][256];
  __shared__ float red[3][256];
  const int t = threadIdx.x;
  const int s0 = blockIdx.x * 256;
  sW[0][t] = Wh[t];
  sW[1][t] = Wh[256 + t];
  __syncthreads();
  const int s = s0 + t;
  float lm = 0.f, lb = 0.f;
  sg[0][t] = 0.f;
  sg[1][t] = 0.f;
  if (s < B) {
    const uint16_t* row = H + size_t(s) * 256;
    float a0 = bh[0], a1 = bh[1];
    for (int k = 0; k < 256; ++k) {
      const float h = bf16_val(row[k]);
      a0 = fmaf(sW[0][k], h, a0);
      a1 = fmaf(sW[1][k], h, a1);
    }
    const float al = alpha[s], m = mu[s];
    const float e = a0 - m;
    lm = al * e * e;
    lb = fmaxf(a1, 0.f) + log1pf(expf(-fabsf(a1))) - al * a1;
    const float invB = 1.0f / float(B);
    sg[0][t] = 2.0f * al * e * invB;
    sg[1][t] = w_hit * (1.0f / (1.0f + expf(-a1)) - al) * invB;
  }
  red[0][t] = lm;
  red[1][t] = lb;
  red[2][t] = 0.f;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      red[0][t] += red[0][t + off];
      red[1][t] += red[1][t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    const float invB = 1.0f / float(B);
    atomicAdd(&loss[1], red[0][0] * invB);
    atomicAdd(&loss[2], red[1][0] * invB);
    atomicAdd(&loss[0], (red[0][0] + w_hit * red[1][0]) * invB);
  }
  // phase 2: thread t owns feature k = t
  const int k = t;
  float gw0 = 0.f, gw1 = 0.f;
  const int ns = min(256, B - s0);
  for (int i = 0; i < ns; ++i) {
    const size_t idx = size_t(s0 + i) * 256 + k;
    const float h = bf16_val(H[idx]);
    const float g0 = sg[0][i], g1 = sg[1][i];
    gw0 = fmaf(g0, h, gw0);
    gw1 = fmaf(g1, h, gw1);
    G[idx] = bf16_bits(h > 0.0f ? fmaf(g0, sW[0][k], g1 * sW[1][k]) : 0.0f);
  }
  atomicAdd(&gWh[k], gw0);
  atomicAdd(&gWh[256 + k], gw1);
  if (t < 2) {
    float sum = 0.f;
    for (int i = 0; i < ns; ++i) sum += sg[t][i];
    atomicAdd(&gbh[t], sum);
  }
}

// Bias gradient: column sums of G [B][N] (N = blockDim).
__global__ void k_colsum(const uint16_t* G, int B, int N, int rows_per_block, float* gb) {
  const int n = threadIdx.x;
  const int r0 = blockIdx.x * rows_per_block, r1 = min(B, r0 + rows_per_block);
  float sum = 0.f;
  for (int r = r0; r < r1; ++r) sum += bf16_val(G[size_t(r) * N + n]);
  atomicAdd(&gb[n], sum);
}

__global__ void k_zero_f32(float* p, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// Adam (Kingma & Ba 2015) with bias correction, step t = *step + 1; the
// bfloat16 copy of weight matrices is refreshed in the same pass.
__global__ void k_adam(float* p, float* m, float* v, const float* g, int n, const int64_t* step, float lr,
                       float b1, float b2, float eps, uint16_t* w16, int K, int Kpad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float t = float(*step + 1);
  const float bc1 = 1.0f - powf(b1, t), bc2 = 1.0f - powf(b2, t);
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  p[i] = pi;
  if (w16) w16[size_t(i / K) * Kpad + (i % K)] = bf16_bits(pi);
}

__global__ void k_step_inc(int64_t* step) {
  if (threadIdx.x == 0) *step += 1;
}

// Initial state: master weights from float32 arrays, moments and gradients
// zero, bfloat16 copies (zero padded).
__global__ void k_copy_w(const float* src, float* dst, uint16_t* w16, int N, int K, int Kpad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * Kpad) return;
  const int r = i / Kpad, c = i % Kpad;
  if (c < K) {
    const float v = src[r * K + c];
    if (dst) dst[r * K + c] = v;
    if (w16) w16[i] = bf16_bits(v);
  } else if (w16) {
    w16[i] = 0;
  }
}

unsigned blocks(size_t n, int b = 256) { return unsigned((n + b - 1) / b); }

template <int AT, int BT, int EPI>
void gemm(const GemmArgs& g, int splits, hipStream_t s) {
  dim3 grid(g.M / GT_BM, (g.N + GT_BN - 1) / GT_BN, splits);
  hipLaunchKernelGGL((k_gemm<AT, BT, EPI>), grid, dim3(256), 0, s, g);
}

}  // namespace

size_t train_ws_bytes(const nedf_mlp_shape& sh, int B) {
  const nedf_train_layout tl = nedf_train_layout_of(sh);
  size_t off = 0;
  off = nedf_tl_align(off + size_t(B) * tl.L[0].Kpad * 2);           // H_in
  off = nedf_tl_align(off + size_t(B) * sh.width * 2 * sh.n_hidden);  // H_0..H_{n-1}
  off = nedf_tl_align(off + size_t(B) * sh.width * 2 * 2);            // G ping-pong
  off = nedf_tl_align(off + size_t(B) * 4 * 2);                       // mu, alpha
  return off;
}

hipError_t launch_train_init(const nedf_mlp_shape& sh, const float* const* W, const float* const* b, uint8_t* st,
                             hipStream_t s) {
  const nedf_train_layout tl = nedf_train_layout_of(sh);
  hipLaunchKernelGGL(k_zero_f32, dim3(blocks(tl.total / 4)), dim3(256), 0, s, reinterpret_cast<float*>(st),
                     tl.total / 4);
  for (int i = 0; i < tl.n_layers; ++i) {
    const nedf_train_layer& l = tl.L[i];
    hipLaunchKernelGGL(k_copy_w, dim3(blocks(size_t(l.N) * l.Kpad)), dim3(256), 0, s, W[i],
                       reinterpret_cast<float*>(st + l.W), reinterpret_cast<uint16_t*>(st + l.W16), l.N, l.K, l.Kpad);
    hipLaunchKernelGGL(k_copy_w, dim3(blocks(size_t(l.N))), dim3(256), 0, s, b[i],
                       reinterpret_cast<float*>(st + l.b), static_cast<uint16_t*>(nullptr), 1, l.N, l.N);
  }
  return hipGetLastError();
}

hipError_t launch_train_step(const nedf_mlp_shape& sh, uint8_t* st, const float* o_l, const float* d_l,
                             const float* depth, const uint8_t* hit, int B, float lr, float b1, float b2, float eps,
                             float w_hit, float bound, float* loss, uint8_t* ws, hipStream_t s) {
  const nedf_train_layout tl = nedf_train_layout_of(sh);
  const int W = sh.width, NH = sh.n_hidden;
  const int K0p = tl.L[0].Kpad;
  size_t off = 0;
  uint16_t* Hin = reinterpret_cast<uint16_t*>(ws + off);
  off = nedf_tl_align(off + size_t(B) * K0p * 2);
  uint16_t* Hs = reinterpret_cast<uint16_t*>(ws + off);
  off = nedf_tl_align(off + size_t(B) * W * 2 * NH);
  uint16_t* G0 = reinterpret_cast<uint16_t*>(ws + off);
  uint16_t* G1 = G0 + size_t(B) * W;
  off = nedf_tl_align(off + size_t(B) * W * 2 * 2);
  float* mu = reinterpret_cast<float*>(ws + off);
  float* alpha = mu + B;
  auto Hl = [&](int l) { return Hs + size_t(l) * B * W; };
  auto F = [&](size_t o) { return reinterpret_cast<float*>(st + o); };
  auto U = [&](size_t o) { return reinterpret_cast<uint16_t*>(st + o); };

  prof_mark("train.step", s, true);
  // zero gradients and the loss
  for (int i = 0; i < tl.n_layers; ++i) {
    const nedf_train_layer& l = tl.L[i];
    hipLaunchKernelGGL(k_zero_f32, dim3(blocks(size_t(l.N) * l.K)), dim3(256), 0, s, F(l.gW), size_t(l.N) * l.K);
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(256), 0, s, F(l.gb), size_t(l.N));
  }
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, loss, size_t(3));
  hipLaunchKernelGGL(k_train_encode, dim3(blocks(B)), dim3(256), 0, s, o_l, d_l, depth, hit, B, sh.in_kind, sh.enc_L,
                     K0p, bound, Hin, mu, alpha);
  // forward: H_l = relu(H_{l-1} W_l^T + b_l)
  for (int l = 0; l < NH; ++l) {
    GemmArgs g{};
    g.A = l == 0 ? Hin : Hl(l - 1);
    g.lda = l == 0 ? K0p : W;
    g.B = U(tl.L[l].W16);
    g.ldb = tl.L[l].Kpad;
    g.M = B; g.N = W; g.K = tl.L[l].Kpad;
    g.k_per_split = g.K;
    g.bias = F(tl.L[l].b);
    g.out16 = Hl(l);
    g.ldo = W;
    gemm<0, 1, 0>(g, 1, s);
  }
  // head, loss, G_{NH-1}
  const nedf_train_layer& hd = tl.L[NH];
  hipLaunchKernelGGL(k_head_loss, dim3(blocks(B)), dim3(256), 0, s, Hl(NH - 1), F(hd.W), F(hd.b), mu, alpha, B,
                     w_hit, loss, G0, F(hd.gW), F(hd.gb));
  // backward through the hidden layers
  uint16_t* Gc = G0;
  uint16_t* Gn = G1;
  for (int l = NH - 1; l >= 0; --l) {
    const nedf_train_layer& L = tl.L[l];
    // weight gradient dW_l = G_l^T H_{l-1}   (split-K over the batch)
    GemmArgs w{};
    w.A = Gc; w.lda = W;                            // stored [B][W] = [K][M]
    w.B = l == 0 ? Hin : Hl(l - 1);
    w.ldb = l == 0 ? K0p : W;                       // stored [B][Kpad] = [K][N]
    w.M = W; w.N = L.Kpad; w.K = B;
    const int splits = (B >= 4096 && B % 1024 == 0) ? B / 1024 : 1;
    w.k_per_split = (B + splits - 1) / splits;
    w.out32 = F(L.gW);
    w.ldo = L.K;
    w.n_valid = L.K;
    gemm<1, 0, 2>(w, splits, s);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(B, 256)), dim3(W), 0, s, Gc, B, W, 256, F(L.gb));
    if (l > 0) {
      // data gradient G_{l-1} = (G_l W_l) * (H_{l-1} > 0)
      GemmArgs d{};
      d.A = Gc; d.lda = W;                          // [B][W]
      d.B = U(L.W16); d.ldb = L.Kpad;               // W_l [W][Kpad] = [K][N]
      d.M = B; d.N = W; d.K = W;
      d.k_per_split = W;
      d.mask = Hl(l - 1); d.ldm = W;
      d.out16 = Gn; d.ldo = W;
      gemm<0, 0, 1>(d, 1, s);
      uint16_t* tmp = Gc; Gc = Gn; Gn = tmp;
    }
  }
  // Adam on every parameter array
  const int64_t* step = reinterpret_cast<const int64_t*>(st);
  for (int i = 0; i < tl.n_layers; ++i) {
    const nedf_train_layer& L = tl.L[i];
    const int nw = L.N * L.K;
    hipLaunchKernelGGL(k_adam, dim3(blocks(nw)), dim3(256), 0, s, F(L.W), F(L.mW), F(L.vW), F(L.gW), nw, step, lr, b1,
                       b2, eps, U(L.W16), L.K, L.Kpad);
    hipLaunchKernelGGL(k_adam, dim3(blocks(L.N)), dim3(256), 0, s, F(L.b), F(L.mb), F(L.vb), F(L.gb), L.N, step, lr,
                       b1, b2, eps, static_cast<uint16_t*>(nullptr), 1, 1);
  }
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, s, reinterpret_cast<int64_t*>(st));
  prof_mark("train.step", s, false);
  return hipGetLastError();
}

// Per-layer E4M3 scales of a network from a calibration batch: the bfloat16
// forward pass of the training path records amax of every hidden layer's
// input; weight scales from the float32 weights.  ws holds a temporary
// training state followed by the forward workspace.
hipError_t launch_fp8_calibrate(const nedf_mlp_shape& sh, const float* const* W, const float* const* b,
                                const float* o_l, const float* d_l, int B, float* scales, uint8_t* ws,
                                hipStream_t s) {
  const nedf_train_layout tl = nedf_train_layout_of(sh);
  uint8_t* st = ws;
  uint8_t* fw = ws + nedf_tl_align(tl.total);
  uint32_t* amax = reinterpret_cast<uint32_t*>(fw + train_ws_bytes(sh, B));
  const int W_ = sh.width, NH = sh.n_hidden;
  hipError_t e = launch_train_init(sh, W, b, st, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, reinterpret_cast<float*>(amax), size_t(2 * NEDF_MAX_LAYERS));
  const int K0p = tl.L[0].Kpad;
  uint16_t* Hin = reinterpret_cast<uint16_t*>(fw);
  uint16_t* Hs = reinterpret_cast<uint16_t*>(fw + nedf_tl_align(size_t(B) * K0p * 2));
  float* mu = nullptr;
  hipLaunchKernelGGL(k_train_encode, dim3(blocks(B)), dim3(256), 0, s, o_l, d_l, static_cast<const float*>(nullptr),
                     static_cast<const uint8_t*>(nullptr), B, sh.in_kind, sh.enc_L, K0p, 1.0f, Hin, mu, mu);
  hipLaunchKernelGGL(k_amax16, dim3(256), dim3(256), 0, s, Hin, size_t(B) * K0p, amax + NEDF_MAX_LAYERS);
  for (int l = 0; l < NH; ++l) {
    GemmArgs g{};
    g.A = l == 0 ? Hin : Hs + size_t(l - 1) * B * W_;
    g.lda = l == 0 ? K0p : W_;
    g.B = reinterpret_cast<const uint16_t*>(st + tl.L[l].W16);
    g.ldb = tl.L[l].Kpad;
    g.M = B; g.N = W_; g.K = tl.L[l].Kpad;
    g.k_per_split = g.K;
    g.bias = reinterpret_cast<const float*>(st + tl.L[l].b);
    g.out16 = Hs + size_t(l) * B * W_;
    g.ldo = W_;
    gemm<0, 1, 0>(g, 1, s);
    if (l + 1 < NH) hipLaunchKernelGGL(k_amax16, dim3(256), dim3(256), 0, s, g.out16, size_t(B) * W_, amax + NEDF_MAX_LAYERS + l + 1);
    hipLaunchKernelGGL(k_amax32, dim3(64), dim3(256), 0, s, reinterpret_cast<const float*>(st + tl.L[l].W),
                       size_t(tl.L[l].N) * tl.L[l].K, amax + l);
  }
  hipLaunchKernelGGL(k_fp8_scales, dim3(1), dim3(64), 0, s, amax, amax + NEDF_MAX_LAYERS, NH, scales);
  return hipGetLastError();
}

size_t fp8_calibrate_ws_bytes(const nedf_mlp_shape& sh, int B) {
  return nedf_tl_align(nedf_train_layout_of(sh).total) + train_ws_bytes(sh, B) + 2 * NEDF_MAX_LAYERS * 4 + 256;
}

hipError_t launch_train_export(const nedf_mlp_shape& sh, const uint8_t* st, float* const* W, float* const* b,
                               bool grads, hipStream_t s) {
  const nedf_train_layout tl = nedf_train_layout_of(sh);
  for (int i = 0; i < tl.n_layers; ++i) {
    const nedf_train_layer& l = tl.L[i];
    const size_t ow = grads ? l.gW : l.W, ob = grads ? l.gb : l.b;
    hipError_t e = hipMemcpyAsync(W[i], st + ow, size_t(l.N) * l.K * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(b[i], st + ob, size_t(l.N) * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace nedf
