// Training of an intersection network (Eq. 6 in regression form, training
// details of the paper: Adam, lr 5e-4): input encoding and label conversion
// (inverse of Eq. 2), bfloat16 matrix-core GEMMs with fused epilogues for the
// forward pass, the ReLU-masked data gradients and split-K weight gradients,
// the head + loss kernel and Adam on float32 master weights.
#include <algorithm>
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
// mu* = (t_perp - D) / l and alpha = hit.  One thread per sample and group
// of 8 features (one 16-byte store; a sample's row is written by
// consecutive threads).
// N: input components (6 Pluecker, 3 xyz), a constant so that the feature
// index arithmetic divides by constants.
template <int N>
__global__ void k_train_encode(const float* o_l, const float* d_l, const float* depth, const uint8_t* hit,
                               int B, int L, int Kpad, float bound, uint16_t* H, float* mu, float* alpha) {
  const int groups = Kpad / 8;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = tid / groups, grp = tid % groups;
  if (s >= B) return;
  const float o[3] = {o_l[3 * s], o_l[3 * s + 1], o_l[3 * s + 2]};
  const float d[3] = {d_l[3 * s], d_l[3 * s + 1], d_l[3 * s + 2]};
  float p[6], plo[6] = {0, 0, 0, 0, 0, 0}, tperp = 0.0f;
  constexpr int n = N;
  if constexpr (N == 6) {
    line_of_local(o, d, p, plo, tperp);
  } else {
    float pl[6], pllo[6];
    line_of_local(o, d, pl, pllo, tperp);
    p[0] = o[0]; p[1] = o[1]; p[2] = o[2];
    p[3] = p[4] = p[5] = 0.0f;
  }
  uint32_t packed[4];
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    float v2[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int f = 8 * grp + e + u;
      float v = 0.0f;
      if (f < n) {
        v = p[f];
      } else if (f < n * (1 + 2 * L)) {
        const int q = f - n, level = q / (2 * n), w = q % (2 * n), c = w % n;
        v = sinpi_hw(float(1 << level) * p[c], float(1 << level) * plo[c], w >= n ? 1 : 0);
      }
      v2[u] = v;
    }
    packed[e / 2] = uint32_t(bf16_bits(v2[0])) | (uint32_t(bf16_bits(v2[1])) << 16);
  }
  *reinterpret_cast<uint4*>(H + size_t(s) * Kpad + 8 * grp) = make_uint4(packed[0], packed[1], packed[2], packed[3]);
  if (!depth || grp != 0) return;  // calibration: no labels
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
// C[M][N] = sum_k A(m, k) B(n, k) on 32x32x16 bf16 matrix cores with float32
// accumulation.  A workgroup computes a BM x BN tile (BM = 128 or 256, BN =
// 128 or 256) with one wave per (BM / 2) x 64 block (BM / 64 x 2 blocks of
// 32 x 32); K runs in stages of
// 64, staged in LDS as [row][k] (k contiguous; rows padded to 72 elements, so
// that the 16-byte fragment reads of a wave's 16-lane groups fall on distinct
// banks) and double-buffered.  Global loads run two stages ahead of the
// matrix cores (two register sets), so a stage's loads have two stages of
// multiplies to arrive in.  An operand is stored either k-contiguous (KC:
// X[row][k], copied 16 bytes at a time) or row-contiguous (RC: X[k][row],
// loaded as 8 x 8 blocks and transposed in registers by byte permutes on the
// way to LDS; only with BN = 128).  bfloat16 outputs go through LDS after the
// last stage and leave as whole 16-byte row pieces.  M is a multiple of BM,
// N of BN and K of 128 per split.
enum { KC = 0, RC = 1 };
constexpr int GT_BM = 128, GT_BK = 64, GT_LD = 72;  // rows per tile, K stage, LDS row stride (bf16)
// A stage row holds 8 chunks of 16 bytes.  LDS serves 16 lanes of a 16-byte
// access per cycle over 64 banks; a row is 36 words (9 groups of 4 banks)
// long, so the fragment reads (16 consecutive rows, one chunk: 9 j mod 16
// distinct) are conflict-free.  The transposed stores of a row-contiguous
// (RC) operand write rows 8 apart from 16 lanes (8 j mod 16: two groups, an
// 8-way conflict), so there chunk c of row r sits at position
// c ^ ((r / 16) % 8), which spreads them over 16 groups and keeps the reads
// conflict-free; k-contiguous operands keep the plain layout.
template <int LAYOUT>
__device__ __forceinline__ int stage_chunk(int row, int chunk) {
  return LAYOUT == RC ? chunk ^ ((row >> 4) & 7) : chunk;
}

struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  int M, N, K, lda, ldb;
  int k_per_split;
  // epilogue
  const float* bias;     // EPI 0: out16 = relu(acc + bias[col])
  const uint16_t* mask;  // EPI 1: out16 = acc * (mask[row][col] > 0), mask [M][ldm]
  int ldm;
  uint16_t* out16;       // EPI 0/1 [M][ldo]
  float* part;           // EPI 2: part[split][M][N] float32
  float* colsum;         //        colsum[split][M] (A is RC: sums over k of A(m, k))
  int ldo;
  // EPI 3: out32 = acc + bias[col] (float32 logits)
  // EPI 4: v = acc (+ resid32); out32 = v (if set); out16 = v * (mask > 0)
  //        (if set): the float32 gradient stream of a residual network
  // EPI 5: r = relu(acc + bias[col]); out16 = resid16 + r rounded once,
  //        out16b = r (a residual block's second layer)
  float* out32;
  const float* resid32;
  const uint16_t* resid16;
  uint16_t* out16b;
  // EPI 6 (last hidden layer of the regression form, N = 256 = width):
  // h = relu(acc + bias) rounded to bfloat16 (stored to out16 if set); the
  // head (mu_hat, z) = head_w h + head_b and the loss terms of Eq. 6 per
  // row; out16b = G = (g_mu head_w[0] + g_z head_w[1]) * (h > 0); part
  // [tile][HEAD_PART] = this tile's head weight and bias gradients and loss
  // sums
  const float* head_w;   // [2][256]
  const float* head_b;   // [2]
  const float* mu;       // [M] target mu (0 for misses)
  const float* alpha;    // [M] hit label
  float w_hit;
  // ReLU masks as bits, [M][ldo / 8] bytes, bit e of byte c of a row for
  // column 8 c + e: EPI 0 writes them for its output (if set), EPI 1 reads
  // them in place of the bfloat16 mask (if set)
  uint8_t* bits_out;
  const uint8_t* bits_in;
};
constexpr int HEAD_PART = 520;  // 512 weight grads, 2 bias grads, 3 loss terms (total, mse, bce)

// 8 x 8 transpose of bfloat16: v[j] holds 8 consecutive rows at k = j; w[r]
// gets the 8 values of row r in k order.
__device__ __forceinline__ void transpose8x8(const uint4 (&v)[8], uint4 (&w)[8]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t sel = (r & 1) ? 0x07060302u : 0x05040100u;
    uint32_t d[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const uint32_t lo = reinterpret_cast<const uint32_t*>(&v[2 * p])[r >> 1];
      const uint32_t hi = reinterpret_cast<const uint32_t*>(&v[2 * p + 1])[r >> 1];
      d[p] = __builtin_amdgcn_perm(hi, lo, sel);
    }
    w[r] = make_uint4(d[0], d[1], d[2], d[3]);
  }
}

// Register staging of one operand's stage (ROWS rows x 64 k) by NT threads.
template <int LAYOUT, int ROWS, int NT>
struct Stage;
// Staging registers are plain 4 x 32-bit vectors (not the HIP vector
// classes, which the compiler keeps in memory here).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int ROWS, int NT>
struct Stage<KC, ROWS, NT> {
  static constexpr int PER = ROWS * 8 / NT;  // 16-byte chunks per thread
  u32x4 v[PER];
  // chunk c = t + NT i: row c / 8, k 8 (c % 8)
  __device__ __forceinline__ void load(const uint16_t* X, int ld, int row0, int k0, int t, bool) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int c = t + NT * i;
      v[i] = *reinterpret_cast<const u32x4*>(X + size_t(row0 + (c >> 3)) * ld + k0 + 8 * (c & 7));
    }
  }
  __device__ __forceinline__ void store(uint16_t* S, int t, bool, float*) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int c = t + NT * i;
      *reinterpret_cast<u32x4*>(S + (c >> 3) * GT_LD + 8 * (c & 7)) = v[i];
    }
  }
};
template <int ROWS, int NT>
struct Stage<RC, ROWS, NT> {
  // block b of ROWS: rows 8 (b % (ROWS / 8)), k 8 (b / (ROWS / 8)); one
  // block per thread of the operand's half of the workgroup
  static constexpr int RB = ROWS / 8;
  uint4 v[8];
  __device__ __forceinline__ void load(const uint16_t* X, int ld, int row0, int k0, int b, bool mine) {
    if (!mine) return;
    const int rb = b % RB, kb = b / RB;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      v[j] = *reinterpret_cast<const uint4*>(X + size_t(k0 + 8 * kb + j) * ld + row0 + 8 * rb);
  }
  __device__ __forceinline__ void store(uint16_t* S, int b, bool mine, float* colsum8) const {
    if (!mine) return;
    const int rb = b % RB, kb = b / RB;
    uint4 w[8];
    transpose8x8(v, w);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      *reinterpret_cast<uint4*>(S + (8 * rb + r) * GT_LD + 8 * stage_chunk<RC>(8 * rb + r, kb)) = w[r];
      if (colsum8) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(&w[r]);
        float s = 0.f;
#pragma unroll
        for (int e = 0; e < 4; ++e) s += __uint_as_float(q[e] << 16) + __uint_as_float(q[e] & 0xFFFF0000u);
        colsum8[r] += s;
      }
    }
  }
};

// Head and loss of the regression form from the bfloat16 tile h [128][LO]
// of the last hidden layer in LDS (all 256 features of 128 rows), followed
// in LDS by the head weights (float [2][256]).  Four threads per row form
// the two head outputs (a fixed pairing of their partial sums); the row's
// loss terms (Eq. 6: alpha (mu_hat - mu)^2 and the logistic loss of the
// hit logit) and gradients g = dLoss/d(mu_hat, z) go to LDS; then the
// gradient G of the tile, the tile's head weight gradients (rows summed in
// order) and its bias and loss sums.
// Head weights in LDS: weight k (0..511, row-major [2][256]) at
// k + 4 (k / 64), so that reads 64 weights apart fall on different banks and
// groups of 4 stay 16-byte aligned.
__device__ __forceinline__ int head_w_slot(int k) { return k + 4 * (k >> 6); }
constexpr int HEAD_W_SLOTS = 544;  // 512 + 8 pads of 4
__device__ __forceinline__ float4 head_w4(const float* sW, int k) {  // weights k .. k + 3, k a multiple of 4
  return *reinterpret_cast<const float4*>(sW + head_w_slot(k));
}

template <int NT, int LO>
__device__ __forceinline__ void head_loss_epilogue(const GemmArgs& g, uint16_t* lds, int m0, int tile, int t,
                                                   float mu_r, float alpha_r) {
  static_assert(NT == 512, "four threads per row of a 128-row tile, two per head weight");
  const float* sW = reinterpret_cast<const float*>(lds + GT_BM * LO);
  float* sg = const_cast<float*>(sW) + HEAD_W_SLOTS;  // [2][128]
  float* sred = sg + 256;                    // [2][128]
  const float invB = 1.0f / float(g.M);
  {
    // wave w takes rows 16 w .. 16 w + 15; a row's four threads (quarters p
    // of its 256 features) are 16 lanes apart, so that the 8 lanes of an LDS
    // cycle read 8 different rows (distinct banks)
    const int r = 16 * (t >> 6) + (t & 15), p = (t >> 4) & 3;
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int k = 64 * p + 8 * m;
      const uint4 q = *reinterpret_cast<const uint4*>(lds + r * LO + k);
      const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
      const float4 u0 = head_w4(sW, k), u1 = head_w4(sW, k + 4);
      const float4 v0 = head_w4(sW, 256 + k), v1 = head_w4(sW, 256 + k + 4);
      const float wa[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
      const float wb[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float h0 = __uint_as_float(w4[e] << 16), h1 = __uint_as_float(w4[e] & 0xFFFF0000u);
        a0 = fmaf(wa[2 * e], h0, a0);
        a1 = fmaf(wb[2 * e], h0, a1);
        a0 = fmaf(wa[2 * e + 1], h1, a0);
        a1 = fmaf(wb[2 * e + 1], h1, a1);
      }
    }
    // (p0 + p1) + (p2 + p3)
    a0 += __shfl_xor(a0, 16);
    a1 += __shfl_xor(a1, 16);
    a0 += __shfl_xor(a0, 32);
    a1 += __shfl_xor(a1, 32);
    if (p == 0) {
      a0 += g.head_b[0];
      a1 += g.head_b[1];
      const float al = alpha_r, e = a0 - mu_r;  // labels of row r, loaded before the K loop
      sred[r] = al * e * e;
      sred[128 + r] = fmaxf(a1, 0.f) + log1pf(expf(-fabsf(a1))) - al * a1;
      sg[r] = 2.0f * al * e * invB;
      sg[128 + r] = g.w_hit * (1.0f / (1.0f + expf(-a1)) - al) * invB;
    }
  }
  __syncthreads();
  // G = (g_mu W_0 + g_z W_1) * (h > 0), 16-byte row pieces
#pragma unroll
  for (int i = 0; i < GT_BM * 256 / 8 / NT; ++i) {
    const int c = t + NT * i;
    const int r = c >> 5, c8 = 8 * (c & 31);
    const uint4 q = *reinterpret_cast<const uint4*>(lds + r * LO + c8);
    const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
    const float g0 = sg[r], g1 = sg[128 + r];
    const float4 u0 = head_w4(sW, c8), u1 = head_w4(sW, c8 + 4);
    const float4 z0 = head_w4(sW, 256 + c8), z1 = head_w4(sW, 256 + c8 + 4);
    const float wa[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
    const float wb[8] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w};
    uint32_t o4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float h0 = __uint_as_float(w4[e] << 16), h1 = __uint_as_float(w4[e] & 0xFFFF0000u);
      const float v0 = h0 > 0.f ? fmaf(g0, wa[2 * e], g1 * wb[2 * e]) : 0.f;
      const float v1 = h1 > 0.f ? fmaf(g0, wa[2 * e + 1], g1 * wb[2 * e + 1]) : 0.f;
      o4[e] = uint32_t(bf16_bits(v0)) | (uint32_t(bf16_bits(v1)) << 16);
    }
    *reinterpret_cast<uint4*>(g.out16b + size_t(m0 + r) * g.ldo + c8) = make_uint4(o4[0], o4[1], o4[2], o4[3]);
  }
  // head weight gradients of the tile: thread (row group rg, features
  // 8 kq .. 8 kq + 7) sums g_j h_k over its 8 rows in order; the 16 row
  // groups' partials (LDS after the head data) are then added in order
  float* P = g.part + size_t(tile) * HEAD_PART;
  {
    float* red = sred + 256;  // [16][512]
    static_assert(GT_BM * LO * 2 + (HEAD_W_SLOTS + 512 + 16 * 512) * 4 <= 2 * (GT_BM + 256) * GT_LD * 2,
                  "head partials fit the stage buffers");
    const int kq = t & 31, rg = t >> 5;
    float a0[8], a1[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) a0[e] = a1[e] = 0.f;
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
      const int r = 8 * rg + rr;
      const uint4 q = *reinterpret_cast<const uint4*>(lds + r * LO + 8 * kq);
      const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
      const float g0 = sg[r], g1 = sg[128 + r];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float h0 = __uint_as_float(w4[e] << 16), h1 = __uint_as_float(w4[e] & 0xFFFF0000u);
        a0[2 * e] = fmaf(g0, h0, a0[2 * e]);
        a1[2 * e] = fmaf(g1, h0, a1[2 * e]);
        a0[2 * e + 1] = fmaf(g0, h1, a0[2 * e + 1]);
        a1[2 * e + 1] = fmaf(g1, h1, a1[2 * e + 1]);
      }
    }
    float* dst = red + 512 * rg + 8 * kq;
    *reinterpret_cast<float4*>(dst) = make_float4(a0[0], a0[1], a0[2], a0[3]);
    *reinterpret_cast<float4*>(dst + 4) = make_float4(a0[4], a0[5], a0[6], a0[7]);
    *reinterpret_cast<float4*>(dst + 256) = make_float4(a1[0], a1[1], a1[2], a1[3]);
    *reinterpret_cast<float4*>(dst + 260) = make_float4(a1[4], a1[5], a1[6], a1[7]);
    __syncthreads();
    float acc = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += red[512 * q + t];
    P[t] = acc;  // t = 256 j + k
  }
  // bias gradients and loss sums of the tile (one wave: lane l adds rows l
  // and l + 64, then a fixed butterfly)
  if (t < 64) {
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float* src = q < 2 ? sg + 128 * q : sred + 128 * (q - 2);
      v[q] = src[t] + src[t + 64];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off);
    }
    if (t == 0) {
      P[512] = v[0];
      P[513] = v[1];
      P[514] = (v[2] + g.w_hit * v[3]) * invB;
      P[515] = v[2] * invB;
      P[516] = v[3] * invB;
    }
  }
}

// One output tile (bx, by) of split bz, BM rows (128, or 256 for
// k-contiguous operands: half the re-reads of the B operand from L2 and
// six fragment reads per eight matrix ops instead of four per four).
template <int AL, int BL, int EPI, bool COLSUM, int BN, int BM>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, const int bx, const int by, const int bz) {
  constexpr int NT = BN * 2;            // threads: 2 x (BN / 64) waves
  constexpr int WN = BN / 64;           // waves along N
  constexpr int MI = BM / 64;           // 32-row blocks per wave (a wave takes BM / 2 rows)
  constexpr int SA = BM * GT_LD, SB = BN * GT_LD;
  static_assert(AL == KC || BN == 128, "row-contiguous operands need BN = 128");
  static_assert(BL == KC || BN == 128, "row-contiguous operands need BN = 128");
  static_assert(BM == GT_BM || (BM == 256 && AL == KC && BL == KC && !COLSUM && (EPI == 0 || EPI == 1)),
                "256-row tiles: k-contiguous operands, bias/ReLU or bit-mask epilogues");
  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * (SA + SB)];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int m0 = bx * BM, n0 = by * BN;
  const int kb = bz * g.k_per_split;
  const int ke = min(g.K, kb + g.k_per_split);
  const int n_stages = (ke - kb) / GT_BK;
  // epilogue inputs loaded before the K loop, which hides their latency:
  // the masks of this thread's output pieces (EPI 1; loaded in the store
  // loop they would wait one by one behind the stores, which the compiler
  // may not move them past), and the head weights plus this thread's row
  // labels (EPI 6)
  constexpr int PIECES = BM * BN / 8 / NT;
  uint32_t pre_bits[EPI == 1 ? PIECES : 1];
  uint4 pre_mask[EPI == 1 && BM == GT_BM ? PIECES : 1];  // 256-row tiles take bit masks only
  if constexpr (EPI == 1) {
#pragma unroll
    for (int i = 0; i < PIECES; ++i) {
      const int c = t + NT * i;
      const int r = c / (BN / 8), c8 = 8 * (c % (BN / 8));
      if (g.bits_in) pre_bits[i] = g.bits_in[size_t(m0 + r) * (g.ldm / 8) + (n0 + c8) / 8];
      else if constexpr (BM == GT_BM) pre_mask[i] = *reinterpret_cast<const uint4*>(g.mask + size_t(m0 + r) * g.ldm + n0 + c8);
    }
  }
  float pre_w = 0.f, pre_mu = 0.f, pre_al = 0.f;
  if constexpr (EPI == 6) {
    static_assert(NT == 512, "one head weight per thread");
    pre_w = g.head_w[t];
    const int r = 16 * (t >> 6) + (t & 15);  // the row whose labels this thread uses in the head epilogue
    pre_mu = g.mu[m0 + r];
    pre_al = g.alpha[m0 + r];
  }
  // row-contiguous operands: A's blocks by threads 0..127, B's by 128..255
  const int rc = t & 127;
  const bool a_mine = AL == KC || t < 128;
  const bool b_mine = BL == KC || (AL == RC ? t >= 128 : t < 128);
  const int ta = AL == KC ? t : rc, tb = BL == KC ? t : rc;
  // two register sets, named (not indexed) so that they stay in registers
  Stage<AL, BM, NT> ra0, ra1;
  Stage<BL, BN, NT> rb0, rb1;
  float cs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  f32x16_t acc[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x16_t{};
  if (n_stages <= 0) return;  // never launched so (K a multiple of 64 per split)
  ra0.load(g.A, g.lda, m0, kb, ta, a_mine);
  rb0.load(g.B, g.ldb, n0, kb, tb, b_mine);
  {
    const int k1 = kb + min(1, n_stages - 1) * GT_BK;
    ra1.load(g.A, g.lda, m0, k1, ta, a_mine);
    rb1.load(g.B, g.ldb, n0, k1, tb, b_mine);
  }
  if (n_stages > 0) {
    ra0.store(lds, ta, a_mine, COLSUM ? cs : nullptr);
    rb0.store(lds + SA, tb, b_mine, nullptr);
  }
  __syncthreads();
  // one stage: multiply LDS buffer BUF; register set CUR (stage s, then
  // free) takes stage s + 2; set NXT (stage s + 1) goes to buffer BUF ^ 1.
  // Written out for each parity (a macro, not a function), so that both
  // register sets stay named registers.
#define NEDF_GEMM_STAGE(S_, BUF, RA_CUR, RB_CUR, RA_NXT, RB_NXT)                                           \
  {                                                                                                       \
    {                                                                                                     \
      /* unconditional (the last stage again past the end): a conditional */                            \
      /* load would keep the register set in memory */                                                    \
      const int kl = kb + min((S_) + 2, n_stages - 1) * GT_BK;                                            \
      RA_CUR.load(g.A, g.lda, m0, kl, ta, a_mine);                                                        \
      RB_CUR.load(g.B, g.ldb, n0, kl, tb, b_mine);                                                        \
    }                                                                                                     \
    const uint16_t* A_ = lds + (BUF) * (SA + SB) + (wm * (BM / 2) + (lane & 31)) * GT_LD;                  \
    const uint16_t* B_ = lds + (BUF) * (SA + SB) + SA + (wn * 64 + (lane & 31)) * GT_LD;                   \
    _Pragma("unroll") for (int ks = 0; ks < GT_BK / 16; ++ks) {                                           \
      bf16x8_t a[MI], b[2];                                                                               \
      /* row 64 w + 32 i + lane % 32 (RC: 128-row tiles): (row / 16) % 8 = (4 w + 2 i + bit 4 of lane) % 8 */ \
      const int c_ = 2 * ks + (lane >> 5), l4 = (lane >> 4) & 1;                                          \
      _Pragma("unroll") for (int i = 0; i < MI; ++i) {                                                    \
        const int ca = AL == RC ? c_ ^ ((4 * wm + 2 * i + l4) & 7) : c_;                                  \
        a[i] = *reinterpret_cast<const bf16x8_t*>(A_ + 32 * i * GT_LD + 8 * ca);                          \
      }                                                                                                   \
      _Pragma("unroll") for (int i = 0; i < 2; ++i) {                                                     \
        const int cb = BL == RC ? c_ ^ ((4 * wn + 2 * i + l4) & 7) : c_;                                  \
        b[i] = *reinterpret_cast<const bf16x8_t*>(B_ + 32 * i * GT_LD + 8 * cb);                          \
      }                                                                                                   \
      _Pragma("unroll") for (int i = 0; i < MI; ++i)                                                      \
      _Pragma("unroll") for (int j = 0; j < 2; ++j)                                                       \
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[j], a[i], acc[i][j], 0, 0, 0);              \
    }                                                                                                     \
    if ((S_) + 1 < n_stages) {                                                                            \
      RA_NXT.store(lds + ((BUF) ^ 1) * (SA + SB), ta, a_mine, COLSUM ? cs : nullptr);                     \
      RB_NXT.store(lds + ((BUF) ^ 1) * (SA + SB) + SA, tb, b_mine, nullptr);                              \
    }                                                                                                     \
    __syncthreads();                                                                                      \
  }
  // operands swapped in the matrix-core call (B tile first): the accumulators
  // of lane l then hold row m = l % 32 of the block and, per group of four
  // registers, four consecutive columns
  // the stage count is even (K a multiple of 128 per split), so both copies
  // run every iteration
#pragma unroll 1
  for (int s = 0; s < n_stages; s += 2) {
    NEDF_GEMM_STAGE(s, 0, ra0, rb0, ra1, rb1)
    NEDF_GEMM_STAGE(s + 1, 1, ra1, rb1, ra0, rb0)
  }
#undef NEDF_GEMM_STAGE
  // accumulator r of block (i, j): row 64 wm + 32 i + lane % 32, column
  // 64 wn + 32 j + 8 (r / 4) + 4 (lane / 32) + r % 4 of the tile
  static_assert(EPI >= 0 && EPI <= 6, "unknown epilogue");
  if constexpr (EPI >= 3 && EPI <= 5) {
    // straight from the accumulators: four consecutive columns per store.
    // Per accumulator row block, every input of its 8 column groups is
    // loaded first: a load placed after a store would wait for it (the
    // compiler may not move a load past a store to memory that can alias).
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      const int row = m0 + wm * (BM / 2) + 32 * i + (lane & 31);
      float4 in4[2][4];  // bias (EPI 3, 5) or the float32 stream (EPI 4)
      uint2 in2[2][4];   // the bfloat16 mask (EPI 4) or the residual input (EPI 5)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int col = n0 + wn * 64 + 32 * j + 8 * q + 4 * (lane >> 5);
          const size_t o = size_t(row) * g.ldo + col;
          if constexpr (EPI == 3 || EPI == 5) in4[j][q] = *reinterpret_cast<const float4*>(g.bias + col);
          if constexpr (EPI == 4) {
            in4[j][q] = g.resid32 ? *reinterpret_cast<const float4*>(g.resid32 + o) : make_float4(0.f, 0.f, 0.f, 0.f);
            in2[j][q] = g.out16 ? *reinterpret_cast<const uint2*>(g.mask + size_t(row) * g.ldm + col) : make_uint2(0u, 0u);
          }
          if constexpr (EPI == 5) in2[j][q] = *reinterpret_cast<const uint2*>(g.resid16 + o);
        }
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int col = n0 + wn * 64 + 32 * j + 8 * q + 4 * (lane >> 5);
          const size_t o = size_t(row) * g.ldo + col;
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = acc[i][j][4 * q + e];
          if constexpr (EPI == 3) {
            const float4 bb = in4[j][q];
            *reinterpret_cast<float4*>(g.out32 + o) = make_float4(v[0] + bb.x, v[1] + bb.y, v[2] + bb.z, v[3] + bb.w);
          } else if constexpr (EPI == 4) {
            if (g.resid32) {
              const float4 r = in4[j][q];
              v[0] += r.x; v[1] += r.y; v[2] += r.z; v[3] += r.w;
            }
            if (g.out32) *reinterpret_cast<float4*>(g.out32 + o) = make_float4(v[0], v[1], v[2], v[3]);
            if (g.out16) {
              const uint2 mk = in2[j][q];
              const float m0v = __uint_as_float(mk.x << 16), m1v = __uint_as_float(mk.x & 0xFFFF0000u);
              const float m2v = __uint_as_float(mk.y << 16), m3v = __uint_as_float(mk.y & 0xFFFF0000u);
              *reinterpret_cast<uint2*>(g.out16 + o) =
                  make_uint2(uint32_t(bf16_bits(m0v > 0.f ? v[0] : 0.f)) | (uint32_t(bf16_bits(m1v > 0.f ? v[1] : 0.f)) << 16),
                             uint32_t(bf16_bits(m2v > 0.f ? v[2] : 0.f)) | (uint32_t(bf16_bits(m3v > 0.f ? v[3] : 0.f)) << 16));
            }
          } else {  // EPI 5
            static_assert(EPI == 5, "residual epilogue");
            const float4 bb = in4[j][q];
            const float r0 = fmaxf(v[0] + bb.x, 0.f), r1 = fmaxf(v[1] + bb.y, 0.f);
            const float r2 = fmaxf(v[2] + bb.z, 0.f), r3 = fmaxf(v[3] + bb.w, 0.f);
            const uint2 h = in2[j][q];
            const float h0 = __uint_as_float(h.x << 16), h1 = __uint_as_float(h.x & 0xFFFF0000u);
            const float h2 = __uint_as_float(h.y << 16), h3 = __uint_as_float(h.y & 0xFFFF0000u);
            *reinterpret_cast<uint2*>(g.out16 + o) =
                make_uint2(uint32_t(bf16_bits(h0 + r0)) | (uint32_t(bf16_bits(h1 + r1)) << 16),
                           uint32_t(bf16_bits(h2 + r2)) | (uint32_t(bf16_bits(h3 + r3)) << 16));
            *reinterpret_cast<uint2*>(g.out16b + o) =
                make_uint2(uint32_t(bf16_bits(r0)) | (uint32_t(bf16_bits(r1)) << 16),
                           uint32_t(bf16_bits(r2)) | (uint32_t(bf16_bits(r3)) << 16));
          }
        }
    }
  } else if constexpr (EPI == 2) {
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      const int row = m0 + wm * (BM / 2) + 32 * i + (lane & 31);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int col = n0 + wn * 64 + 32 * j + 8 * q + 4 * (lane >> 5);
          *reinterpret_cast<float4*>(g.part + (size_t(bz) * g.M + row) * g.N + col) =
              make_float4(acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]);
        }
    }
  } else {
    // EPI 0, 1, 6: bfloat16 tile in LDS ([128][BN + 8]), then 16-byte row pieces
    static_assert(EPI == 0 || EPI == 1 || EPI == 6, "tile epilogues");
    constexpr int LO = BN + 8;
    static_assert(BM * LO <= 2 * (SA + SB), "output tile must fit the stage buffers");
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      const int r = wm * (BM / 2) + 32 * i + (lane & 31);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = wn * 64 + 32 * j + 8 * q + 4 * (lane >> 5);
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = acc[i][j][4 * q + e];
          if constexpr (EPI == 0 || EPI == 6) {
            const float4 bb = *reinterpret_cast<const float4*>(g.bias + n0 + c);
            v[0] = fmaxf(v[0] + bb.x, 0.f); v[1] = fmaxf(v[1] + bb.y, 0.f);
            v[2] = fmaxf(v[2] + bb.z, 0.f); v[3] = fmaxf(v[3] + bb.w, 0.f);
          }
          *reinterpret_cast<uint2*>(lds + r * LO + c) =
              make_uint2(uint32_t(bf16_bits(v[0])) | (uint32_t(bf16_bits(v[1])) << 16),
                         uint32_t(bf16_bits(v[2])) | (uint32_t(bf16_bits(v[3])) << 16));
        }
    }
    if constexpr (EPI == 6) {
      float* sW = reinterpret_cast<float*>(lds + BM * LO);
      sW[head_w_slot(t)] = pre_w;
    }
    __syncthreads();
    constexpr int CH = BM * BN / 8;  // 16-byte pieces of the tile
    static_assert(EPI != 6 || BN == 256, "head epilogue: whole rows in one tile");
    if (EPI != 6 || g.out16) {
#pragma unroll
    for (int i = 0; i < CH / NT; ++i) {
      const int c = t + NT * i;
      const int r = c / (BN / 8), c8 = 8 * (c % (BN / 8));
      uint4 v = *reinterpret_cast<const uint4*>(lds + r * LO + c8);
      if constexpr (EPI == 1) {
        uint32_t vw[4] = {v.x, v.y, v.z, v.w};
        if (g.bits_in) {
          const uint32_t mb = pre_bits[i];
#pragma unroll
          for (int e = 0; e < 4; ++e)
            vw[e] &= ((mb >> (2 * e)) & 1u ? 0x0000FFFFu : 0u) | ((mb >> (2 * e + 1)) & 1u ? 0xFFFF0000u : 0u);
        } else if constexpr (BM == GT_BM) {
          const uint4 mk = pre_mask[i];
          const uint32_t mw[4] = {mk.x, mk.y, mk.z, mk.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t lo = __uint_as_float(mw[e] << 16) > 0.f ? 0x0000FFFFu : 0u;
            const uint32_t hi = __uint_as_float(mw[e] & 0xFFFF0000u) > 0.f ? 0xFFFF0000u : 0u;
            vw[e] &= lo | hi;
          }
        }
        v = make_uint4(vw[0], vw[1], vw[2], vw[3]);
      }
      if constexpr (EPI == 0) {
        if (g.bits_out) {
          const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
          uint32_t mb = 0;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            mb |= (__uint_as_float(vw[e] << 16) > 0.f ? 1u : 0u) << (2 * e) |
                  (__uint_as_float(vw[e] & 0xFFFF0000u) > 0.f ? 1u : 0u) << (2 * e + 1);
          g.bits_out[size_t(m0 + r) * (g.ldo / 8) + (n0 + c8) / 8] = uint8_t(mb);
        }
      }
      *reinterpret_cast<uint4*>(g.out16 + size_t(m0 + r) * g.ldo + n0 + c8) = v;
    }
    }
    if constexpr (EPI == 6) head_loss_epilogue<NT, LO>(g, lds, m0, bx, t, pre_mu, pre_al);
  }
  if constexpr (COLSUM) {
    // column sums of A over this split's k, one set per m tile (written by
    // the workgroups of the first n tile): the 8 threads of one row block
    // (k blocks 0..7) combine in a fixed order
    __shared__ float s_cs[128][8];
    if (t < 128) {
#pragma unroll
      for (int r = 0; r < 8; ++r) s_cs[8 * (rc % 16) + r][rc / 16] = cs[r];
    }
    __syncthreads();
    if (by == 0 && t < 128) {
      float s_ = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) s_ += s_cs[t][q];
      g.colsum[size_t(bz) * g.M + m0 + t] = s_;
    }
  }
}

template <int AL, int BL, int EPI, bool COLSUM, int BN, int BM>
__global__ __launch_bounds__(BN * 2) void k_gemm(GemmArgs g) {
  gemm_tile<AL, BL, EPI, COLSUM, BN, BM>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Weight gradients of several layers in one launch: dW_p = G_p^T X_p over S
// batch splits, with the column sums of G_p (bias gradients).  Both operands
// are stored [batch][features] (row-contiguous in the product's terms);
// M = width for every problem.  blockIdx.z = problem * S + split; the
// workgroups of a problem's n tiles beyond its own N leave at once.  Two
// workgroups of four waves share a compute unit (registers and LDS fit), so
// a launch of more than one workgroup per compute unit keeps the matrix
// cores busy while the other workgroup stages.
struct WgradProb {
  const uint16_t* G;  // [B][M]
  const uint16_t* X;  // [B][ldx], N = padded input width
  float* part;        // [S][M][N]
  float* colsum;      // [S][M]
  int ldx, N;
};
struct WgradBatch {
  WgradProb p[NEDF_TRAIN_MAX_LAYERS];
  int n, S, M, B;
};
__global__ __launch_bounds__(256, 2) void k_wgrad(WgradBatch wb) {
  // The tiles of one (problem, split) read the same rows of both operands.
  // Workgroups are handed to the 8 XCDs (each with its own L2) round-robin
  // by linear id, so logical workgroup l = (id % 8) * (total / 8) + id / 8
  // (a bijection when total is a multiple of 8) puts consecutive logical
  // ids, and with them a slice's tiles, on one XCD: the second read of each
  // operand row is an L2 hit instead of an HBM read.
  const int nx = gridDim.x, ny = gridDim.y;
  const int total = nx * ny * int(gridDim.z);
  const int id = int(blockIdx.x) + nx * (int(blockIdx.y) + ny * int(blockIdx.z));
  const int lid = total % 8 == 0 ? (id % 8) * (total / 8) + id / 8 : id;
  const int bx = lid % nx, by = (lid / nx) % ny, bz = lid / (nx * ny);
  const int prob = bz / wb.S, split = bz % wb.S;
  const WgradProb& p = wb.p[prob];
  if (by * 128 >= p.N) return;  // the whole workgroup
  GemmArgs g{};
  g.A = p.G; g.lda = wb.M;
  g.B = p.X; g.ldb = p.ldx;
  g.M = wb.M; g.N = p.N; g.K = wb.B;
  g.k_per_split = wb.B / wb.S;
  g.part = p.part;
  g.colsum = p.colsum;
  gemm_tile<RC, RC, 2, true, 128, GT_BM>(g, bx, by, split);
}

template <int AL, int BL, int EPI, bool COLSUM = false, int BN = 256, int BM = GT_BM>
void gemm(const GemmArgs& g, int splits, hipStream_t s) {
  dim3 grid(g.M / BM, g.N / BN, splits);
  hipLaunchKernelGGL((k_gemm<AL, BL, EPI, COLSUM, BN, BM>), grid, dim3(BN * 2), 0, s, g);
}

// Weight and bias gradients of every hidden layer from the split partials,
// summed over the splits in order (deterministic): gW[m][k] for k < K, gb[m].
// With head partials (regression form), the slice blockIdx.y = n_layers
// sums them too: one wave per output (512 head weight gradients, 2 bias
// gradients, 3 loss terms), lane l adding tiles l, l + 64, ... in order, then
// a fixed butterfly.  The first thread also counts the update in the Adam
// step counter, which the Adam launch after this one reads.
struct ReduceLayer {
  const float* part;   // [S][M][N]
  const float* csum;   // [S][M]
  float* gW;           // [M][K]
  float* gb;           // [M]
  int M, N, K;
};
struct ReduceArgs {
  ReduceLayer L[NEDF_TRAIN_MAX_LAYERS];
  int n_layers, S;
  int64_t* step;
  const float* hpart;  // [h_blocks][HEAD_PART] or null
  int h_blocks;
  float *gWh, *gbh, *loss;
};
__global__ void k_reduce_grads(ReduceArgs r) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *r.step += 1;
  if (int(blockIdx.y) == r.n_layers) {
    const int j = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= 517) return;
    float s = 0.f;
    for (int q = lane; q < r.h_blocks; q += 64) s += r.hpart[size_t(q) * HEAD_PART + j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane != 0) return;
    if (j < 512) r.gWh[j] = s;
    else if (j < 514) r.gbh[j - 512] = s;
    else r.loss[j - 514] = s;
    return;
  }
  const ReduceLayer& L = r.L[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int MN = L.M * L.N;
  if (i < MN) {
    const int m = i / L.N, n = i % L.N;
    if (n < L.K) {
      float s = 0.f;
      for (int q = 0; q < r.S; ++q) s += L.part[size_t(q) * MN + i];
      L.gW[size_t(m) * L.K + n] = s;
    }
  } else if (i < MN + L.M) {
    const int m = i - MN;
    float s = 0.f;
    for (int q = 0; q < r.S; ++q) s += L.csum[size_t(q) * L.M + m];
    L.gb[m] = s;
  }
}

__global__ void k_zero_f32(float* p, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// Adam (Kingma & Ba 2015) with bias correction, step t = *step (counted by
// the gradient reduction just before), over every
// parameter array of the network in one launch (segments listed in AdamArgs;
// a block never spans two segments); the bfloat16 copy of weight matrices is
// refreshed in the same pass.
struct AdamSeg {
  float *p, *m, *v;
  const float* g;
  uint16_t* w16;  // or null: [N][Kpad] copy
  uint16_t* w16t; // or null: [Kpad][N] copy
  int n, K, Kpad, N;
  int block0;     // first block of this segment
};
struct AdamArgs {
  AdamSeg seg[2 * (NEDF_MAX_LAYERS + 1)];
  int n_seg;
  const int64_t* step;
  float lr, b1, b2, eps;
};
__global__ void k_adam(AdamArgs a) {
  int si = 0;
  while (si + 1 < a.n_seg && int(blockIdx.x) >= a.seg[si + 1].block0) ++si;
  const AdamSeg& S = a.seg[si];
  const int i = (int(blockIdx.x) - S.block0) * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const float t = float(*a.step);
  const float bc1 = 1.0f - powf(a.b1, t), bc2 = 1.0f - powf(a.b2, t);
  const float gi = S.g[i];
  const float mi = a.b1 * S.m[i] + (1.0f - a.b1) * gi;
  const float vi = a.b2 * S.v[i] + (1.0f - a.b2) * gi * gi;
  S.m[i] = mi;
  S.v[i] = vi;
  const float pi = S.p[i] - a.lr * (mi / bc1) / (sqrtf(vi / bc2) + a.eps);
  S.p[i] = pi;
  if (S.w16) S.w16[size_t(i / S.K) * S.Kpad + (i % S.K)] = bf16_bits(pi);
  if (S.w16t) S.w16t[size_t(i % S.K) * S.N + (i / S.K)] = bf16_bits(pi);
}

// Initial state: master weights from float32 arrays, moments and gradients
// zero, bfloat16 copies (zero padded).
__global__ void k_copy_w(const float* src, float* dst, uint16_t* w16, uint16_t* w16t, int N, int K, int Kpad,
                         int Nsrc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * Kpad) return;
  const int r = i / Kpad, c = i % Kpad;
  const float v = (c < K && r < Nsrc) ? src[r * K + c] : 0.0f;
  if (c < K && dst) dst[r * K + c] = v;
  if (w16) w16[i] = bf16_bits(v);
  if (w16t) w16t[size_t(c) * N + r] = bf16_bits(v);
}

unsigned blocks(size_t n, int b = 256) { return unsigned((n + b - 1) / b); }

void launch_train_encode(const nedf_mlp_shape& sh, const float* o_l, const float* d_l, const float* depth,
                         const uint8_t* hit, int B, int K0p, float bound, uint16_t* H, float* mu, float* alpha,
                         hipStream_t s) {
  const dim3 grid(blocks(size_t(B) * (K0p / 8)));
  if (sh.in_kind == NEDF_IN_PLUECKER)
    hipLaunchKernelGGL(k_train_encode<6>, grid, dim3(256), 0, s, o_l, d_l, depth, hit, B, sh.enc_L, K0p, bound, H,
                       mu, alpha);
  else
    hipLaunchKernelGGL(k_train_encode<3>, grid, dim3(256), 0, s, o_l, d_l, depth, hit, B, sh.enc_L, K0p, bound, H,
                       mu, alpha);
}

// ---- classifier-form network (NEDF_IN_POINTS16) ---------------------------------
// Encoded input of the 16 line points (natural order: point-major, each
// [x, sin(2^0 pi x), cos(2^0 pi x), ...], 63 values) zero padded to Kpad, and
// labels mu* = (t_perp - D) / l, alpha = hit.  The points come from the
// compensated frame of the inference kernel, applied to the local ray.
template <int L>
__global__ void k_train_encode_points(const float* o_l, const float* d_l, const float* depth, const uint8_t* hit,
                                      int B, int Kpad, float bound, uint16_t* H, float* mu, float* alpha) {
  constexpr int per = 3 * (1 + 2 * L);  // features per point
  const int groups = Kpad / 8;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = tid / groups, grp = tid % groups;
  if (s >= B) return;
  const float o[3] = {o_l[3 * s], o_l[3 * s + 1], o_l[3 * s + 2]};
  const float d[3] = {d_l[3 * s], d_l[3 * s + 1], d_l[3 * s + 2]};
  const float zero[3] = {0.f, 0.f, 0.f};
  W2L id{};
  id.rt[0] = id.rt[4] = id.rt[8] = 1.0f;
  id.s = id.inv_s = 1.0f;
  f2 q[3], dv[3];
  float tperp, ol[3];
  local_points_frame(id, o, d, zero, bound, q, dv, tperp, ol);
  // point p of the line (compensated: value and low part), for the at most
  // two points this thread's 8 features belong to
  auto point = [&](int p, float (&x)[3], float (&xlo)[3]) {
    const float cp = float(2 * p + 1) * 0.0625f - 1.0f;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma clang fp contract(off)
      const f2 pp = two_prod(cp, dv[r].hi);
      const f2 sm = two_sum(q[r].hi, pp.hi);
      x[r] = sm.hi;
      xlo[r] = sm.lo + ((pp.lo + q[r].lo) + cp * dv[r].lo);
    }
  };
  const int pa = (8 * grp) / per;
  float xa[3], xla[3], xb[3], xlb[3];
  point(pa, xa, xla);
  point(pa + 1, xb, xlb);
  uint32_t packed[4];
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    float v2[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int f = 8 * grp + e + u;
      float v = 0.0f;
      if (f < NEDF_CLS_POINTS * per) {
        const bool second = f >= (pa + 1) * per;
        const int e2 = f - (second ? pa + 1 : pa) * per;
        float x[3], xlo[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          x[r] = second ? xb[r] : xa[r];
          xlo[r] = second ? xlb[r] : xla[r];
        }
        if (e2 < 3) {
          v = e2 == 0 ? x[0] : e2 == 1 ? x[1] : x[2];
        } else {
          const int qq = e2 - 3, level = qq / 6, w = qq % 6, c = w % 3;
          const float xc = c == 0 ? x[0] : c == 1 ? x[1] : x[2];
          const float xlc = c == 0 ? xlo[0] : c == 1 ? xlo[1] : xlo[2];
          v = sinpi_hw(float(1 << level) * xc, float(1 << level) * xlc, w >= 3 ? 1 : 0);
        }
      }
      v2[u] = v;
    }
    packed[e / 2] = uint32_t(bf16_bits(v2[0])) | (uint32_t(bf16_bits(v2[1])) << 16);
  }
  *reinterpret_cast<uint4*>(H + size_t(s) * Kpad + 8 * grp) = make_uint4(packed[0], packed[1], packed[2], packed[3]);
  if (grp != 0) return;
  const bool h = hit[s] != 0;
  alpha[s] = h ? 1.0f : 0.0f;
  mu[s] = h ? (tperp - depth[s]) / bound : 0.0f;
}

// Loss of Eq. 6 in the classifier form and its gradient at the tail's
// outputs: one wave per sample (logits [B][ld], rows: hit logit, 64 coarse,
// 128 fine bins), target bins from S of mu*; binary cross-entropy with
// logits, bins averaged per level and counted for hits only, the hit term
// weighted by w_hit, all divided by B.  G gets the gradient in bfloat16 (zero
// past the 193 outputs); part[block] = (total, bins, hit) of its four samples.
constexpr int CLS_OUT = 1 + NEDF_CLS_COARSE + NEDF_CLS_FINE;
__device__ __forceinline__ float softplus_f(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
__global__ __launch_bounds__(256) void k_cls_loss(const float* logits, int ld, const float* mu, const float* alpha,
                                                  int B, float w_hit, uint16_t* G, float* part) {
  __shared__ float red[4][3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int s = blockIdx.x * 4 + w;
  float lb = 0.f, lh = 0.f;
  if (s < B) {
    const float al = alpha[s];
    // S: u = (mu + l) / 2l with mu* = mu / l
    const float u = (mu[s] + 1.0f) * 0.5f;
    const int c = min(max(int(floorf(float(NEDF_CLS_COARSE) * u)), 0), NEDF_CLS_COARSE - 1);
    const int f = min(max(int(floorf(float(NEDF_CLS_FINE) * (float(NEDF_CLS_COARSE) * u - float(c)))), 0),
                      NEDF_CLS_FINE - 1);
    const float invB = 1.0f / float(B);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = lane + 64 * k;
      if (j >= ld) break;
      float g = 0.f;
      if (j < CLS_OUT) {
        const float z = logits[size_t(s) * ld + j];
        const float sg = 1.0f / (1.0f + expf(-z));
        if (j == 0) {
          lh += softplus_f(z) - al * z;
          g = w_hit * (sg - al) * invB;
        } else if (j <= NEDF_CLS_COARSE) {
          const float y = (j - 1 == c) ? 1.f : 0.f;
          lb += al * (softplus_f(z) - y * z) * (1.0f / NEDF_CLS_COARSE);
          g = al * (sg - y) * (invB / NEDF_CLS_COARSE);
        } else {
          const float y = (j - 1 - NEDF_CLS_COARSE == f) ? 1.f : 0.f;
          lb += al * (softplus_f(z) - y * z) * (1.0f / NEDF_CLS_FINE);
          g = al * (sg - y) * (invB / NEDF_CLS_FINE);
        }
      }
      G[size_t(s) * ld + j] = bf16_bits(g);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    lb += __shfl_xor(lb, off);
    lh += __shfl_xor(lh, off);
  }
  if (lane == 0) {
    red[w][0] = lb + w_hit * lh;
    red[w][1] = lb;
    red[w][2] = lh;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int i = threadIdx.x;
    part[size_t(blockIdx.x) * 3 + i] = ((red[0][i] + red[1][i]) + (red[2][i] + red[3][i]));
  }
}

// loss[i] = (sum over blocks of part[block][i]) / B, blocks added in a fixed
// order (lane l takes blocks l, l + 64, ...; then a fixed butterfly).
__global__ void k_cls_loss_reduce(const float* part, int n_blocks, int B, float* loss) {
  const int i = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (i >= 3) return;
  float s = 0.f;
  for (int q = lane; q < n_blocks; q += 64) s += part[size_t(q) * 3 + i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) loss[i] = s / float(B);
}


}  // namespace

// Split count of a batched weight-gradient launch over `tiles` 128 x 128
// output tiles: a power of two up to 64 giving at most 640 workgroups (two
// per compute unit and a quarter more, so that the last wave of workgroups
// is short), with the batch a multiple of 128 per split (an even number of
// 64-deep stages; the batch is a multiple of 256).
int wgrad_batch_splits(int B, int tiles) {
  int S = 1;
  while (S < 64 && tiles * S * 2 <= 640 && B % (S * 2 * 2 * GT_BK) == 0) S *= 2;
  return S;
}

// 128 x 128 output tiles of the regression form's hidden-layer weight gradients.
int regression_wgrad_tiles(const nedf_mlp_shape& sh, const nedf_train_layout& tl) {
  int t = 0;
  for (int l = 0; l < sh.n_hidden; ++l) t += (sh.width / 128) * (tl.L[l].Kpad / 128);
  return t;
}

size_t train_ws_bytes_cls(const nedf_mlp_shape& sh, int B);

size_t train_ws_bytes(const nedf_mlp_shape& sh, int B) {
  if (sh.in_kind == NEDF_IN_POINTS16) return train_ws_bytes_cls(sh, B);
  const nedf_train_layout tl = nedf_train_layout_of(sh);
  const int S = wgrad_batch_splits(B, regression_wgrad_tiles(sh, tl));
  size_t off = 0;
  off = nedf_tl_align(off + size_t(B) * tl.L[0].Kpad * 2);           // H_in
  off = nedf_tl_align(off + size_t(B) * sh.width * 2 * sh.n_hidden);  // H_0..H_{n-1}
  off = nedf_tl_align(off + size_t(B) * sh.width * 2 * sh.n_hidden);  // G_0..G_{n-1}
  off = nedf_tl_align(off + size_t(B) * (sh.width / 8) * sh.n_hidden);  // ReLU mask bits of H_0..H_{n-1}
  off = nedf_tl_align(off + size_t(B) * 4 * 2);                       // mu, alpha
  for (int l = 0; l < sh.n_hidden; ++l)                                // weight-gradient partials
    off = nedf_tl_align(off + size_t(S) * sh.width * (tl.L[l].Kpad + 1) * 4);
  off = nedf_tl_align(off + size_t(B / GT_BM) * HEAD_PART * 4);  // head partials, per 128-row tile
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
                       reinterpret_cast<float*>(st + l.W), reinterpret_cast<uint16_t*>(st + l.W16),
                       reinterpret_cast<uint16_t*>(st + l.W16T), l.N, l.K, l.Kpad, l.Nsrc);
    // the bias as one row of N values, of which the caller's array holds Nsrc
    hipLaunchKernelGGL(k_copy_w, dim3(blocks(size_t(l.N))), dim3(256), 0, s, b[i],
                       reinterpret_cast<float*>(st + l.b), static_cast<uint16_t*>(nullptr),
                       static_cast<uint16_t*>(nullptr), 1, l.Nsrc, l.N, 1);
  }
  return hipGetLastError();
}

hipError_t launch_train_step_cls(const nedf_mlp_shape& sh, uint8_t* st, const float* o_l, const float* d_l,
                                 const float* depth, const uint8_t* hit, int B, float lr, float b1, float b2,
                                 float eps, float w_hit, float bound, float* loss, uint8_t* ws, hipStream_t s);

hipError_t launch_train_step(const nedf_mlp_shape& sh, uint8_t* st, const float* o_l, const float* d_l,
                             const float* depth, const uint8_t* hit, int B, float lr, float b1, float b2, float eps,
                             float w_hit, float bound, float* loss, uint8_t* ws, hipStream_t s) {
  if (sh.in_kind == NEDF_IN_POINTS16)
    return launch_train_step_cls(sh, st, o_l, d_l, depth, hit, B, lr, b1, b2, eps, w_hit, bound, loss, ws, s);
  const nedf_train_layout tl = nedf_train_layout_of(sh);
  const int W = sh.width, NH = sh.n_hidden;
  const int K0p = tl.L[0].Kpad;
  const int S = wgrad_batch_splits(B, regression_wgrad_tiles(sh, tl));
  size_t off = 0;
  uint16_t* Hin = reinterpret_cast<uint16_t*>(ws + off);
  off = nedf_tl_align(off + size_t(B) * K0p * 2);
  uint16_t* Hs = reinterpret_cast<uint16_t*>(ws + off);
  off = nedf_tl_align(off + size_t(B) * W * 2 * NH);
  uint16_t* Gs = reinterpret_cast<uint16_t*>(ws + off);
  off = nedf_tl_align(off + size_t(B) * W * 2 * NH);
  uint8_t* bits = ws + off;
  off = nedf_tl_align(off + size_t(B) * (W / 8) * NH);
  float* mu = reinterpret_cast<float*>(ws + off);
  float* alpha = mu + B;
  off = nedf_tl_align(off + size_t(B) * 4 * 2);
  float* wpart[NEDF_MAX_LAYERS];
  for (int l = 0; l < NH; ++l) {
    wpart[l] = reinterpret_cast<float*>(ws + off);
    off = nedf_tl_align(off + size_t(S) * W * (tl.L[l].Kpad + 1) * 4);
  }
  float* hpart = reinterpret_cast<float*>(ws + off);
  const int hblocks = B / GT_BM;  // tiles of the last forward layer
  auto Hl = [&](int l) { return Hs + size_t(l) * B * W; };
  auto Gl = [&](int l) { return Gs + size_t(l) * B * W; };  // gradient at layer l's pre-activation
  auto Ml = [&](int l) { return bits + size_t(l) * B * (W / 8); };  // H_l > 0 as bits
  auto F = [&](size_t o) { return reinterpret_cast<float*>(st + o); };
  auto U = [&](size_t o) { return reinterpret_cast<uint16_t*>(st + o); };

  prof_mark("train.step", s, true);
  launch_train_encode(sh, o_l, d_l, depth, hit, B, K0p, bound, Hin, mu, alpha, s);
  // forward: H_l = relu(H_{l-1} W_l^T + b_l)
  // the last hidden layer's epilogue forms the head, the loss terms and
  // G_{NH-1} (its activation is not stored)
  const nedf_train_layer& hd = tl.L[NH];
  for (int l = 0; l < NH; ++l) {
    GemmArgs g{};
    g.A = l == 0 ? Hin : Hl(l - 1);
    g.lda = l == 0 ? K0p : W;
    g.B = U(tl.L[l].W16);
    g.ldb = tl.L[l].Kpad;
    g.M = B; g.N = W; g.K = tl.L[l].Kpad;
    g.k_per_split = g.K;
    g.bias = F(tl.L[l].b);
    g.ldo = W;
    if (l + 1 < NH) {
      g.out16 = Hl(l);
      g.bits_out = Ml(l);
      gemm<KC, KC, 0, false, 256, 256>(g, 1, s);  // B is a multiple of 256
    } else {
      g.out16b = Gl(NH - 1);
      g.head_w = F(hd.W); g.head_b = F(hd.b);
      g.mu = mu; g.alpha = alpha; g.w_hit = w_hit;
      g.part = hpart;
      gemm<KC, KC, 6>(g, 1, s);
    }
  }
  // backward through the hidden layers: data gradients
  // G_{l-1} = (G_l W_l) * (H_{l-1} > 0) (the mask from the forward pass's
  // bits), every G_l kept
  for (int l = NH - 1; l > 0; --l) {
    const nedf_train_layer& L = tl.L[l];
    GemmArgs d{};
    d.A = Gl(l); d.lda = W;                         // [B][W]: k-contiguous
    d.B = U(L.W16T); d.ldb = W;                     // W_l^T [Kpad][W] = [N][K]: k-contiguous
    d.M = B; d.N = W; d.K = W;
    d.k_per_split = W;
    d.bits_in = Ml(l - 1); d.ldm = W;       // the ReLU mask of H_{l-1} (256-row tiles take bits only)
    d.out16 = Gl(l - 1); d.ldo = W;
    gemm<KC, KC, 1, false, 256, 256>(d, 1, s);
  }
  // weight-gradient partials dW_l = G_l^T H_{l-1} of every layer in one
  // launch, then their sums over the splits in order
  {
    WgradBatch wb{};
    wb.n = NH; wb.S = S; wb.M = W; wb.B = B;
    ReduceArgs ra{};
    ra.n_layers = NH;
    ra.S = S;
    ra.step = reinterpret_cast<int64_t*>(st);
    ra.hpart = hpart; ra.h_blocks = hblocks;
    ra.gWh = F(hd.gW); ra.gbh = F(hd.gb); ra.loss = loss;
    int maxmn = 517, ny = 1;
    for (int l = 0; l < NH; ++l) {
      const nedf_train_layer& L = tl.L[l];
      wb.p[l] = WgradProb{Gl(l), l == 0 ? Hin : Hl(l - 1), wpart[l], wpart[l] + size_t(S) * W * L.Kpad,
                          l == 0 ? K0p : W, L.Kpad};
      ra.L[l] = ReduceLayer{wb.p[l].part, wb.p[l].colsum, F(L.gW), F(L.gb), W, L.Kpad, L.K};
      maxmn = std::max(maxmn, W * L.Kpad + W);
      ny = std::max(ny, L.Kpad / 128);
    }
    hipLaunchKernelGGL(k_wgrad, dim3(W / GT_BM, ny, NH * S), dim3(256), 0, s, wb);
    hipLaunchKernelGGL(k_reduce_grads, dim3(blocks(maxmn), NH + 1), dim3(256), 0, s, ra);
  }
  // Adam on every parameter array, one launch
  AdamArgs aa{};
  aa.step = reinterpret_cast<const int64_t*>(st);
  aa.lr = lr; aa.b1 = b1; aa.b2 = b2; aa.eps = eps;
  int nb = 0;
  for (int i = 0; i < tl.n_layers; ++i) {
    const nedf_train_layer& L = tl.L[i];
    aa.seg[aa.n_seg++] = AdamSeg{F(L.W), F(L.mW), F(L.vW), F(L.gW), U(L.W16), U(L.W16T), L.N * L.K, L.K, L.Kpad,
                                 L.N, nb};
    nb += int(blocks(size_t(L.N) * L.K));
    aa.seg[aa.n_seg++] = AdamSeg{F(L.b), F(L.mb), F(L.vb), F(L.gb), nullptr, nullptr, L.N, 1, 1, 1, nb};
    nb += int(blocks(size_t(L.N)));
  }
  hipLaunchKernelGGL(k_adam, dim3(nb), dim3(256), 0, s, aa);
  prof_mark("train.step", s, false);
  return hipGetLastError();
}

// ---- classifier-form training step ----------------------------------------------
namespace {
// 128 x 128 output tiles of every layer's weight gradient (the tail's N
// padded to the width).
int cls_wgrad_tiles(const nedf_train_layout& tl, int W) {
  int t = 0;
  for (int i = 0; i < tl.n_layers; ++i) t += (W / 128) * (tl.L[i].Kpad / 128);
  return t;
}
struct ClsTrainWs {
  uint16_t *X, *H, *A, *R, *G;
  float *LG, *Gh, *mu, *alpha, *wpart, *lpart;
  size_t part_off[NEDF_TRAIN_MAX_LAYERS];  // each layer's split partials, floats from wpart
  size_t end;
};
ClsTrainWs cls_train_ws(const nedf_mlp_shape& sh, int B, uint8_t* base) {
  const nedf_train_layout tl = nedf_train_layout_of(sh);
  const int W = sh.width, NB = sh.n_hidden, K0p = tl.L[0].Kpad;
  const int S = wgrad_batch_splits(B, cls_wgrad_tiles(tl, W));
  ClsTrainWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    uint8_t* p = base ? base + off : nullptr;
    off = nedf_tl_align(off + bytes);
    return p;
  };
  w.X = reinterpret_cast<uint16_t*>(take(size_t(B) * K0p * 2));
  w.H = reinterpret_cast<uint16_t*>(take(size_t(B) * W * 2 * (NB + 1)));
  w.A = reinterpret_cast<uint16_t*>(take(size_t(B) * W * 2 * NB));
  w.R = reinterpret_cast<uint16_t*>(take(size_t(B) * W * 2 * NB));
  // the bfloat16 gradient at every layer's pre-activation
  w.G = reinterpret_cast<uint16_t*>(take(size_t(B) * W * 2 * tl.n_layers));
  w.LG = reinterpret_cast<float*>(take(size_t(B) * W * 4));
  w.Gh = reinterpret_cast<float*>(take(size_t(B) * W * 4));
  w.mu = reinterpret_cast<float*>(take(size_t(B) * 4));
  w.alpha = reinterpret_cast<float*>(take(size_t(B) * 4));
  size_t nf = 0;
  for (int i = 0; i < tl.n_layers; ++i) {
    w.part_off[i] = nf;
    nf += size_t(S) * W * (tl.L[i].Kpad + 1);
    nf = (nf + 63) & ~size_t(63);
  }
  w.wpart = reinterpret_cast<float*>(take(nf * 4));
  w.lpart = reinterpret_cast<float*>(take(size_t(B / 4 + 1) * 3 * 4));
  w.end = off;
  return w;
}
}  // namespace

size_t train_ws_bytes_cls(const nedf_mlp_shape& sh, int B) { return cls_train_ws(sh, B, nullptr).end; }

// One Adam step of a classifier-form network (Eq. 6): forward through the
// head, the residual blocks (skip addition in the second layer's epilogue)
// and the tail; loss and tail gradient; backward with a float32 gradient
// stream for the skip path (each block adds its branch's data gradient to
// it in the GEMM epilogue, which also forms the next masked bfloat16
// gradient); weight gradients by split-K GEMMs reduced in order, per layer.
hipError_t launch_train_step_cls(const nedf_mlp_shape& sh, uint8_t* st, const float* o_l, const float* d_l,
                                 const float* depth, const uint8_t* hit, int B, float lr, float b1, float b2,
                                 float eps, float w_hit, float bound, float* loss, uint8_t* ws, hipStream_t s) {
  const nedf_train_layout tl = nedf_train_layout_of(sh);
  const int W = sh.width, NB = sh.n_hidden;
  const int K0p = tl.L[0].Kpad;
  const int S = wgrad_batch_splits(B, cls_wgrad_tiles(tl, W));
  const ClsTrainWs w = cls_train_ws(sh, B, ws);
  auto F = [&](size_t o) { return reinterpret_cast<float*>(st + o); };
  auto U = [&](size_t o) { return reinterpret_cast<uint16_t*>(st + o); };
  auto Hk = [&](int k) { return w.H + size_t(k) * B * W; };
  auto Ak = [&](int k) { return w.A + size_t(k) * B * W; };
  auto Rk = [&](int k) { return w.R + size_t(k) * B * W; };
  auto Gi = [&](int i) { return w.G + size_t(i) * B * W; };  // gradient at layer i's pre-activation
  const int tail = tl.n_layers - 1;
  prof_mark("train.step", s, true);
  // gamma_10 (the only classifier encoding training accepts)
  hipLaunchKernelGGL(k_train_encode_points<10>, dim3(blocks(size_t(B) * (K0p / 8))), dim3(256), 0, s, o_l, d_l, depth,
                     hit, B, K0p, bound, w.X, w.mu, w.alpha);
  // forward
  {
    GemmArgs g{};
    g.A = w.X; g.lda = K0p;
    g.B = U(tl.L[0].W16); g.ldb = K0p;
    g.M = B; g.N = W; g.K = K0p; g.k_per_split = K0p;
    g.bias = F(tl.L[0].b);
    g.out16 = Hk(0); g.ldo = W;
    gemm<KC, KC, 0>(g, 1, s);
  }
  for (int k = 0; k < NB; ++k) {
    const nedf_train_layer &L1 = tl.L[1 + 2 * k], &L2 = tl.L[2 + 2 * k];
    GemmArgs g{};
    g.A = Hk(k); g.lda = W;
    g.B = U(L1.W16); g.ldb = W;
    g.M = B; g.N = W; g.K = W; g.k_per_split = W;
    g.bias = F(L1.b);
    g.out16 = Ak(k); g.ldo = W;
    gemm<KC, KC, 0>(g, 1, s);
    GemmArgs r{};
    r.A = Ak(k); r.lda = W;
    r.B = U(L2.W16); r.ldb = W;
    r.M = B; r.N = W; r.K = W; r.k_per_split = W;
    r.bias = F(L2.b);
    r.resid16 = Hk(k);
    r.out16 = Hk(k + 1); r.out16b = Rk(k); r.ldo = W;
    gemm<KC, KC, 5>(r, 1, s);
  }
  {
    GemmArgs g{};
    g.A = Hk(NB); g.lda = W;
    g.B = U(tl.L[tail].W16); g.ldb = W;
    g.M = B; g.N = W; g.K = W; g.k_per_split = W;
    g.bias = F(tl.L[tail].b);
    g.out32 = w.LG; g.ldo = W;
    gemm<KC, KC, 3>(g, 1, s);
  }
  const int lblocks = (B + 3) / 4;
  hipLaunchKernelGGL(k_cls_loss, dim3(lblocks), dim3(256), 0, s, w.LG, W, w.mu, w.alpha, B, w_hit, Gi(tail), w.lpart);
  hipLaunchKernelGGL(k_cls_loss_reduce, dim3(1), dim3(256), 0, s, w.lpart, lblocks, B, loss);
  // data gradient through layer i: out = G W_i, plus epilogue options
  auto dgrad = [&](int i) {
    GemmArgs g{};
    g.A = Gi(i); g.lda = W;
    g.B = U(tl.L[i].W16T); g.ldb = W;
    g.M = B; g.N = W; g.K = W; g.k_per_split = W;
    g.ldo = W; g.ldm = W;
    return g;
  };
  // tail
  {
    GemmArgs g = dgrad(tail);
    g.out32 = w.Gh;
    g.mask = Rk(NB - 1);
    g.out16 = Gi(2 * NB);  // gradient at the last block's second pre-activation
    gemm<KC, KC, 4>(g, 1, s);
  }
  for (int k = NB - 1; k >= 0; --k) {
    const int i1 = 1 + 2 * k, i2 = 2 + 2 * k;
    {
      GemmArgs g = dgrad(i2);
      g.mask = Ak(k);
      g.out16 = Gi(i1);  // gradient at the first layer's pre-activation
      gemm<KC, KC, 1>(g, 1, s);
    }
    {
      GemmArgs g = dgrad(i1);
      g.resid32 = w.Gh;
      g.out32 = w.Gh;                         // skip path plus the branch
      g.mask = k > 0 ? Rk(k - 1) : Hk(0);     // next: block k-1's second layer, or the head
      g.out16 = Gi(i1 - 1);
      gemm<KC, KC, 4>(g, 1, s);
    }
  }
  // weight gradients of every layer from its pre-activation gradient and its
  // input, in one launch, then their sums over the splits in order
  {
    WgradBatch wb{};
    wb.n = tl.n_layers; wb.S = S; wb.M = W; wb.B = B;
    ReduceArgs ra{};
    ra.n_layers = tl.n_layers;
    ra.S = S;
    ra.step = reinterpret_cast<int64_t*>(st);
    int maxmn = 0, ny = 1;
    for (int i = 0; i < tl.n_layers; ++i) {
      const nedf_train_layer& L = tl.L[i];
      const uint16_t* X = i == 0 ? w.X : i == tail ? Hk(NB) : (i % 2 == 1 ? Hk((i - 1) / 2) : Ak((i - 2) / 2));
      float* part = w.wpart + w.part_off[i];
      wb.p[i] = WgradProb{Gi(i), X, part, part + size_t(S) * W * L.Kpad, i == 0 ? K0p : W, L.Kpad};
      ra.L[i] = ReduceLayer{part, part + size_t(S) * W * L.Kpad, F(L.gW), F(L.gb), W, L.Kpad, L.K};
      maxmn = std::max(maxmn, W * L.Kpad + W);
      ny = std::max(ny, L.Kpad / 128);
    }
    hipLaunchKernelGGL(k_wgrad, dim3(W / GT_BM, ny, tl.n_layers * S), dim3(256), 0, s, wb);
    hipLaunchKernelGGL(k_reduce_grads, dim3(blocks(maxmn), tl.n_layers), dim3(256), 0, s, ra);
  }
  // Adam, in launches of at most one argument block of segments
  AdamArgs aa{};
  aa.step = reinterpret_cast<const int64_t*>(st);
  aa.lr = lr; aa.b1 = b1; aa.b2 = b2; aa.eps = eps;
  int nb = 0;
  auto flush = [&]() {
    if (aa.n_seg) hipLaunchKernelGGL(k_adam, dim3(nb), dim3(256), 0, s, aa);
    aa.n_seg = 0;
    nb = 0;
  };
  constexpr int MAXSEG = int(sizeof(aa.seg) / sizeof(aa.seg[0]));
  for (int i = 0; i < tl.n_layers; ++i) {
    if (aa.n_seg + 2 > MAXSEG) flush();
    const nedf_train_layer& L = tl.L[i];
    aa.seg[aa.n_seg++] = AdamSeg{F(L.W), F(L.mW), F(L.vW), F(L.gW), U(L.W16), U(L.W16T), L.N * L.K, L.K, L.Kpad,
                                 L.N, nb};
    nb += int(blocks(size_t(L.N) * L.K));
    aa.seg[aa.n_seg++] = AdamSeg{F(L.b), F(L.mb), F(L.vb), F(L.gb), nullptr, nullptr, L.N, 1, 1, 1, nb};
    nb += int(blocks(size_t(L.N)));
  }
  flush();
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
  launch_train_encode(sh, o_l, d_l, nullptr, nullptr, B, K0p, 1.0f, Hin, mu, mu, s);
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
    gemm<KC, KC, 0>(g, 1, s);
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
    hipError_t e = hipMemcpyAsync(W[i], st + ow, size_t(l.Nsrc) * l.K * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(b[i], st + ob, size_t(l.Nsrc) * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace nedf
