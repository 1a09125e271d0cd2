// Register-resident MLP engine on gfx950 matrix cores.
//
// A workgroup of 4 waves evaluates one network for 4 x 32 x NB samples.  Each
// wave keeps its samples' activations in registers as matrix-core B operands
// for the whole network (see blob_layout.h); the workgroup streams the
// weights through LDS one output block ("chunk": 32 output features x all K,
// plus that block's bias and head rows) at a time, double-buffered: while the
// waves multiply chunk i from one LDS buffer, chunk i+1 is copied from global
// memory (L2) straight into the other buffer; one barrier per chunk.
#pragma once
#include "device_common.h"

namespace eng {

constexpr int WAVES = 4;
constexpr int THREADS = 64 * WAVES;

template <int DT> struct Tr;

template <> struct Tr<1> {  // bfloat16 inputs, float32 accumulate
  using frag = bf16x8_t;
  static constexpr int KPS = 16;     // K values per step
  static constexpr int FRAG = 1024;  // bytes per K-step fragment (64 lanes x 16 B)
  static constexpr int KPR = 1;      // K-steps per 16-byte LDS read
  static constexpr int NB = 1;       // 32-sample blocks per wave
  __device__ static __forceinline__ f32x16_t mma(frag a, frag b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ frag pick(const uint4& w, int) { return __builtin_bit_cast(frag, w); }
};

template <> struct Tr<0> {  // float32
  using frag = float;
  static constexpr int KPS = 2;
  static constexpr int FRAG = 256;
  static constexpr int KPR = 4;
  static constexpr int NB = 1;
  __device__ static __forceinline__ f32x16_t mma(frag a, frag b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ frag pick(const uint4& w, int i) {
    return __uint_as_float(i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w);
  }
};

// Bytes of one chunk: K-steps of fragments, bias, head rows.
template <int DT>
constexpr int chunk_bytes(int ks, int heads) {
  return ks * Tr<DT>::FRAG + 128 * (1 + heads);
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// ---- chunk staging ---------------------------------------------------------
// Chunks go global -> LDS directly (global_load_lds_dwordx4): each wave moves
// 1 KB pieces, 16 bytes per lane, no staging registers.  The caller waits
// for the loads (vmcnt) and barriers before the buffer is read.
template <int BYTES>
__device__ __forceinline__ void dma_chunk(const uint8_t* src, uint8_t* dst) {
  constexpr int P = (BYTES + 1023) / 1024;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < (P + WAVES - 1) / WAVES; ++i) {
    const int piece = wave + i * WAVES;
    if (piece < P) {
      const int off = piece * 1024 + lane * 16;
      if (BYTES % 1024 == 0 || off < BYTES)
        __builtin_amdgcn_global_load_lds(src + off, dst + piece * 1024, 16, 0, 0);
    }
  }
}

__device__ __forceinline__ void dma_wait_barrier() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

// ---- epilogues ---------------------------------------------------------------
// ReLU of output block fb, written as the next layer's B operand.
template <int DT, int NB, int KSO>
__device__ __forceinline__ void epi_hidden(int fb, const f32x16_t (&acc)[NB],
                                           typename Tr<DT>::frag (&Bout)[NB][KSO]) {
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if constexpr (DT == 1) {
      // round to bfloat16, then ReLU on the packed 16-bit patterns (a signed
      // 16-bit max with 0 clears exactly the negative values)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2_t;
        typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;
        bf16x8_t v;
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const f32x2_t f = {acc[nb][8 * q + j], acc[nb][8 * q + j + 1]};
          const bf16x2_t b = __builtin_convertvector(f, bf16x2_t);
          v[j] = b[0];
          v[j + 1] = b[1];
        }
        typedef __attribute__((__vector_size__(8 * sizeof(short)))) short s16x8_t;
        const s16x8_t zero = {0, 0, 0, 0, 0, 0, 0, 0};
        s16x8_t r = __builtin_elementwise_max(__builtin_bit_cast(s16x8_t, v), zero);
        Bout[nb][2 * fb + q] = __builtin_bit_cast(bf16x8_t, r);
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) Bout[nb][16 * fb + r] = fmaxf(acc[nb][r], 0.0f);
    }
  }
}

// Narrow heads: partial[nb][o] += sum_r w[o][h][r] * relu(acc[nb][r]), with
// the head rows of this block read from the chunk in LDS.
template <int NB, int NOUT>
__device__ __forceinline__ void epi_head(const f32x16_t (&acc)[NB], const uint8_t* heads, int half,
                                         float (&partial)[NB][NOUT]) {
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const float4* w4 = reinterpret_cast<const float4*>(heads + 128 * o + 64 * half);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = w4[q];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        partial[nb][o] = fmaf(t.x, fmaxf(acc[nb][4 * q + 0], 0.0f), partial[nb][o]);
        partial[nb][o] = fmaf(t.y, fmaxf(acc[nb][4 * q + 1], 0.0f), partial[nb][o]);
        partial[nb][o] = fmaf(t.z, fmaxf(acc[nb][4 * q + 2], 0.0f), partial[nb][o]);
        partial[nb][o] = fmaf(t.w, fmaxf(acc[nb][4 * q + 3], 0.0f), partial[nb][o]);
      }
    }
  }
}

__device__ __forceinline__ f32x16_t bias_acc(const uint8_t* bias, int half) {
  const float4* b4 = reinterpret_cast<const float4*>(bias + 64 * half);
  f32x16_t a;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 t = b4[q];
    a[4 * q + 0] = t.x; a[4 * q + 1] = t.y; a[4 * q + 2] = t.z; a[4 * q + 3] = t.w;
  }
  return a;
}

// ---- one layer -----------------------------------------------------------
// Multiplies the FB chunks of a layer (KS_IN K-steps each, CB_THIS bytes)
// against Bin.  Chunk 0 must be in LDS buffer `cur` on entry; the next chunk
// (next block, or the first chunk of the following layer at w_next, CB_NEXT
// bytes) is prefetched during each block.
// MODE 0: hidden epilogue into Bout.  MODE 1: head epilogue.  MODE 2: both.
template <int DT, int NB, int KS_IN, int FB, int CB_THIS, int CB_NEXT, int KSO, int NOUT, int MODE,
          int CHUNK>
__device__ __forceinline__ void layer(const typename Tr<DT>::frag (&Bin)[NB][KS_IN],
                                      typename Tr<DT>::frag (&Bout)[NB][KSO], const uint8_t* w_this,
                                      const uint8_t* w_next, uint8_t* lds, int& cur,
                                      float (&partial)[NB][NOUT]) {
  using T = Tr<DT>;
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  constexpr int R = KS_IN / T::KPR;             // 16-byte LDS reads per chunk
  static_assert(KS_IN % T::KPR == 0, "K-steps must fill whole LDS reads");
  // hidden-layer epilogues are deferred by one block so that their vector
  // work overlaps the next block's matrix ops
  constexpr bool DEFER = (MODE == 0);
  f32x16_t prev[NB];
#pragma unroll
  for (int fb = 0; fb < FB; ++fb) {
    uint8_t* nbuf = lds + (cur ^ 1) * CHUNK;
    if (fb + 1 < FB) {
      dma_chunk<CB_THIS>(w_this + size_t(fb + 1) * CB_THIS, nbuf);
    } else if (w_next != nullptr) {
      if constexpr (CB_NEXT > 0) dma_chunk<CB_NEXT>(w_next, nbuf);
    }
    const uint8_t* chunk = lds + cur * CHUNK;
    const uint4* words = reinterpret_cast<const uint4*>(chunk) + lane;
    f32x16_t acc[NB];
    {
      const f32x16_t b0 = bias_acc(chunk + KS_IN * T::FRAG, half);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = b0;
    }
    // Software pipeline over the chunk's 16-byte LDS reads: the reads of
    // group g+1 are issued before the matrix ops of group g; scheduling
    // barriers keep the compiler from sinking them, so LDS latency is
    // covered by a group of matrix ops.
    constexpr int G = 4;
    constexpr int NG = (R + G - 1) / G;
    uint4 wbuf[2][G];
#pragma unroll
    for (int r = 0; r < G; ++r)
      if (r < R) wbuf[0][r] = words[r * 64];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      if (gi + 1 < NG) {
#pragma unroll
        for (int r = 0; r < G; ++r)
          if ((gi + 1) * G + r < R) wbuf[(gi + 1) & 1][r] = words[((gi + 1) * G + r) * 64];
      }
#pragma unroll
      for (int r = 0; r < G; ++r) {
        if (gi * G + r < R) {
#pragma unroll
          for (int i = 0; i < T::KPR; ++i) {
            const int ks = (gi * G + r) * T::KPR + i;
            const typename T::frag a = T::pick(wbuf[gi & 1][r], i);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb] = T::mma(a, Bin[nb][ks], acc[nb]);
          }
        }
      }
      if constexpr (DEFER) {
        if (fb > 0 && gi == 0) epi_hidden<DT, NB, KSO>(fb - 1, prev, Bout);
      }
      // order inside the region: next group's LDS reads, then matrix ops
      // interleaved with the deferred epilogue's vector ops
      if (gi + 1 < NG) __builtin_amdgcn_sched_group_barrier(0x100, G, 0);
      if (DEFER && fb > 0 && gi == 0) {
#pragma unroll
        for (int m = 0; m < G * T::KPR * NB; ++m) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 10, 0);
        }
      } else {
        __builtin_amdgcn_sched_group_barrier(0x008, G * T::KPR * NB, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (DEFER) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) prev[nb] = acc[nb];
    } else {
      if constexpr (MODE == 2) epi_hidden<DT, NB, KSO>(fb, acc, Bout);
      epi_head<NB, NOUT>(acc, chunk + KS_IN * T::FRAG + 128, half, partial);
    }
    dma_wait_barrier();
    cur ^= 1;
  }
  if constexpr (DEFER) epi_hidden<DT, NB, KSO>(FB - 1, prev, Bout);
}

// ---- whole trunk ------------------------------------------------------------
// Hidden layers 0..NHID-1 of the blob on the encoded input Benc; the head dot
// products accumulate into `partial` (each lane half over its own features;
// the caller adds the halves).  With KEEP_LAST the last hidden activation is
// also left in Blast as a B operand (input of the colour layer, whose first
// chunk, CB_AFTER bytes at w_after, is prefetched).
template <int DT, int WIDTH, int KS0, int NHID, int NOUT, int CHUNK, bool KEEP_LAST, int CB_AFTER>
__device__ __forceinline__ void trunk(const nedf_blob_header* hb, const uint8_t* blob,
                                      const typename Tr<DT>::frag (&Benc)[Tr<DT>::NB][KS0],
                                      uint8_t* lds, float (&partial)[Tr<DT>::NB][NOUT],
                                      typename Tr<DT>::frag (&Blast)[Tr<DT>::NB][WIDTH / Tr<DT>::KPS],
                                      const uint8_t* w_after, int* cur_io = nullptr) {
  using T = Tr<DT>;
  constexpr int NB = T::NB;
  constexpr int FB = WIDTH / 32;
  constexpr int KSH = WIDTH / T::KPS;
  constexpr int CB0 = chunk_bytes<DT>(KS0, 0);
  constexpr int CBH = chunk_bytes<DT>(KSH, 0);
  constexpr int CBL = chunk_bytes<DT>(KSH, NOUT);
  static_assert(NHID >= 3, "need at least three hidden layers");
  static_assert(CHUNK >= CB0 && CHUNK >= CBL, "LDS chunk buffer too small");
  typename T::frag X[NB][KSH], Y[NB][KSH];
  int cur = cur_io ? *cur_io : 0;
  const uint64_t* off = hb->off_layer;
  dma_chunk<CB0>(blob + off[0], lds + cur * CHUNK);
  dma_wait_barrier();
  // layer 0: encoding -> X; then pairs X -> Y -> X; the last layer feeds the head
  layer<DT, NB, KS0, FB, CB0, CBH, KSH, NOUT, 0, CHUNK>(Benc, X, blob + off[0], blob + off[1], lds, cur,
                                                       partial);
  constexpr int PAIRS = (NHID - 2) / 2;
  for (int p = 0; p < PAIRS; ++p) {
    const int L = 1 + 2 * p;
    layer<DT, NB, KSH, FB, CBH, CBH, KSH, NOUT, 0, CHUNK>(X, Y, blob + off[L], blob + off[L + 1], lds, cur,
                                                         partial);
    if ((NHID - 2) % 2 == 0 && p == PAIRS - 1) {
      layer<DT, NB, KSH, FB, CBH, CBL, KSH, NOUT, 0, CHUNK>(Y, X, blob + off[L + 1], blob + off[L + 2], lds,
                                                           cur, partial);
    } else {
      layer<DT, NB, KSH, FB, CBH, CBH, KSH, NOUT, 0, CHUNK>(Y, X, blob + off[L + 1], blob + off[L + 2], lds,
                                                           cur, partial);
    }
  }
  constexpr int LAST_MODE = KEEP_LAST ? 2 : 1;
  if constexpr ((NHID - 2) % 2 == 1) {
    layer<DT, NB, KSH, FB, CBH, CBL, KSH, NOUT, 0, CHUNK>(X, Y, blob + off[NHID - 2], blob + off[NHID - 1],
                                                         lds, cur, partial);
    layer<DT, NB, KSH, FB, CBL, CB_AFTER, KSH, NOUT, LAST_MODE, CHUNK>(Y, Blast, blob + off[NHID - 1], w_after,
                                                                      lds, cur, partial);
  } else {
    layer<DT, NB, KSH, FB, CBL, CB_AFTER, KSH, NOUT, LAST_MODE, CHUNK>(X, Blast, blob + off[NHID - 1], w_after,
                                                                      lds, cur, partial);
  }
  if (cur_io) *cur_io = cur;
}

// ---- first-layer encoding ----------------------------------------------------
// Slot a holds sin(pi (2^level p_comp + h / 2)) for a < n L (h = 0 gives
// sin, h = 1 cos), then the identity components two per slot, then zeros.
template <int N, int L>
__device__ __forceinline__ float enc_slot(const float (&p)[N], int a, int half) {
  if (a < N * L) {
    const int level = a / N, comp = a % N;
    return sinpi_hw(fmaf(float(1 << level), p[comp], 0.5f * float(half)));
  }
  const int i = a - N * L;
  if (i >= (N + 1) / 2) return 0.0f;
  if (2 * i + 1 < N) return half ? p[2 * i + 1] : p[2 * i];
  return half ? 0.0f : p[2 * i];
}

template <int DT, int N, int L, int KS0>
__device__ __forceinline__ void encode_input(const float (&p)[N], int half,
                                             typename Tr<DT>::frag (&B)[KS0]) {
  if constexpr (DT == 1) {
#pragma unroll
    for (int ks = 0; ks < KS0; ++ks) {
      bf16x8_t v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = static_cast<__bf16>(enc_slot<N, L>(p, 8 * ks + j, half));
      B[ks] = v;
    }
  } else {
#pragma unroll
    for (int ks = 0; ks < KS0; ++ks) B[ks] = enc_slot<N, L>(p, ks, half);
  }
}

// K-steps of an encoded input with n components and L levels.
template <int DT>
constexpr int ks_for_slots(int slots) {
  return DT == 1 ? (slots + 7) / 8 : (slots + 3) / 4 * 4;
}

}  // namespace eng
