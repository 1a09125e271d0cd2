// Register-resident MLP engine on gfx950 matrix cores.
//
// A workgroup of NW waves (4 or 8) evaluates one network for NW x 32 x NB
// samples.  Each
// wave keeps its samples' activations in registers as matrix-core B operands
// for the whole network (see blob_layout.h); the workgroup streams the
// weights through LDS.  A "chunk" is one output block (32 output features x
// all K, plus that block's bias and head rows); SB consecutive chunks form a
// superchunk, the unit of one global->LDS copy and one barrier.  Three LDS
// slots form a ring: while the waves multiply superchunk i, superchunks i+1
// and i+2 are being copied from global memory (L2) straight into the other
// two slots.
#pragma once
#include <utility>

#include "device_common.h"

namespace eng {

// Four 32-bit lanes as a native vector (so inline asm can bind it to a
// 128-bit VGPR tuple).
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

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
  __device__ static __forceinline__ frag pick(const u32x4& w, int) { return __builtin_bit_cast(frag, w); }
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
  __device__ static __forceinline__ frag pick(const u32x4& w, int i) {
    return __uint_as_float(i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w);
  }
};

template <> struct Tr<2> {  // OCP E4M3 inputs with per-layer scales, float32 accumulate
  typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8_t;
  using frag = i32x8_t;              // 32 fp8 values per lane
  static constexpr int KPS = 64;
  static constexpr int FRAG = 2048;  // two 1 KB halves (lane words 0..15 and 16..31)
  static constexpr int KPR = 1;      // unused for FP8 (two reads per K-step)
  static constexpr int NB = 1;
  __device__ static __forceinline__ f32x16_t mma(frag a, frag b, f32x16_t c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
  }
  __device__ static __forceinline__ frag pick2(const u32x4& lo, const u32x4& hi) {
    frag f;
    f[0] = int(lo.x); f[1] = int(lo.y); f[2] = int(lo.z); f[3] = int(lo.w);
    f[4] = int(hi.x); f[5] = int(hi.y); f[6] = int(hi.z); f[7] = int(hi.w);
    return f;
  }
};

// MX E4M3 (OCP Microscaling): E4M3 values with one E8M0 scale per 32 along
// K, applied by the scaled matrix op.  In the operand registers a lane's
// bytes 0..15 belong to the first 32-value block of the K-step (with the
// other lane half's bytes 0..15) and bytes 16..31 to the second; the scale
// of the first block comes from the lane in half 0 and that of the second
// from the lane in half 1, each in byte 0 of its scale operand.
template <> struct Tr<3> {
  typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8_t;
  struct frag {
    i32x8_t v;  // 32 E4M3 values
    int sc;     // this lane's block scale (E8M0 in byte 0)
  };
  static constexpr int KPS = 64;
  static constexpr int FRAG = 2048;
  static constexpr int KPR = 1;
  static constexpr int NB = 1;
  __device__ static __forceinline__ f32x16_t mma(const i32x8_t& a, int a_sc, const frag& b, f32x16_t c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b.v, c, 0, 0, 0, a_sc, 0, b.sc);
  }
  __device__ static __forceinline__ i32x8_t pick2(const u32x4& lo, const u32x4& hi) {
    i32x8_t f;
    f[0] = int(lo.x); f[1] = int(lo.y); f[2] = int(lo.z); f[3] = int(lo.w);
    f[4] = int(hi.x); f[5] = int(hi.y); f[6] = int(hi.z); f[7] = int(hi.w);
    return f;
  }
};

// E8M0 block scale of a block whose largest magnitude is amax (>= 0): the
// smallest power of two 2^e with amax / 2^e <= 448 (E4M3's largest value):
// floor(log2 amax) - 8, plus one when the significand of amax exceeds 1.75
// (amax / 2^e would pass 448); as a biased byte, and 2^-e, the factor the
// values are multiplied by before rounding to E4M3 (1 for an all-zero block,
// whose byte is 0).
__device__ __forceinline__ void mx_scale(float amax, int& byte, float& inv) {
  const uint32_t bits = __float_as_uint(amax);
  const int eb = int((bits >> 23) & 0xFFu);  // biased exponent; 0 for zero and subnormals
  if (eb == 0) {
    byte = 0;
    inv = 1.0f;
    return;
  }
  const int e = eb - 127 - 8 + ((bits & 0x7FFFFFu) > 0x600000u ? 1 : 0);  // scale exponent
  byte = e + 127 < 0 ? 0 : (e + 127 > 254 ? 254 : e + 127);
  inv = __builtin_amdgcn_ldexpf(1.0f, -(byte - 127));
}

// Quantise 16 values of one lane with a block scale: four packed E4M3 words.
__device__ __forceinline__ void mx_pack16(const float (&v)[16], float inv, int (&w)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float t[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) t[j] = fminf(fmaxf(v[4 * q + j] * inv, -448.0f), 448.0f);
    int x = __builtin_amdgcn_cvt_pk_fp8_f32(t[0], t[1], 0, false);
    w[q] = __builtin_amdgcn_cvt_pk_fp8_f32(t[2], t[3], x, true);
  }
}

// Matrix ops of one group of G consecutive 16-byte LDS reads (read r0..r0+G-1
// of the chunk) against the B operand.
template <int DT, int NB, int KS_IN, int G>
__device__ __forceinline__ void mma_group(const u32x4 (&w)[G], int r0, int R,
                                          const typename Tr<DT>::frag (&Bin)[NB][KS_IN], f32x16_t (&acc)[NB],
                                          uint32_t wsc = 0u) {
  using T = Tr<DT>;
  if constexpr (DT == 3) {
    // wsc: this lane's weight-block scales, byte ks for K-step ks
#pragma unroll
    for (int r = 0; r + 1 < G; r += 2) {
      if (r0 + r + 1 < R) {
        const int ks = (r0 + r) / 2;
        const typename T::i32x8_t a = T::pick2(w[r], w[r + 1]);
        const int asc = int((wsc >> (8 * ks)) & 0xFFu);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = T::mma(a, asc, Bin[nb][ks], acc[nb]);
      }
    }
  } else if constexpr (DT == 2) {
#pragma unroll
    for (int r = 0; r + 1 < G; r += 2) {
      if (r0 + r + 1 < R) {
        const int ks = (r0 + r) / 2;
        const typename T::frag a = T::pick2(w[r], w[r + 1]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = T::mma(a, Bin[nb][ks], acc[nb]);
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < G; ++r) {
      if (r0 + r < R) {
#pragma unroll
        for (int i = 0; i < T::KPR; ++i) {
          const int ks = (r0 + r) * T::KPR + i;
          const typename T::frag a = T::pick(w[r], i);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb] = T::mma(a, Bin[nb][ks], acc[nb]);
        }
      }
    }
  }
}

// Matrix ops per group (for scheduling hints).
template <int DT, int NB, int G>
constexpr int mma_per_group() { return DT >= 2 ? (G / 2) * NB : G * Tr<DT>::KPR * NB; }

// Bytes of one chunk: K-steps of fragments, bias, head rows.
// MX adds 1 KB of weight-block scales after the fragments ([lane][16] bytes,
// byte ks of lane l the scale of K-step ks's block that lane supplies).
template <int DT>
constexpr int mx_scale_bytes() { return DT == 3 ? 1024 : 0; }
template <int DT>
constexpr int chunk_bytes(int ks, int heads) {
  return ks * Tr<DT>::FRAG + mx_scale_bytes<DT>() + 128 * (1 + heads);
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// ---- chunk staging ---------------------------------------------------------
// Chunks go global -> LDS directly (global_load_lds_dwordx4): 1 KB pieces,
// 16 bytes per lane.  Every wave issues the same number of copy
// instructions per chunk (waves without a piece of their own repeat the last
// piece, which writes identical bytes), so the number of a wave's
// outstanding copies is a compile-time constant and the wait for a chunk can
// leave the younger chunk's copies in flight.
constexpr int dma_instr(int bytes, int nw = WAVES) { return ((bytes + 1023) / 1024 + nw - 1) / nw; }

template <int BYTES, int NW = WAVES>
__device__ __forceinline__ void dma_chunk(const uint8_t* src, uint8_t* dst) {
  constexpr int P = (BYTES + 1023) / 1024;
  constexpr int NI = dma_instr(BYTES, NW);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    int piece = wave + i * NW;
    piece = piece < P ? piece : P - 1;
    const int off = piece * 1024 + lane * 16;
    if (BYTES % 1024 == 0 || off < BYTES)
      __builtin_amdgcn_global_load_lds(src + off, dst + piece * 1024, 16, 0, 0);
  }
}

// Wait until at most N vector-memory operations of this wave are pending
// (lgkm and exp counters left at their maxima), then barrier.
template <int N>
__device__ __forceinline__ void dma_wait_barrier_n() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  // A plain __syncthreads() would add a release fence, which waits for every
  // outstanding global->LDS copy (vmcnt 0) including the younger prefetch.
  // The memory clobber keeps all memory operations on their side of the
  // barrier; the LDS reads of this wave are already complete (their explicit
  // lgkmcnt waits precede this point in program order).
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

__device__ __forceinline__ void dma_wait_barrier() { dma_wait_barrier_n<0>(); }

constexpr int NBUF = 3;  // LDS chunk buffers (prefetch distance 2)

// LDS reads of a chunk.  The compiler waits for every outstanding
// global->LDS copy (vmcnt 0) before any LDS read it can see, because it cannot
// tell that the copy targets another buffer; these reads are therefore issued
// as inline ds_read_b128 and completed with explicit lgkmcnt waits that are
// tied to the destination registers (LDS operations complete in order, so
// "at most N outstanding" guarantees every read issued before the last N).
typedef __attribute__((address_space(3))) uint8_t lds_byte_t;

__device__ __forceinline__ uint32_t lds_offset(const uint8_t* p) {
  return uint32_t(reinterpret_cast<uintptr_t>((const lds_byte_t*)p));
}

template <int OFF>
__device__ __forceinline__ u32x4 lds_read16(uint32_t addr) {
  static_assert(OFF >= 0 && OFF < 65536 && OFF % 16 == 0, "ds_read_b128 offset");
  u32x4 v;
  asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(v) : "v"(addr), "n"(OFF));
  return v;
}

// A 16-byte LDS write issued the same way (no wait is implied by the
// compiler; reads of the same address by the same wave return it in order).
__device__ __forceinline__ void lds_write16(uint32_t addr, u32x4 v) {
  asm volatile("ds_write_b128 %0, %1" ::"v"(addr), "v"(v));
}

template <int N>
__device__ __forceinline__ void lds_wait4(u32x4& a, u32x4& b, u32x4& c, u32x4& d) {
  asm volatile("s_waitcnt lgkmcnt(%4)" : "+v"(a), "+v"(b), "+v"(c), "+v"(d) : "n"(N));
}

// ---- epilogues ---------------------------------------------------------------
// ReLU of output block fb, written as the next layer's B operand.
template <int DT, int NB, int KSO>
__device__ __forceinline__ void epi_hidden(int fb, const f32x16_t (&acc)[NB],
                                           typename Tr<DT>::frag (&Bout)[NB][KSO], float2 qs) {
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if constexpr (DT == 3) {
      // ReLU; block fb (this sample's 32 features, 16 in each lane half) is
      // one MX block of K-step fb / 2: its scale from the larger of the two
      // halves' maxima, the lane's 16 values quantised into bytes
      // 16 (fb % 2) .. + 15; the half whose turn it is (half fb % 2)
      // carries the scale byte
      float v[16];
      float mx = 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        v[r] = fmaxf(acc[nb][r], 0.0f);
        mx = fmaxf(mx, v[r]);
      }
      mx = fmaxf(mx, __shfl_xor(mx, 32));
      int byte;
      float inv;
      mx_scale(mx, byte, inv);
      int w[4];
      mx_pack16(v, inv, w);
#pragma unroll
      for (int q = 0; q < 4; ++q) Bout[nb][fb / 2].v[(fb % 2) * 4 + q] = w[q];
      const int half = (threadIdx.x & 63) >> 5;
      if (half == (fb % 2)) Bout[nb][fb / 2].sc = byte;
      (void)qs;
    } else if constexpr (DT == 2) {
      // real = acc * qs.x; ReLU; quantise real / a_next = acc * (qs.x * qs.y)
      // to E4M3 (saturating at +-448); block fb fills half of K-step fb / 2
      const float m = qs.x * qs.y;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = fminf(fmaxf(acc[nb][4 * q + j] * m, 0.0f), 448.0f);
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
        Bout[nb][fb / 2][(fb % 2) * 4 + q] = w;
      }
    } else if constexpr (DT == 1) {
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

// Residual epilogue: the block's B-operand words already hold the residual
// stream h; they become h + ReLU(acc), rounded to the operand type once the
// single-precision sum is formed (F32 and BF16 only).
template <int DT, int NB, int KSO>
__device__ __forceinline__ void epi_residual(int fb, const f32x16_t (&acc)[NB], typename Tr<DT>::frag (&Bout)[NB][KSO]) {
  static_assert(DT == 0 || DT == 1, "residual epilogue: F32 or BF16");
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if constexpr (DT == 1) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        bf16x8_t v = Bout[nb][2 * fb + q];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = static_cast<__bf16>(static_cast<float>(v[j]) + fmaxf(acc[nb][8 * q + j], 0.0f));
        Bout[nb][2 * fb + q] = v;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) Bout[nb][16 * fb + r] = Bout[nb][16 * fb + r] + fmaxf(acc[nb][r], 0.0f);
    }
  }
}

// Classifier epilogue: running first-maximum of the coarse bins (features
// 0..63) and fine bins (64..191) of this lane's sample over its own
// features, and the hit logit (feature 192).  st[nb] = {best coarse value,
// its bin, best fine value, its bin, hit logit}; a lane's features increase
// with r, so a strict comparison keeps the first maximum.
template <int NB, int NOUT>
__device__ __forceinline__ void epi_argmax(int fb, const f32x16_t (&acc)[NB], float (&st)[NB][NOUT]) {
  static_assert(NOUT >= 5, "argmax state needs five values");
  const int half = (threadIdx.x & 63) >> 5;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int f = 32 * fb + 8 * (r / 4) + 4 * half + (r % 4);
      const float v = acc[nb][r];
      if (f < NEDF_CLS_COARSE) {
        if (v > st[nb][0]) { st[nb][0] = v; st[nb][1] = float(f); }
      } else if (f < NEDF_CLS_COARSE + NEDF_CLS_FINE) {
        if (v > st[nb][2]) { st[nb][2] = v; st[nb][3] = float(f - NEDF_CLS_COARSE); }
      } else if (f == NEDF_CLS_HIT_ROW) {
        st[nb][4] = v;
      }
    }
  }
}

// Forces the B-operand words written by epi_hidden(fb) to be computed before
// this point in the instruction stream (an empty volatile asm that reads them).
template <int DT, int NB, int KSO>
__device__ __forceinline__ void pin_block(int fb, typename Tr<DT>::frag (&Bout)[NB][KSO]) {
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if constexpr (DT == 3) {
      asm volatile("" ::"v"(Bout[nb][fb / 2].v[(fb % 2) * 4 + 0]), "v"(Bout[nb][fb / 2].v[(fb % 2) * 4 + 1]),
                   "v"(Bout[nb][fb / 2].v[(fb % 2) * 4 + 2]), "v"(Bout[nb][fb / 2].v[(fb % 2) * 4 + 3]),
                   "v"(Bout[nb][fb / 2].sc));
    } else if constexpr (DT == 2) {
      asm volatile("" ::"v"(Bout[nb][fb / 2][(fb % 2) * 4 + 0]), "v"(Bout[nb][fb / 2][(fb % 2) * 4 + 1]),
                   "v"(Bout[nb][fb / 2][(fb % 2) * 4 + 2]), "v"(Bout[nb][fb / 2][(fb % 2) * 4 + 3]));
    } else if constexpr (DT == 1) {
      asm volatile("" ::"v"(Bout[nb][2 * fb]), "v"(Bout[nb][2 * fb + 1]));
    } else {
#pragma unroll
      for (int r = 0; r < 16; r += 4)
        asm volatile("" ::"v"(Bout[nb][16 * fb + r]), "v"(Bout[nb][16 * fb + r + 1]), "v"(Bout[nb][16 * fb + r + 2]),
                     "v"(Bout[nb][16 * fb + r + 3]));
    }
  }
}

// ---- one layer -----------------------------------------------------------
// Output blocks are streamed in "superchunks" of SB consecutive chunks (one
// barrier per superchunk; the chunks of a layer are contiguous in the blob).
// Default chunks per superchunk by dtype (the autotuner may pick another
// instantiated value).
template <int DT> constexpr int sb_default() { return DT == 0 ? 1 : DT == 1 ? 2 : 4; }
// Chunks per superchunk of a layer with fb chunks when sbx are requested:
// the largest power of two <= sbx dividing fb with at least two superchunks.
constexpr int sb_for(int fb, int sbx) {
  int s = sbx;
  while (s > 1 && (fb % s != 0 || fb / s < 2)) s /= 2;
  return s;
}
// LDS bytes of one ring slot for chunks of at most `chunk` bytes.
constexpr int slot_bytes(int chunk, int sbx) { return chunk * sbx; }

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1.
template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// Multiplies the FB chunks of a layer (KS_IN K-steps each, CB_THIS bytes)
// against Bin.  Superchunk 0 must be in LDS slot `cur` on entry and
// superchunk 1 in flight into the next slot; superchunk sc + 2 (of this
// layer, or of the following one at w_next: FB_NEXT chunks of CB_NEXT bytes)
// is started while superchunk sc is multiplied.
//
// Within a superchunk the LDS reads form one fixed sequence of read groups,
// per block: bias (4 reads), fragment groups of up to G reads, and for the
// head modes one group per head row; D groups are kept in flight ahead of the
// group being consumed.
// MODE 0: hidden epilogue into Bout.  MODE 1: head epilogue.  MODE 2: both.
// MODE 3: residual epilogue into Bout (Bout holds the stream on entry).
// MODE 4: classifier epilogue into `partial` (see epi_argmax).
template <int DT, int NB, int KS_IN, int FB, int CB_THIS, int CB_NEXT, int KSO, int NOUT, int MODE,
          int CHUNK, int FB_NEXT = FB, int SBX = sb_default<DT>(), int NW = WAVES>
__device__ __forceinline__ void layer(const typename Tr<DT>::frag (&Bin)[NB][KS_IN],
                                      typename Tr<DT>::frag (&Bout)[NB][KSO], const uint8_t* w_this,
                                      const uint8_t* w_next, uint8_t* lds, int& cur,
                                      float (&partial)[NB][NOUT], float2 qscale = make_float2(1.f, 1.f)) {
  using T = Tr<DT>;
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  constexpr int SLOT = slot_bytes(CHUNK, SBX);
  constexpr int SB = sb_for(FB, SBX);
  constexpr int NSC = FB / SB;
  constexpr int SB_N = sb_for(FB_NEXT, SBX);
  constexpr int SCB = SB * CB_THIS;
  constexpr int SCB_N = SB_N * CB_NEXT;
  static_assert(FB % SB == 0 && NSC >= 2, "layer must span at least two superchunks");
  static_assert(SCB <= SLOT && SCB_N <= SLOT, "LDS slot too small");
  static_assert(SCB < 65536, "LDS read offsets are 16-bit");
  constexpr int R = KS_IN * T::FRAG / 1024;  // 16-byte-per-lane LDS reads per chunk
  static_assert((KS_IN * T::FRAG) % 1024 == 0, "K-steps must fill whole LDS reads");
  constexpr int G = 4;
  constexpr int NG = (R + G - 1) / G;
  constexpr int NH = (MODE == 1 || MODE == 2) ? NOUT : 0;
  constexpr bool MX = (DT == 3);    // one more read per block: the weight-block scales
  constexpr int PER = 1 + (MX ? 1 : 0) + NG + NH;  // read groups per block
  constexpr int E = SB * PER;       // read groups per superchunk
  constexpr int D = 3;              // groups issued ahead of consumption
  constexpr int SCALES = KS_IN * T::FRAG;
  constexpr int BIAS = SCALES + mx_scale_bytes<DT>();
  // hidden-layer epilogues are deferred by one block so that their vector
  // work overlaps the next block's matrix ops
  constexpr bool DEFER = (MODE == 0 || MODE == 3);
  auto epi_deferred = [&](int fbx, const f32x16_t(&ax)[NB]) __attribute__((always_inline)) {
    if constexpr (MODE == 3) epi_residual<DT, NB, KSO>(fbx, ax, Bout);
    else epi_hidden<DT, NB, KSO>(fbx, ax, Bout, qscale);
  };
  f32x16_t prev[NB];
  // Read groups of a superchunk in consumption order: the bias of its first
  // block, then per block k its fragment groups, with the bias of block k + 1
  // placed before block k's last fragment group (so that initialising the
  // next accumulator overlaps block k's last matrix ops), then block k's head
  // rows.  kind 0 bias, 1 fragment group (idx g), 2 head row (idx o), 3 the
  // block's weight-block scales (MX; one read, right after its bias).
  struct Grp {
    int kind, k, idx;
  };
  constexpr auto grp = [](int e) constexpr {
    int n = 0;
    for (int k = 0; k < SB; ++k) {
      if (k == 0) {
        if (n == e) return Grp{0, 0, 0};
        ++n;
        if (MX) {
          if (n == e) return Grp{3, 0, 0};
          ++n;
        }
      }
      for (int g = 0; g < NG; ++g) {
        if (g == NG - 1 && k + 1 < SB) {
          if (n == e) return Grp{0, k + 1, 0};
          ++n;
          if (MX) {
            if (n == e) return Grp{3, k + 1, 0};
            ++n;
          }
        }
        if (n == e) return Grp{1, k, g};
        ++n;
      }
      for (int o = 0; o < NH; ++o) {
        if (n == e) return Grp{2, k, o};
        ++n;
      }
    }
    return Grp{-1, 0, 0};
  };
  // number of reads of group e
  constexpr auto cnt = [grp](int e) constexpr {
    if (e >= E) return 0;
    const Grp q = grp(e);
    if (q.kind == 3) return 1;
    if (q.kind != 1) return 4;
    return R - q.idx * G < G ? R - q.idx * G : G;
  };
  u32x4 ring[D][G];
  // issue the reads of group e of the superchunk at LDS byte address `base`
  auto issue = [&](auto ec, uint32_t base) __attribute__((always_inline)) {
    constexpr int e = decltype(ec)::value;
    if constexpr (e < E) {
      constexpr Grp q = grp(e);
      constexpr int k = q.k;
      u32x4(&dst)[G] = ring[e % D];
      const uint32_t fbase = base + uint32_t(lane) * 16u;  // fragment reads
      const uint32_t bbase = base + uint32_t(half) * 64u;  // bias and head rows
      if constexpr (q.kind == 0) {
        static_for<4>([&](auto qc) __attribute__((always_inline)) {
          constexpr int i = decltype(qc)::value;
          dst[i] = lds_read16<k * CB_THIS + BIAS + 16 * i>(bbase);
        });
      } else if constexpr (q.kind == 1) {
        constexpr int g = q.idx;
        static_for<cnt(e)>([&](auto rc) __attribute__((always_inline)) {
          constexpr int r = decltype(rc)::value;
          dst[r] = lds_read16<k * CB_THIS + (g * G + r) * 1024>(fbase);
        });
      } else if constexpr (q.kind == 3) {
        dst[0] = lds_read16<k * CB_THIS + SCALES>(fbase);
      } else {
        constexpr int o = q.idx;
        static_for<4>([&](auto qc) __attribute__((always_inline)) {
          constexpr int i = decltype(qc)::value;
          dst[i] = lds_read16<k * CB_THIS + BIAS + 128 + 128 * o + 16 * i>(bbase);
        });
      }
    }
  };
  // accumulators alternate between consecutive blocks of a superchunk
  f32x16_t acc2[2][NB];
  uint32_t wsc2[2] = {0u, 0u};  // MX: the lane's weight-block scales of those blocks
  // consume group e (already in registers cw) of superchunk sc
  auto consume = [&](auto ec, int sc, const u32x4(&cw)[G]) __attribute__((always_inline)) {
    constexpr int e = decltype(ec)::value;
    constexpr Grp q = grp(e);
    constexpr int k = q.k;
    f32x16_t(&acc)[NB] = acc2[k & 1];
    const int fb = sc * SB + k;
    if constexpr (q.kind == 0) {
      f32x16_t b0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        b0[4 * i + 0] = __uint_as_float(cw[i].x); b0[4 * i + 1] = __uint_as_float(cw[i].y);
        b0[4 * i + 2] = __uint_as_float(cw[i].z); b0[4 * i + 3] = __uint_as_float(cw[i].w);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = b0;
    } else if constexpr (q.kind == 1) {
      constexpr int g = q.idx;
      mma_group<DT, NB, KS_IN, G>(cw, g * G, R, Bin, acc, wsc2[k & 1]);
      if constexpr (DEFER && g == 0) {
        if (fb > 0) epi_deferred(fb - 1, prev);
      }
      // interleave vector work (epilogues, accumulator set-up) with the
      // matrix ops instead of letting it pile up between two of them
      static_for<mma_per_group<DT, NB, G>()>([&](auto) __attribute__((always_inline)) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix op
        __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);  // up to five VALU ops
      });
      if constexpr (g == NG - 1) {
        if constexpr (DEFER) {
          // the previous block's epilogue must be finished by the end of
          // this block (otherwise the compiler sinks every epilogue of the
          // layer to its end, holding all accumulators live)
          if (fb > 0) pin_block<DT, NB, KSO>(fb - 1, Bout);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) prev[nb] = acc[nb];
        } else if constexpr (MODE == 2) {
          epi_hidden<DT, NB, KSO>(fb, acc, Bout, qscale);
        } else if constexpr (MODE == 4) {
          epi_argmax<NB, NOUT>(fb, acc, partial);
        }
      }
    } else if constexpr (q.kind == 3) {
      wsc2[k & 1] = cw[0].x;
    } else {
      // head row o: partial[nb][o] += w . relu(real(acc))
      constexpr int o = q.idx;
      const float tr = qscale.x;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          float s = partial[nb][o];
          s = fmaf(__uint_as_float(cw[i].x), fmaxf(acc[nb][4 * i + 0] * tr, 0.0f), s);
          s = fmaf(__uint_as_float(cw[i].y), fmaxf(acc[nb][4 * i + 1] * tr, 0.0f), s);
          s = fmaf(__uint_as_float(cw[i].z), fmaxf(acc[nb][4 * i + 2] * tr, 0.0f), s);
          s = fmaf(__uint_as_float(cw[i].w), fmaxf(acc[nb][4 * i + 3] * tr, 0.0f), s);
          partial[nb][o] = s;
        }
      }
      // computed here, not sunk past the layer with the head rows held live
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) asm volatile("" : "+v"(partial[nb][o]));
    }
  };
  // the first D groups of superchunk 0
  {
    const uint32_t base0 = lds_offset(lds + cur * SLOT);
    static_for<D>([&](auto ec) __attribute__((always_inline)) { issue(ec, base0); });
  }
#pragma unroll
  for (int sc = 0; sc < NSC; ++sc) {
    // superchunk sc is in slot `cur` (its first D groups already issued),
    // sc + 1 in flight into cur + 1; start sc + 2 (this layer, or the
    // following one at w_next) into the slot sc - 1 used
    const int nslot = cur + 2 >= NBUF ? cur + 2 - NBUF : cur + 2;
    uint8_t* nbuf = lds + nslot * SLOT;
    bool issued = false;
    if (sc + 2 < NSC) {
      dma_chunk<SCB, NW>(w_this + size_t(sc + 2) * SCB, nbuf);
      issued = true;
    } else if (w_next != nullptr) {
      if constexpr (CB_NEXT > 0) {
        dma_chunk<SCB_N, NW>(w_next + size_t(sc + 2 - NSC) * SCB_N, nbuf);
        issued = true;
      }
    }
    const uint32_t base = lds_offset(lds + cur * SLOT);
    static_for<E>([&](auto ec) __attribute__((always_inline)) {
      constexpr int e = decltype(ec)::value;
      u32x4(&cw)[G] = ring[e % D];
      // groups e + 1 .. e + D - 1 may stay in flight
      constexpr int after = cnt(e + 1) + cnt(e + 2);
      static_assert(D == 3, "wait count assumes three groups in flight");
      lds_wait4<after>(cw[0], cw[1], cw[2], cw[3]);
      if constexpr (e + 1 < E) {
        consume(ec, sc, cw);
        issue(std::integral_constant<int, e + D>{}, base);
      } else if (sc + 1 < NSC) {
        // last group of a superchunk that is not the layer's last: every
        // read of this superchunk has completed, so pass the barrier first,
        // start the next superchunk's reads, and only then run this
        // group's matrix ops, which cover the reads' latency
        u32x4 tail[G] = {cw[0], cw[1], cw[2], cw[3]};
        // superchunk sc + 1 must have landed; sc + 2's copies may stay in flight
        if (issued) {
          if (sc + 2 < NSC) dma_wait_barrier_n<dma_instr(SCB, NW)>();
          else dma_wait_barrier_n<dma_instr(SCB_N > 0 ? SCB_N : 1024, NW)>();
        } else {
          dma_wait_barrier();
        }
        const uint32_t nbase = lds_offset(lds + (cur + 1 >= NBUF ? cur + 1 - NBUF : cur + 1) * SLOT);
        static_for<D>([&](auto gc) __attribute__((always_inline)) { issue(gc, nbase); });
        // the matrix ops below may not move above the reads just issued
        asm volatile("" : "+v"(tail[0]), "+v"(tail[1]), "+v"(tail[2]), "+v"(tail[3]));
        consume(ec, sc, tail);
      } else {
        consume(ec, sc, cw);
      }
    });
    if (sc + 1 == NSC) {
      // the layer's last superchunk: the next layer's first superchunk must
      // have landed; its second may stay in flight
      if (issued) {
        if (sc + 2 < NSC) dma_wait_barrier_n<dma_instr(SCB, NW)>();
        else dma_wait_barrier_n<dma_instr(SCB_N > 0 ? SCB_N : 1024, NW)>();
      } else {
        dma_wait_barrier();
      }
    }
    cur = cur + 1 >= NBUF ? cur + 1 - NBUF : cur + 1;
  }
  if constexpr (DEFER) epi_deferred(FB - 1, prev);
}

// ---- whole trunk ------------------------------------------------------------
// Hidden layers 0..NHID-1 of the blob on the encoded input Benc; the head dot
// products accumulate into `partial` (each lane half over its own features;
// the caller adds the halves).  With KEEP_LAST the last hidden activation is
// also left in Blast as a B operand (input of the colour layer of FB_AFTER
// chunks of CB_AFTER bytes at w_after, whose first two superchunks are
// prefetched).  Otherwise,
// when next_blob is given (a blob of the same shape), the last layer
// prefetches that network's first two superchunks so that the next pass can
// start with primed = true.  *cur_io is the LDS slot of the pass's first
// superchunk.  The caller's LDS array holds NBUF slots of slot_bytes(CHUNK,
// SBX) bytes.
template <int DT, int WIDTH, int KS0, int NHID, int NOUT, int CHUNK, bool KEEP_LAST, int CB_AFTER,
          int FB_AFTER = WIDTH / 32, int SBX = sb_default<DT>(), int NB = Tr<DT>::NB, int NW = WAVES>
__device__ __forceinline__ void trunk(const nedf_blob_header* hb, const uint8_t* blob,
                                      const typename Tr<DT>::frag (&Benc)[NB][KS0],
                                      uint8_t* lds, float (&partial)[NB][NOUT],
                                      typename Tr<DT>::frag (&Blast)[NB][WIDTH / Tr<DT>::KPS],
                                      const uint8_t* w_after, int* cur_io = nullptr,
                                      const uint8_t* next_blob = nullptr, bool primed = false) {
  using T = Tr<DT>;
  constexpr int FB = WIDTH / 32;
  constexpr int KSH = WIDTH / T::KPS;
  constexpr int CB0 = chunk_bytes<DT>(KS0, 0);
  constexpr int CBH = chunk_bytes<DT>(KSH, 0);
  constexpr int CBL = chunk_bytes<DT>(KSH, NOUT);
  static_assert(NHID >= 3, "need at least three hidden layers");
  static_assert(CHUNK >= CB0 && CHUNK >= CBL, "LDS chunk buffer too small");
  typename T::frag X[NB][KSH], Y[NB][KSH];
  int cur = cur_io ? *cur_io : 0;
  // header fields are read through the scalar cache (see uniform_load_u64)
  auto off = [&](int L) { return uniform_load_u64(&hb->off_layer[L]); };
  // FP8: per-layer (to-real multiplier, inverse scale of the next input)
  const float* qsc = reinterpret_cast<const float*>(blob + (DT == 2 ? uniform_load_u64(&hb->off_scales) : 0));
  auto QS = [&](int L) {
    return DT == 2 ? make_float2(uniform_load_f32(qsc + 1 + 2 * L), uniform_load_f32(qsc + 2 + 2 * L))
                   : make_float2(1.f, 1.f);
  };
  constexpr int SLOT = slot_bytes(CHUNK, SBX);
  constexpr int SC0 = sb_for(FB, SBX) * CB0;  // first-layer superchunk bytes
  if (!primed) {
    dma_chunk<SC0, NW>(blob + off(0), lds + cur * SLOT);
    dma_chunk<SC0, NW>(blob + off(0) + SC0, lds + (cur + 1 >= NBUF ? cur + 1 - NBUF : cur + 1) * SLOT);
    dma_wait_barrier_n<dma_instr(SC0, NW)>();
  }
  // chunks after the last hidden layer: the colour layer, or the next pass
  constexpr int CB_TAIL = KEEP_LAST ? CB_AFTER : CB0;
  constexpr int FB_TAIL = KEEP_LAST ? FB_AFTER : FB;
  const uint8_t* w_tail = KEEP_LAST ? w_after : (next_blob ? next_blob + off(0) : nullptr);
  // layer 0: encoding -> X; then pairs X -> Y -> X; the last layer feeds the head
  layer<DT, NB, KS0, FB, CB0, CBH, KSH, NOUT, 0, CHUNK, FB, SBX, NW>(Benc, X, blob + off(0), blob + off(1), lds, cur,
                                                       partial, QS(0));
  constexpr int PAIRS = (NHID - 2) / 2;
  for (int p = 0; p < PAIRS; ++p) {
    const int L = 1 + 2 * p;
    layer<DT, NB, KSH, FB, CBH, CBH, KSH, NOUT, 0, CHUNK, FB, SBX, NW>(X, Y, blob + off(L), blob + off(L + 1), lds, cur,
                                                         partial, QS(L));
    if ((NHID - 2) % 2 == 0 && p == PAIRS - 1) {
      layer<DT, NB, KSH, FB, CBH, CBL, KSH, NOUT, 0, CHUNK, FB, SBX, NW>(Y, X, blob + off(L + 1), blob + off(L + 2), lds,
                                                           cur, partial, QS(L + 1));
    } else {
      layer<DT, NB, KSH, FB, CBH, CBH, KSH, NOUT, 0, CHUNK, FB, SBX, NW>(Y, X, blob + off(L + 1), blob + off(L + 2), lds,
                                                           cur, partial, QS(L + 1));
    }
  }
  constexpr int LAST_MODE = KEEP_LAST ? 2 : 1;
  if constexpr ((NHID - 2) % 2 == 1) {
    layer<DT, NB, KSH, FB, CBH, CBL, KSH, NOUT, 0, CHUNK, FB, SBX, NW>(X, Y, blob + off(NHID - 2), blob + off(NHID - 1),
                                                         lds, cur, partial, QS(NHID - 2));
    layer<DT, NB, KSH, FB, CBL, CB_TAIL, KSH, NOUT, LAST_MODE, CHUNK, FB_TAIL, SBX, NW>(Y, Blast, blob + off(NHID - 1), w_tail,
                                                                     lds, cur, partial, QS(NHID - 1));
  } else {
    layer<DT, NB, KSH, FB, CBL, CB_TAIL, KSH, NOUT, LAST_MODE, CHUNK, FB_TAIL, SBX, NW>(X, Blast, blob + off(NHID - 1), w_tail,
                                                                     lds, cur, partial, QS(NHID - 1));
  }
  if (cur_io) *cur_io = cur;
}

// ---- first-layer encoding ----------------------------------------------------
// Slot a holds sin(pi (2^level p_comp + h / 2)) for a < n L (h = 0 gives
// sin, h = 1 cos), then the identity components two per slot, then zeros.
// plo carries residuals of the components (p + plo their values to beyond
// single precision; zero for inputs exact as given): the scaled residual
// joins the sine's argument after the exact period reduction, so a
// top-level feature is not off by 2^level times p's rounding.
template <int N, int L>
__device__ __forceinline__ float enc_slot(const float (&p)[N], const float (&plo)[N], int a, int half) {
  if (a < N * L) {
    const int level = a / N, comp = a % N;
    return sinpi_hw(float(1 << level) * p[comp], float(1 << level) * plo[comp], half);
  }
  const int i = a - N * L;
  if (i >= (N + 1) / 2) return 0.0f;
  if (2 * i + 1 < N) return half ? p[2 * i + 1] : p[2 * i];
  return half ? 0.0f : p[2 * i];
}

template <int DT, int N, int L, int KS0>
__device__ __forceinline__ void encode_input(const float (&p)[N], const float (&plo)[N], int half,
                                             typename Tr<DT>::frag (&B)[KS0], float inv_scale = 1.0f) {
  if constexpr (DT == 3) {
    // MX: the 16 slots of each block from both lane halves share a scale
#pragma unroll
    for (int ks = 0; ks < KS0; ++ks) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        float v[16];
        float mx = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          v[i] = enc_slot<N, L>(p, plo, 32 * ks + 16 * b + i, half);
          mx = fmaxf(mx, fabsf(v[i]));
        }
        mx = fmaxf(mx, __shfl_xor(mx, 32));
        int byte;
        float inv;
        mx_scale(mx, byte, inv);
        int w[4];
        mx_pack16(v, inv, w);
#pragma unroll
        for (int q = 0; q < 4; ++q) B[ks].v[4 * b + q] = w[q];
        if (half == b) B[ks].sc = byte;
      }
    }
    (void)inv_scale;
  } else if constexpr (DT == 2) {
    // 32 slots per K-step and lane half, quantised to E4M3 with the
    // input's activation scale
#pragma unroll
    for (int ks = 0; ks < KS0; ++ks) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          v[j] = fminf(fmaxf(enc_slot<N, L>(p, plo, 32 * ks + 4 * q + j, half) * inv_scale, -448.0f), 448.0f);
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
        B[ks][q] = w;
      }
    }
  } else if constexpr (DT == 1) {
#pragma unroll
    for (int ks = 0; ks < KS0; ++ks) {
      bf16x8_t v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = static_cast<__bf16>(enc_slot<N, L>(p, plo, 8 * ks + j, half));
      B[ks] = v;
    }
  } else {
#pragma unroll
    for (int ks = 0; ks < KS0; ++ks) B[ks] = enc_slot<N, L>(p, plo, ks, half);
  }
}
// Inputs exact as given (positions, directions).
template <int DT, int N, int L, int KS0>
__device__ __forceinline__ void encode_input(const float (&p)[N], int half, typename Tr<DT>::frag (&B)[KS0],
                                             float inv_scale = 1.0f) {
  float plo[N];
#pragma unroll
  for (int i = 0; i < N; ++i) plo[i] = 0.0f;
  encode_input<DT, N, L, KS0>(p, plo, half, B, inv_scale);
}

// K-steps of an encoded input with n components and L levels.
template <int DT>
constexpr int ks_for_slots(int slots) {
  return DT >= 2 ? (slots + 31) / 32 : DT == 1 ? (slots + 7) / 8 : (slots + 3) / 4 * 4;
}

}  // namespace eng
