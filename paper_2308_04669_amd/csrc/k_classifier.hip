// Intersection network in the multi-level classifier form (Sec. "Intersection
// network", Eq. 3-4; appendix architecture) on the matrix cores.
//
// A wave takes 32 (ray, instance) pairs of one object.  Each pair's 16 line
// points are encoded in registers one point at a time and multiplied at once
// into all eight accumulator blocks of the head layer (the 1,008-wide encoded
// input never exists as a whole: K-outer order, weights streamed through the
// same three-slot LDS ring as the other matrix-core kernels), so the input
// costs 16 B-operand registers instead of 252.  The residual stream then stays
// in registers as the B operand of the 32 block layers (residual addition in
// the second layer's epilogue), and the tail's epilogue keeps a running
// first-maximum over the coarse and fine bins, so that only (coarse bin, fine
// bin, hit logit) leave the network.  Routing, depth and the fallback list
// are those of the regression network.
#include "pipeline.h"
#include "runtime.h"

namespace nedf {
namespace {

template <int DT>
struct ClsCfg {
  using T = eng::Tr<DT>;
  static constexpr int WIDTH = 256;
  static constexpr int L = 10;
  static constexpr int KSH = WIDTH / T::KPS;     // K-steps of a block layer
  static constexpr int KSP = DT == 1 ? 4 : 32;    // K-steps per point (32 argument slots)
  static constexpr int KSC = DT == 1 ? 4 : 16;    // K-steps per head chunk
  static constexpr int CPP = KSP / KSC;           // head chunks per point
  static constexpr int NHC = NEDF_CLS_POINTS * CPP;
  static constexpr int HCB = 8 * KSC * T::FRAG;   // head chunk: 8 blocks x 4 reads of 1 KB
  static constexpr int CBH = KSH * T::FRAG + 128; // block-layer and tail chunk
  static constexpr int SBX = eng::sb_default<DT>();
  static constexpr int SLOT = eng::slot_bytes(CBH, SBX);
  static constexpr int SCB1 = eng::sb_for(8, SBX) * CBH;  // first block layer's superchunk
  // head chunks are copied with 128 bytes more than they hold (read from
  // what follows them in the blob, written into the slot's spare bytes), so
  // that a head copy and a block-layer superchunk copy take the same number
  // of copy instructions and every wait in the head loop counts the same
  static constexpr int HDMA = HCB + 128;
  static_assert(HCB == 32768, "head chunk layout");
  static_assert(HDMA <= SLOT, "head chunk copy must fit an LDS slot");
  static_assert(eng::dma_instr(HDMA) == eng::dma_instr(SCB1), "uniform copy count in the head loop");
};

template <int DT, int NW>
__global__ __launch_bounds__(64 * NW, 1) void k_nedf_cls(KArgs a) {
  using C = ClsCfg<DT>;
  using T = eng::Tr<DT>;
  using frag = typename T::frag;
  constexpr int KSH = C::KSH;
  constexpr int SLOT = C::SLOT;
  constexpr int NWAIT = eng::dma_instr(C::HDMA, NW);
  __shared__ __attribute__((aligned(16))) uint8_t lds[eng::NBUF * SLOT];
  constexpr int NT = 64 * NW;
  __shared__ __attribute__((aligned(16))) uint8_t s_stash[16 * NT];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
  const uint32_t stash = eng::lds_offset(s_stash) + 16u * threadIdx.x;
  PairList* PL = a.L;  // the current depth slab
  PairList* FBL = &a.C->B;
  const int total = PL->total_items;
  if (threadIdx.x == 0) s_item = atomicAdd(&PL->work_counter, 1);
  __syncthreads();
  int item = s_item;
  int cur = 0;
  bool primed = false;
  int n_hit = 0, n_fb = 0, n_miss = 0;
  while (item < total) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(&PL->work_counter, 1);
    __syncthreads();
    const int next = s_item;
    const int obj = item_object(PL, a.n_obj, item);
    const int first = (item - PL->item_start[obj]) * (32 * NW) + wave * 32 + (lane & 31);
    const ObjDesc& od = a.obj[obj];
    const uint8_t* blob = od.nedf_blob;
    const nedf_cls_header* hc = reinterpret_cast<const nedf_cls_header*>(blob);
    const uint8_t* next_blob = next < total ? a.obj[item_object(PL, a.n_obj, next)].nedf_blob : nullptr;
    const float l = od.bound;
    const uint8_t* head = blob + uniform_load_u64(&hc->off_head);
    const float* hbias = reinterpret_cast<const float*>(blob + uniform_load_u64(&hc->off_head_bias));
    const uint8_t* hid = blob + uniform_load_u64(&hc->off_hidden);
    const uint64_t hstride = uniform_load_u64(&hc->hidden_layer_bytes);
    const uint8_t* tail = blob + uniform_load_u64(&hc->off_tail);
    const int nblk = int(uniform_load_u32(&hc->n_blocks));
    // ---- the pair's line
    const bool valid = first < PL->cnt[obj];
    const uint2 pr = a.pairs[PL->off[obj] + (valid ? first : 0)];
    f2 q[3], dv[3];
    {
      const W2L g = load_w2l(a.w2l, int(pr.y));
      float o[3], d[3], dlo[3], ol[3];
      make_ray(a.rays, pr.x, o, d, dlo);
      float tperp;
      local_points_frame(g, o, d, dlo, l, q, dv, tperp, ol);
      const bool inside = ol[0] * ol[0] + ol[1] * ol[1] + ol[2] * ol[2] < l * l;
      // ray and instance ids (flags in bit 31), t_perp and s, parked in LDS
      // across the network
      eng::lds_write16(stash, eng::u32x4{pr.x | (valid ? 0x80000000u : 0u), pr.y | (inside ? 0x80000000u : 0u),
                                         __float_as_uint(tperp), __float_as_uint(g.s)});
    }
    // ---- head: acc[fb] = bias, then point by point
    f32x16_t acc[8][1];
#pragma unroll
    for (int fb = 0; fb < 8; ++fb) {
      const float4* bp = reinterpret_cast<const float4*>(hbias + (fb * 2 + half) * 16);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float4 v = bp[i];
        acc[fb][0][4 * i + 0] = v.x;
        acc[fb][0][4 * i + 1] = v.y;
        acc[fb][0][4 * i + 2] = v.z;
        acc[fb][0][4 * i + 3] = v.w;
      }
    }
    if (!primed) {
      eng::dma_chunk<C::HDMA, NW>(head, lds + cur * SLOT);
      eng::dma_chunk<C::HDMA, NW>(head + C::HCB, lds + (cur + 1 >= eng::NBUF ? cur + 1 - eng::NBUF : cur + 1) * SLOT);
      eng::dma_wait_barrier_n<NWAIT>();
    }
    int half_v = half;
    asm volatile("" : "+v"(half_v));
    for (int p = 0; p < NEDF_CLS_POINTS; ++p) {
      // point p, divided by l: q + c_p d with c_p = (2p + 1) / 16 - 1 (exact)
      const float cp = float(2 * p + 1) * 0.0625f - 1.0f;
      float x[3], xlo[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
#pragma clang fp contract(off)
        const f2 pp = two_prod(cp, dv[r].hi);
        const f2 sm = two_sum(q[r].hi, pp.hi);
        x[r] = sm.hi;
        xlo[r] = sm.lo + ((pp.lo + q[r].lo) + cp * dv[r].lo);
      }
      eng::static_for<C::CPP>([&](auto ccc) __attribute__((always_inline)) {
        constexpr int cc = decltype(ccc)::value;
        const int c = p * C::CPP + cc;
        // copy chunk c + 2 (a head chunk, or a superchunk of the first block
        // layer) into the slot chunk c - 1 used
        const int t = c + 2;
        uint8_t* nbuf = lds + (cur + 2 >= eng::NBUF ? cur + 2 - eng::NBUF : cur + 2) * SLOT;
        if (t < C::NHC) eng::dma_chunk<C::HDMA, NW>(head + size_t(t) * C::HCB, nbuf);
        else eng::dma_chunk<C::SCB1, NW>(hid + size_t(t - C::NHC) * C::SCB1, nbuf);
        // this chunk's K-steps of the point's encoding
        frag B[C::KSC];
        if constexpr (DT == 1) {
#pragma unroll
          for (int ks = 0; ks < C::KSC; ++ks) {
            bf16x8_t v;
#pragma unroll
            for (int j = 0; j < 8; ++j)
              v[j] = static_cast<__bf16>(eng::enc_slot<3, C::L>(x, xlo, 8 * (cc * C::KSC + ks) + j, half_v));
            B[ks] = v;
          }
        } else {
#pragma unroll
          for (int ks = 0; ks < C::KSC; ++ks) B[ks] = eng::enc_slot<3, C::L>(x, xlo, cc * C::KSC + ks, half_v);
        }
        // 8 blocks x 4 reads; the next block's reads are in flight while a
        // block multiplies
        const uint32_t fbase = eng::lds_offset(lds + cur * SLOT) + uint32_t(lane) * 16u;
        eng::u32x4 w[2][4];
        eng::static_for<4>([&](auto rc) __attribute__((always_inline)) {
          constexpr int r = decltype(rc)::value;
          w[0][r] = eng::lds_read16<r * 1024>(fbase);
        });
        eng::static_for<8>([&](auto fbc) __attribute__((always_inline)) {
          constexpr int fb = decltype(fbc)::value;
          eng::u32x4(&cw)[4] = w[fb & 1];
          if constexpr (fb + 1 < 8) {
            eng::static_for<4>([&](auto rc) __attribute__((always_inline)) {
              constexpr int r = decltype(rc)::value;
              w[(fb + 1) & 1][r] = eng::lds_read16<((fb + 1) * 4 + r) * 1024>(fbase);
            });
            eng::lds_wait4<4>(cw[0], cw[1], cw[2], cw[3]);
          } else {
            eng::lds_wait4<0>(cw[0], cw[1], cw[2], cw[3]);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int i = 0; i < T::KPR; ++i) acc[fb][0] = T::mma(T::pick(cw[r], i), B[r * T::KPR + i], acc[fb][0]);
          }
        });
        // chunk c + 1 must have landed (c + 2 may stay in flight)
        eng::dma_wait_barrier_n<NWAIT>();
        cur = cur + 1 >= eng::NBUF ? cur + 1 - eng::NBUF : cur + 1;
      });
    }
    // ---- residual blocks and tail
    frag X[1][KSH], Tm[1][KSH];
#pragma unroll
    for (int fb = 0; fb < 8; ++fb) eng::epi_hidden<DT, 1, KSH>(fb, acc[fb], X, make_float2(1.f, 1.f));
    float st[1][5] = {{-INFINITY, 0.f, -INFINITY, 0.f, 0.f}};
    for (int b = 0; b < nblk; ++b) {
      const uint8_t* w1 = hid + size_t(2 * b) * hstride;
      const uint8_t* w2 = w1 + hstride;
      eng::layer<DT, 1, KSH, 8, C::CBH, C::CBH, KSH, 5, 0, C::CBH, 8, C::SBX, NW>(X, Tm, w1, w2, lds, cur, st);
      if (b + 1 < nblk)
        eng::layer<DT, 1, KSH, 8, C::CBH, C::CBH, KSH, 5, 3, C::CBH, 8, C::SBX, NW>(Tm, X, w2, w2 + hstride, lds, cur,
                                                                                 st);
      else
        eng::layer<DT, 1, KSH, 8, C::CBH, C::CBH, KSH, 5, 3, C::CBH, NEDF_CLS_TAIL_BLOCKS, C::SBX, NW>(
            Tm, X, w2, tail, lds, cur, st);
    }
    const uint8_t* next_head =
        next_blob ? next_blob + uniform_load_u64(&reinterpret_cast<const nedf_cls_header*>(next_blob)->off_head)
                  : nullptr;
    eng::layer<DT, 1, KSH, NEDF_CLS_TAIL_BLOCKS, C::CBH, C::HCB, KSH, 5, 4, C::CBH, 3, C::SBX, NW>(
        X, Tm, tail, next_head, lds, cur, st);
    primed = next_head != nullptr;
    // ---- both lane halves' maxima: the larger, or the lower bin on a tie
    float bc = st[0][0], ic = st[0][1], bfv = st[0][2], ifv = st[0][3];
    {
      const float obc = __shfl_xor(bc, 32), oic = __shfl_xor(ic, 32);
      if (obc > bc || (obc == bc && oic < ic)) { bc = obc; ic = oic; }
      const float obf = __shfl_xor(bfv, 32), oif = __shfl_xor(ifv, 32);
      if (obf > bfv || (obf == bfv && oif < ifv)) { bfv = obf; ifv = oif; }
    }
    const float alpha_hat = st[0][4];  // lane half 0 holds the hit logit
    eng::u32x4 sv = eng::lds_read16<0>(stash), d1 = sv, d2 = sv, d3 = sv;
    eng::lds_wait4<0>(sv, d1, d2, d3);
    const uint2 prs = make_uint2(sv.x & 0x7FFFFFFFu, sv.y & 0x7FFFFFFFu);
    const bool valid_s = (sv.x >> 31) != 0, inside_s = (sv.y >> 31) != 0;
    // S^-1 (Eq. 4): mu = l ((128 c + f) / 4096 - 1), exact up to the final product
    const int cell = int(ic) * NEDF_CLS_FINE + int(ifv);
    const float mu = l * (float(cell) * (1.0f / 4096.0f) - 1.0f);
    const float pp = sigmoidf_(alpha_hat);
    const float D = __uint_as_float(sv.w) * (__uint_as_float(sv.z) - mu);
    const bool mine = valid_s && half == 0;
    const bool to_fb = mine && (inside_s || (pp >= a.p_lo && pp <= a.p_hi));
    const bool hit = mine && !to_fb && pp > a.p_hi && D > 0.0f;
    if (hit) emit_key(a, prs.x, prs.y, D);
    const uint64_t m = __ballot(to_fb);
    if (m) {
      const int leader = __ffsll((unsigned long long)m) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(&FBL->cnt[obj], __popcll(m));
      base = __shfl(base, leader);
      if (to_fb) a.pairsB[FBL->off[obj] + base + __popcll(m & ((1ull << lane) - 1ull))] = prs;
    }
    const uint64_t mh = __ballot(hit), mv = __ballot(mine);
    n_hit += __popcll(mh);
    n_fb += __popcll(m);
    n_miss += __popcll(mv) - __popcll(mh) - __popcll(m);
    item = next;
  }
  if (lane == 0 && (n_hit | n_fb | n_miss)) {
    atomicAdd(&a.C->stats[0], n_hit);
    atomicAdd(&a.C->stats[1], n_fb);
    atomicAdd(&a.C->stats[2], n_miss);
  }
}

}  // namespace

void launch_nedf_cls(const KArgs& k, hipStream_t s, int dtype) {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 256;
  }
  if (dtype == NEDF_BF16) hipLaunchKernelGGL((k_nedf_cls<1, 4>), dim3(ncu), dim3(256), 0, s, k);
  else hipLaunchKernelGGL((k_nedf_cls<0, 4>), dim3(ncu), dim3(256), 0, s, k);
}

}  // namespace nedf
