// Per-pixel stages after the depth buffer: binning hit pixels by object,
// secant refinement of the winning depth, deferred shading (Eq. 8, Alg. 1
// step 2), shadow rays and the shadow multiplier (Alg. 2), composite.
#include <cstring>

#include "pipeline.h"
#include "runtime.h"

namespace nedf {
namespace {

// Segment offsets and work items of list A over the objects in item_mask.
__global__ void k_scan_pixels(KArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  PairList* L = &a.C->A;
  int64_t off = 0;
  int items = 0;
  for (int m = 0; m < a.n_obj; ++m) {
    if (off + L->cnt[m] > a.capacity) {
      L->cnt[m] = int32_t(a.capacity - off > 0 ? a.capacity - off : 0);
      set_status(a.status, NEDF_ERR_CAPACITY);
    }
    L->off[m] = int32_t(off);
    L->item_start[m] = items;
    if ((a.item_mask >> m) & 1u) items += (L->cnt[m] + a.item_pairs - 1) / a.item_pairs;
    L->fill[m] = 0;
    off += L->cnt[m];
  }
  L->off[a.n_obj] = off;
  L->item_start[a.n_obj] = items;
  L->total_items = items;
  L->total_pairs = off;
  L->work_counter = 0;
}

__global__ void k_zero_list(PairList* L) {
  const int i = threadIdx.x;
  if (i < int(sizeof(PairList) / 4)) reinterpret_cast<int32_t*>(L)[i] = 0;
}

// Bin pixels with a valid ID whose object is in `mask` into list A as
// (pixel, instance) pairs; pass 0 counts, pass 1 writes.  A workgroup takes a
// contiguous range of pixels and aggregates its counts per object in LDS
// (lanes of a wave grouped by object, one LDS atomic per group), so global
// atomics are one per (workgroup, object): per-wave global atomics on the
// few counters of list A serialise across the whole chip.
constexpr unsigned BIN_BLOCKS = 1024;

template <int PASS>
__global__ __launch_bounds__(256) void k_bin(KArgs a, const int32_t* ids, uint32_t mask) {
  __shared__ int s_cnt[NEDF_MAX_OBJECTS], s_base[NEDF_MAX_OBJECTS];
  const int t = threadIdx.x, lane = t & 63;
  const int64_t per = ((a.n_rays + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
  const int64_t p0 = int64_t(blockIdx.x) * per;
  const int64_t p1 = p0 + per < a.n_rays ? p0 + per : a.n_rays;
  PairList* L = &a.C->A;
  if (t < NEDF_MAX_OBJECTS) s_cnt[t] = 0;
  __syncthreads();
  // traversal 0 counts; in pass 1 traversal 1 writes
  for (int trav = 0; trav <= PASS; ++trav) {
    for (int64_t pb = p0; pb < p1; pb += 256) {
      const int64_t p = pb + t;
      const int inst = p < p1 ? ids[p] : -1;
      const int obj = inst >= 0 && inst < a.n_inst ? a.inst_object[inst] : -1;
      const bool want = obj >= 0 && obj < a.n_obj && ((mask >> obj) & 1u);
      uint64_t pending = __ballot(want);
      while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int o = __shfl(obj, leader);
        const uint64_t match = __ballot(want && obj == o);
        int off = 0;
        if (lane == leader) off = atomicAdd(&s_cnt[o], __popcll(match));
        if (trav == 1) {
          off = __shfl(off, leader);
          if (want && obj == o) {
            const int pos = s_base[o] + off + __popcll(match & ((1ull << lane) - 1ull));
            if (pos < L->cnt[o]) a.pairs[L->off[o] + pos] = make_uint2(uint32_t(p), uint32_t(inst));
          }
        }
        pending &= ~match;
      }
    }
    __syncthreads();
    if (t < a.n_obj) {
      const int c = s_cnt[t];
      if (PASS == 0) {
        if (c) atomicAdd(&L->cnt[t], c);
      } else if (trav == 0) {
        s_base[t] = c ? atomicAdd(&L->fill[t], c) : 0;
        s_cnt[t] = 0;
      }
    }
    __syncthreads();
  }
}

// ---- secant refinement --------------------------------------------------------
// f(t) = surface function at the local point of world depth t; seeds D -/+ h,
// `steps` secant updates with a [D - 2h, D + 2h] guard (needs steps + 1
// evaluations; the last iterate is not evaluated).
struct Secant {
  float t0, t1, f0, f1, out, lo, hi;
  bool active;
  __device__ void start(float D, float h) {
    t0 = D - h; t1 = D + h; out = D; lo = D - 2.f * h; hi = D + 2.f * h;
  }
  __device__ float update() {  // returns the new iterate (evaluation point)
    const float den = f1 - f0;
    bool ok = active && den != 0.0f;
    const float tn = ok ? t1 - f1 * (t1 - t0) / den : t1;
    ok = ok && tn >= lo && tn <= hi;
    if (ok) out = tn;
    active = ok;
    return tn;
  }
  __device__ void shift(float tn, float fn) {
    if (active) { t0 = t1; f0 = f1; t1 = tn; f1 = fn; }
  }
};

__global__ void k_refine_analytic(KArgs a, uint32_t mask) {
  const PairList* L = &a.C->A;
  for (int m = 0; m < a.n_obj; ++m) {
    if (!((mask >> m) & 1u)) continue;
    const ObjDesc od = a.obj[m];
    const int cnt = L->cnt[m], off = L->off[m];
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
      const uint2 pr = a.pairs[off + q];
      const W2L g = load_w2l(a.w2l, int(pr.y));
      float o[3], d[3], ol[3], dl[3];
      make_ray(a.rays, pr.x, o, d);
      to_local(g, o, d, ol, dl);
      auto f = [&](float t) {
        const float tl = t * g.inv_s;
        const float x = fmaf(tl, dl[0], ol[0]), y = fmaf(tl, dl[1], ol[1]), z = fmaf(tl, dl[2], ol[2]);
        return (od.param[1] - sqrtf(x * x + y * y + z * z)) / od.param[2];
      };
      Secant s;
      s.start(a.depth[pr.x], a.refine_h * g.s);
      s.f0 = f(s.t0);
      s.f1 = f(s.t1);
      s.active = s.f0 < 0.0f && s.f1 >= 0.0f;
      for (int it = 0; it < a.refine_steps; ++it) {
        const float tn = s.update();
        if (it + 1 < a.refine_steps) s.shift(tn, f(tn));
      }
      a.depth[pr.x] = s.out;
    }
  }
}

// Density-network refinement: items of 128 pixels (32 per wave) of one
// SDF-mode object; each evaluation of f is one pass of the trunk.
template <int DT, int WIDTH, int NHID, int L, int SBX, int OCC, int NW>
__global__ __launch_bounds__(64 * NW, OCC) void k_refine_mlp(KArgs a) {
  using T = eng::Tr<DT>;
  constexpr int NB = T::NB;
  constexpr int KS0 = eng::ks_for_slots<DT>(3 * L + 2);
  constexpr int KSH = WIDTH / T::KPS;
  constexpr int CHUNK = eng::cmax(eng::chunk_bytes<DT>(KS0, 0), eng::chunk_bytes<DT>(KSH, 1));
  __shared__ __attribute__((aligned(16))) uint8_t lds[eng::NBUF * eng::slot_bytes(CHUNK, SBX)];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
  PairList* PL = &a.C->A;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&PL->work_counter, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= PL->total_items) break;
    const int obj = item_object(PL, a.n_obj, item);
    const int local = (item - PL->item_start[obj]) * (32 * NW) + wave * 32 + (lane & 31);
    const bool valid = local < PL->cnt[obj];
    const uint2 pr = a.pairs[PL->off[obj] + (valid ? local : 0)];
    const ObjDesc& od = a.obj[obj];
    const uint8_t* blob = od.blob;
    const nedf_blob_header* hb = reinterpret_cast<const nedf_blob_header*>(blob);
    const float head_b = uniform_load_f32(blob + uniform_load_u64(&hb->off_head_b));
    const W2L g = load_w2l(a.w2l, int(pr.y));
    float o[3], d[3], ol[3], dl[3];
    make_ray(a.rays, pr.x, o, d);
    to_local(g, o, d, ol, dl);
    // the item's field evaluations run back to back on one blob: each pass
    // but the last prefetches the next pass's first chunks
    const int n_eval = 2 + (a.refine_steps > 1 ? a.refine_steps - 1 : 0);
    int eval_i = 0, slot = 0;
    bool primed = false;
    auto f = [&](float t) {
      const float tl = t * g.inv_s;
      float p[3] = {fmaf(tl, dl[0], ol[0]), fmaf(tl, dl[1], ol[1]), fmaf(tl, dl[2], ol[2])};
      typename T::frag Benc[NB][KS0];
      eng::encode_input<DT, 3, L, KS0>(p, half, Benc[0]);
      float partial[NB][1] = {{0.f}};
      typename T::frag Blast[NB][KSH];
      const uint8_t* nb_ = ++eval_i < n_eval ? blob : nullptr;
      eng::trunk<DT, WIDTH, KS0, NHID, 1, CHUNK, false, 0, WIDTH / 32, SBX, NB, NW>(hb, blob, Benc, lds, partial,
                                                                                   Blast, nullptr, &slot, nb_, primed);
      primed = nb_ != nullptr;
      const float u = partial[0][0] + __shfl_xor(partial[0][0], 32) + head_b;
      return mlp_surface(od, u, p[0], p[1], p[2]);
    };
    Secant s;
    s.start(a.depth[pr.x], a.refine_h * g.s);
    s.f0 = f(s.t0);
    s.f1 = f(s.t1);
    s.active = s.f0 < 0.0f && s.f1 >= 0.0f;
    for (int it = 0; it < a.refine_steps; ++it) {
      const float tn = s.update();
      if (it + 1 < a.refine_steps) {
        const float fn = f(tn);
        s.shift(tn, fn);
      }
    }
    if (valid && half == 0) a.depth[pr.x] = s.out;
  }
}

// ---- deferred shading ---------------------------------------------------------
__global__ void k_clear_rgb(KArgs a, const int32_t* ids) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.n_rays) return;
  const int inst = ids[p];
  float c[3] = {a.clear_rgb[0], a.clear_rgb[1], a.clear_rgb[2]};
  if (inst >= 0 && inst < a.n_inst) {
    const ObjDesc& od = a.obj[a.inst_object[inst]];
    if (od.field != NEDF_FIELD_MLP) { c[0] = od.param[3]; c[1] = od.param[4]; c[2] = od.param[5]; }
  }
  a.rgb[3 * p + 0] = c[0];
  a.rgb[3 * p + 1] = c[1];
  a.rgb[3 * p + 2] = c[2];
}

// NeRF shading: a wave shades 32 / K pixels with K samples each; trunk with
// the sigma head, then the colour layer on [h_last, gamma_dirL(d)], then
// local compositing across each pixel's K lanes.
template <int DT, int WIDTH, int NHID, int L, int DIRL, int RGBW, int SBX, int OCC, int NW>
__global__ __launch_bounds__(64 * NW, OCC) void k_shade(KArgs a) {
  using T = eng::Tr<DT>;
  constexpr int NB = T::NB;
  constexpr int KS0 = eng::ks_for_slots<DT>(3 * L + 2);
  constexpr int KSH = WIDTH / T::KPS;
  constexpr int KSD = eng::ks_for_slots<DT>(3 * DIRL + 2);
  constexpr int KSR = KSH + KSD;
  constexpr int CBR = eng::chunk_bytes<DT>(KSR, 3);
  constexpr int CHUNK = eng::cmax(eng::cmax(eng::chunk_bytes<DT>(KS0, 0), eng::chunk_bytes<DT>(KSH, 1)), CBR);
  __shared__ __attribute__((aligned(16))) uint8_t lds[eng::NBUF * eng::slot_bytes(CHUNK, SBX)];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
  const int K = a.shade_K;  // 1, 2, 4, 8, 16 or 32
  const int ppw = 32 / K;
  const int slot = lane & 31, q = slot / K, j = slot % K;
  // first pass: the binned pixels (list A), outliers pushed to list B;
  // second pass (chord mode): list B
  const bool chord = a.shade_chord != 0;
  PairList* PL = chord ? &a.C->B : &a.C->A;
  const uint2* prs_list = chord ? a.pairsB : a.pairs;
  PairList* RS = &a.C->B;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&PL->work_counter, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= PL->total_items) break;
    const int obj = item_object(PL, a.n_obj, item);
    const int local = (item - PL->item_start[obj]) * (ppw * NW) + wave * ppw + q;
    const bool valid = local < PL->cnt[obj];
    const uint2 pr = prs_list[PL->off[obj] + (valid ? local : 0)];
    const ObjDesc& od = a.obj[obj];
    const uint8_t* blob = od.blob;
    const nedf_blob_header* hb = reinterpret_cast<const nedf_blob_header*>(blob);
    const float head_b = uniform_load_f32(blob + uniform_load_u64(&hb->off_head_b));
    const float* rgb_bp = reinterpret_cast<const float*>(blob + uniform_load_u64(&hb->off_rgbh_b));
    const float rgb_b[3] = {uniform_load_f32(rgb_bp), uniform_load_f32(rgb_bp + 1), uniform_load_f32(rgb_bp + 2)};
    const W2L g = load_w2l(a.w2l, int(pr.y));
    float o[3], d[3], ol[3], dl[3];
    make_ray(a.rays, pr.x, o, d);
    to_local(g, o, d, ol, dl);
    // sample window in world units: [D - h, D + h], or (chord mode) the
    // chord of the bounding sphere
    float t_lo, step;
    {
      float ca = 0.0f, cb = 0.0f;
      if (chord && sphere_chord(ol, dl, od.bound, ca, cb)) {
        t_lo = g.s * ca;
        step = g.s * (cb - ca) / float(K);
      } else {
        const float D = a.depth[pr.x];
        t_lo = D - a.shade_h;
        step = 2.0f * a.shade_h / float(K);
      }
    }
    const float t = t_lo + (float(j) + 0.5f) * step;
    const float tl = t * g.inv_s;
    float p[3] = {fmaf(tl, dl[0], ol[0]), fmaf(tl, dl[1], ol[1]), fmaf(tl, dl[2], ol[2])};
    typename T::frag Benc[NB][KS0];
    eng::encode_input<DT, 3, L, KS0>(p, half, Benc[0]);
    float partial[NB][1] = {{0.f}};
    typename T::frag Blast[NB][KSH];
    int cur = 0;
    eng::trunk<DT, WIDTH, KS0, NHID, 1, CHUNK, true, CBR, RGBW / 32, SBX, NB, NW>(
        hb, blob, Benc, lds, partial, Blast, blob + uniform_load_u64(&hb->off_rgb), &cur);
    const float u = partial[0][0] + __shfl_xor(partial[0][0], 32) + head_b;
    const float sig = mlp_sigma(od, u, p[0], p[1], p[2]);
    // colour layer input: [h_last, gamma_dirL(d_l)]
    typename T::frag Bc[NB][KSR];
#pragma unroll
    for (int k = 0; k < KSH; ++k) Bc[0][k] = Blast[0][k];
    {
      typename T::frag Bd[KSD];
      eng::encode_input<DT, 3, DIRL, KSD>(dl, half, Bd);
#pragma unroll
      for (int k = 0; k < KSD; ++k) Bc[0][KSH + k] = Bd[k];
    }
    float prgb[NB][3] = {{0.f, 0.f, 0.f}};
    typename T::frag dummy[NB][1];
    eng::layer<DT, NB, KSR, RGBW / 32, CBR, 0, 1, 3, 1, CHUNK, RGBW / 32, SBX, NW>(
        Bc, dummy, blob + uniform_load_u64(&hb->off_rgb), nullptr, lds, cur, prgb);
    float c[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) c[ch] = sigmoidf_(prgb[0][ch] + __shfl_xor(prgb[0][ch], 32) + rgb_b[ch]);
    // local compositing over the K lanes of this pixel
    const float v = sig * (step * g.inv_s);
    float incl = v;
    for (int off = 1; off < K; off <<= 1) {
      const float y = __shfl_up(incl, off);
      if (j >= off) incl += y;
    }
    const float w = expf(-(incl - v)) * one_minus_exp_neg(v);
    float sw = w, sc0 = w * c[0], sc1 = w * c[1], sc2 = w * c[2];
    for (int off = 1; off < K; off <<= 1) {
      sw += __shfl_xor(sw, off);
      sc0 += __shfl_xor(sc0, off);
      sc1 += __shfl_xor(sc1, off);
      sc2 += __shfl_xor(sc2, off);
    }
    const int near = (K - 1) / 2;
    const int src = (lane & ~(K - 1)) + near;
    const float n0 = __shfl(c[0], src), n1 = __shfl(c[1], src), n2 = __shfl(c[2], src);
    if (!chord && a.rs_sigma > 0.0f) {
      // outlier (Sec. "Deferred Shading"): density below the threshold at
      // every sample of the pixel; pushed to the object's segment of list B
      float smax = sig;
      for (int off = 1; off < K; off <<= 1) smax = fmaxf(smax, __shfl_xor(smax, off));
      const bool outlier = valid && half == 0 && j == 0 && smax < a.rs_sigma;
      const uint64_t m = __ballot(outlier);
      if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        int base = 0;
        if (lane == leader) {
          base = atomicAdd(&RS->cnt[obj], __popcll(m));
          atomicAdd(&a.C->stats[1], __popcll(m));
        }
        base = __shfl(base, leader);
        if (outlier) a.pairsB[RS->off[obj] + base + __popcll(m & ((1ull << lane) - 1ull))] = pr;
      }
    }
    if (valid && half == 0 && j == 0) {
      float* out = a.rgb + 3 * size_t(pr.x);
      if (sw < 1e-6f) {
        out[0] = n0; out[1] = n1; out[2] = n2;
      } else {
        out[0] = sc0 / sw; out[1] = sc1 / sw; out[2] = sc2 / sw;
      }
    }
  }
}

// ---- shadows --------------------------------------------------------------------
// Shadow ray of pixel p for light Lm: origin Lm, direction towards
// x = o + D d; pixels without an ID get a NaN ray (culled everywhere).
// Shadow rays of one light (Alg. 2) for the hit pixels: from a point light
// at (lx, ly, lz) towards x = o + D d, or (dir_dist > 0) for a directional
// light of unit direction of travel (lx, ly, lz), from x - dir_dist l along
// l (parallel, orthographic rays); dist gets the distance from the origin to
// x.  Pixels without a hit get a NaN direction (culled as no candidate).
__global__ void k_shadow_rays(KArgs a, const int32_t* ids, float lx, float ly, float lz, float dir_dist, float* so,
                              float* sd, float* dist) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.n_rays) return;
  float o[3], d[3];
  make_ray(a.rays, p, o, d);
  const float D = a.depth[p];
  const bool hit = ids[p] >= 0;
  const float nan = __int_as_float(0x7fc00000);
  const float px = fmaf(D, d[0], o[0]), py = fmaf(D, d[1], o[1]), pz = fmaf(D, d[2], o[2]);
  if (dir_dist > 0.0f) {
    so[3 * p + 0] = fmaf(-dir_dist, lx, px);
    so[3 * p + 1] = fmaf(-dir_dist, ly, py);
    so[3 * p + 2] = fmaf(-dir_dist, lz, pz);
    sd[3 * p + 0] = hit ? lx : nan; sd[3 * p + 1] = hit ? ly : nan; sd[3 * p + 2] = hit ? lz : nan;
    dist[p] = hit ? dir_dist : 0.f;
    return;
  }
  const float x = px - lx, y = py - ly, z = pz - lz;
  const float r = sqrtf(x * x + y * y + z * z);
  const float inv = hit && r > 0.f ? 1.0f / r : nan;
  so[3 * p + 0] = lx; so[3 * p + 1] = ly; so[3 * p + 2] = lz;
  sd[3 * p + 0] = x * inv; sd[3 * p + 1] = y * inv; sd[3 * p + 2] = z * inv;
  dist[p] = hit ? r : 0.f;
}

__global__ void k_shadow_init(KArgs a, float* shadow) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < a.n_rays) shadow[p] = 1.0f;
}

// Occlusion test of Alg. 2 for one light: D_L + eps < |L - x| multiplies by beta.
__global__ void k_shadow_apply(KArgs a, const int32_t* ids, const float* depth_l, const float* dist, float eps,
                               float beta, float* shadow) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.n_rays || ids[p] < 0) return;
  if (depth_l[p] + eps < dist[p]) shadow[p] *= beta;
}

__global__ void k_composite(KArgs a, const float* shadow, float* rgb) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.n_rays) return;
  const float f = shadow[p];
  rgb[3 * p + 0] *= f;
  rgb[3 * p + 1] *= f;
  rgb[3 * p + 2] *= f;
}

int cu_count2() {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 256;
  }
  return ncu;
}

unsigned grid_n(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return unsigned(g > 0 ? g : 1);
}

}  // namespace

// Bins hit pixels of the objects in `mask` into list A with work items of
// `per` pixels.
void stage_bin_pixels(const KArgs& k0, hipStream_t s, const int32_t* ids, uint32_t mask, int per) {
  KArgs k = k0;
  k.item_mask = mask;
  k.item_pairs = per;
  k.L = &k.C->A;
  const unsigned g = grid_n(k.n_rays) < BIN_BLOCKS ? grid_n(k.n_rays) : BIN_BLOCKS;
  hipLaunchKernelGGL(k_zero_list, dim3(1), dim3(256), 0, s, &k.C->A);
  hipLaunchKernelGGL(k_bin<0>, dim3(g), dim3(256), 0, s, k, ids, mask);
  hipLaunchKernelGGL(k_scan_pixels, dim3(1), dim3(64), 0, s, k);
  hipLaunchKernelGGL(k_bin<1>, dim3(g), dim3(256), 0, s, k, ids, mask);
}

void stage_refine(const KArgs& k, hipStream_t s, const int32_t* ids, uint32_t mlp_mask, uint32_t sphere_mask,
                  int dtype) {
  prof_mark("infer.refine", s, true);
  if (sphere_mask) {
    stage_bin_pixels(k, s, ids, sphere_mask, 1);
    hipLaunchKernelGGL(k_refine_analytic, dim3(256), dim3(256), 0, s, k, sphere_mask);
  }
  if (mlp_mask) {
    // BF16: one workgroup of 8 waves per CU, which streams each weight chunk
    // into LDS once for 256 samples (two workgroups of 4 waves stream it
    // twice; the refinement is bound by that L2 -> LDS stream, and the 8-wave
    // form measured 8 % faster on the 1080p frame); FP32: one of 4 waves
    stage_bin_pixels(k, s, ids, mlp_mask, dtype == NEDF_BF16 ? 32 * 8 : 32 * 4);
    if (dtype == NEDF_BF16)
      hipLaunchKernelGGL((k_refine_mlp<1, 256, 8, 10, 2, 1, 8>), dim3(cu_count2()), dim3(512), 0, s, k);
    else
      hipLaunchKernelGGL((k_refine_mlp<0, 256, 8, 10, eng::sb_default<0>(), 1, 4>), dim3(cu_count2()), dim3(256), 0,
                         s, k);
  }
  prof_mark("infer.refine", s, false);
}

namespace {
void launch_shade(const KArgs& k, hipStream_t s, int dtype) {
  if (dtype == NEDF_BF16)
    hipLaunchKernelGGL((k_shade<1, 256, 8, 10, 4, 128, 2, 1, 8>), dim3(cu_count2()), dim3(512), 0, s, k);
  else
    hipLaunchKernelGGL((k_shade<0, 256, 8, 10, 4, 128, eng::sb_default<0>(), 1, 4>), dim3(cu_count2()), dim3(256),
                       0, s, k);
}
}  // namespace

// List B takes the outliers of the first shading pass in the segments of
// list A (an object's outliers are a subset of its pixels); its counts and the
// resampling count start at zero.
__global__ void k_rs_prepare(KArgs a) {
  const int m = threadIdx.x;
  PairList* A = &a.C->A;
  PairList* B = &a.C->B;
  if (m <= a.n_obj) B->off[m] = A->off[m];
  if (m < a.n_obj) {
    B->cnt[m] = 0;
    B->fill[m] = 0;
  }
  if (m == 0) {
    B->total_items = B->work_counter = B->total_pairs = 0;
    a.C->stats[1] = 0;
  }
}

// Work items of the outlier list (segments fixed by k_rs_prepare).
__global__ void k_rs_items(KArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  PairList* L = &a.C->B;
  int items = 0, total = 0;
  for (int m = 0; m < a.n_obj; ++m) {
    L->item_start[m] = items;
    const int c = L->cnt[m];
    if ((a.item_mask >> m) & 1u) items += (c + a.item_pairs - 1) / a.item_pairs;
    total += c;
  }
  L->item_start[a.n_obj] = items;
  L->total_items = items;
  L->total_pairs = total;
  L->work_counter = 0;
}

void stage_shade(const KArgs& k, hipStream_t s, const int32_t* ids, uint32_t nerf_mask, int dtype, int rs_samples) {
  prof_mark("shade", s, true);
  hipLaunchKernelGGL(k_clear_rgb, dim3(grid_n(k.n_rays)), dim3(256), 0, s, k, ids);
  if (nerf_mask) {
    // BF16: one workgroup of 8 waves per CU sharing each weight copy; FP32: 4 waves
    const int nw = dtype == NEDF_BF16 ? 8 : 4;
    stage_bin_pixels(k, s, ids, nerf_mask, (32 / k.shade_K) * nw);
    KArgs k1 = k;
    k1.shade_chord = 0;
    if (rs_samples > 0) hipLaunchKernelGGL(k_rs_prepare, dim3(1), dim3(NEDF_MAX_OBJECTS + 64), 0, s, k1);
    else k1.rs_sigma = 0.0f;
    launch_shade(k1, s, dtype);
    if (rs_samples > 0) {
      // second pass: the outliers, volume-rendered over the bounding chord
      prof_mark("shade.resample", s, true);
      KArgs k2 = k;
      k2.shade_chord = 1;
      k2.shade_K = rs_samples;
      k2.item_mask = nerf_mask;
      k2.item_pairs = (32 / rs_samples) * nw;
      hipLaunchKernelGGL(k_rs_items, dim3(1), dim3(64), 0, s, k2);
      launch_shade(k2, s, dtype);
      prof_mark("shade.resample", s, false);
    }
  }
  prof_mark("shade", s, false);
}

void stage_shadow_rays(const KArgs& k, hipStream_t s, const int32_t* ids, const float L[3], float dir_dist, float* so,
                       float* sd, float* dist) {
  hipLaunchKernelGGL(k_shadow_rays, dim3(grid_n(k.n_rays)), dim3(256), 0, s, k, ids, L[0], L[1], L[2], dir_dist, so,
                     sd, dist);
}

void stage_shadow_init(const KArgs& k, hipStream_t s, float* shadow) {
  hipLaunchKernelGGL(k_shadow_init, dim3(grid_n(k.n_rays)), dim3(256), 0, s, k, shadow);
}

void stage_shadow_apply(const KArgs& k, hipStream_t s, const int32_t* ids, const float* depth_l, const float* dist,
                        float eps, float beta, float* shadow) {
  hipLaunchKernelGGL(k_shadow_apply, dim3(grid_n(k.n_rays)), dim3(256), 0, s, k, ids, depth_l, dist, eps, beta,
                     shadow);
}

void stage_composite(const KArgs& k, hipStream_t s, const float* shadow, float* rgb) {
  hipLaunchKernelGGL(k_composite, dim3(grid_n(k.n_rays)), dim3(256), 0, s, k, shadow, rgb);
}

}  // namespace nedf
