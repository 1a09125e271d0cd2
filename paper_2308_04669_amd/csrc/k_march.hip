// Plain volume-rendering marcher (Eq. 5) composed over instances (Alg. 1,
// step 1): pair culling/binning, analytic and MLP density marching with a
// packed-key min-reduce, and the final unpack into depth / ID buffers.
#include <cstring>

#include "device_common.h"
#include "launch.h"
#include "mlp_engine.h"
#include "runtime.h"

namespace nedf {
namespace {

struct KArgs {
  RaySrc rays;
  int64_t n_rays;
  int32_t n_obj, n_inst;
  ObjDesc obj[NEDF_MAX_OBJECTS];
  const int32_t* inst_object;
  const float* w2l;
  int32_t n_samples, clip;
  float t_near, t_far, hit_thr;
  uint32_t mlp_mask;  // objects handled by the matrix-core kernel
  int* status;
  WsCounters* C;
  uint64_t* keys;
  uint32_t* opac;
  uint2* pairs;
  int64_t capacity;
  float* depth;
  int32_t* id;
  float* opacity;
};

__global__ void k_init(KArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < a.n_rays) {
    a.keys[i] = NEDF_KEY_EMPTY;
    a.opac[i] = 0u;
  }
  if (i == 0) *a.status = 0;
  if (i < int64_t(sizeof(WsCounters) / 4)) reinterpret_cast<int32_t*>(a.C)[i] = 0;
}

__device__ __forceinline__ bool pair_test(const KArgs& a, const float o[3], const float d[3], int inst,
                                          int obj) {
  if (!a.clip) return true;
  const W2L g = load_w2l(a.w2l, inst);
  float ol[3], dl[3], ta, tb;
  to_local(g, o, d, ol, dl);
  return sphere_chord(ol, dl, a.obj[obj].bound, ta, tb);
}

// Pass 0 counts pairs per object; pass 1 writes them.  One thread per ray,
// wave-aggregated atomics per (wave, instance).
template <int PASS>
__global__ void k_cull(KArgs a) {
  const int64_t ray = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool live = ray < a.n_rays;
  float o[3] = {0, 0, 0}, d[3] = {0, 0, 1};
  if (live) make_ray(a.rays, ray, o, d);
  const int lane = threadIdx.x & 63;
  for (int k = 0; k < a.n_inst; ++k) {
    const int obj = a.inst_object[k];
    const bool pass = live && obj >= 0 && obj < a.n_obj && pair_test(a, o, d, k, obj);
    const uint64_t m = __ballot(pass);
    if (m == 0) continue;
    const int cnt = __popcll(m);
    if (PASS == 0) {
      if (lane == __ffsll((unsigned long long)m) - 1) atomicAdd(&a.C->cnt[obj], cnt);
    } else {
      const int leader = __ffsll((unsigned long long)m) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(&a.C->fill[obj], cnt);
      base = __shfl(base, leader);
      if (pass) {
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        const int pos = base + rank;
        if (pos < a.C->cnt[obj]) a.pairs[a.C->off[obj] + pos] = make_uint2(uint32_t(ray), uint32_t(k));
      }
    }
  }
}

__global__ void k_scan(KArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  WsCounters* C = a.C;
  int64_t off = 0;
  int items = 0;
  bool over = false;
  for (int m = 0; m < a.n_obj; ++m) {
    int64_t c = C->cnt[m];
    if (off + c > a.capacity) {
      c = a.capacity - off > 0 ? a.capacity - off : 0;
      over = true;
    }
    C->cnt[m] = int32_t(c);
    C->off[m] = int32_t(off);
    C->item_start[m] = items;
    if ((a.mlp_mask >> m) & 1u) items += int32_t((c + eng::WAVES - 1) / eng::WAVES);
    C->fill[m] = 0;
    off += c;
  }
  C->off[a.n_obj] = int32_t(off);
  C->item_start[a.n_obj] = items;
  C->total_items = items;
  C->total_pairs = int32_t(off);
  C->work_counter = 0;
  if (over) set_status(a.status, NEDF_ERR_CAPACITY);
}

__device__ __forceinline__ void neu_add(float& s, float& c, float x) {
  const float t = s + x;
  c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

__device__ __forceinline__ void emit(const KArgs& a, uint2 pr, float A, float S, float s) {
  if (A >= a.hit_thr && A > 0.0f) {
    const float D = s * (S / A);
    atomicMin(reinterpret_cast<unsigned long long*>(&a.keys[pr.x]),
              (unsigned long long)pack_key(D, int(pr.y)));
  }
  atomicMax(&a.opac[pr.x], __float_as_uint(fmaxf(A, 0.0f)));
}

__device__ __forceinline__ float analytic_sigma(const ObjDesc& od, float x, float y, float z) {
  if (od.field == NEDF_FIELD_SPHERE) {
    const float r = sqrtf(x * x + y * y + z * z);
    return od.param[0] * sigmoidf_((od.param[1] - r) / od.param[2]);
  }
  return (z >= od.param[1] && z <= od.param[2]) ? od.param[0] : 0.0f;
}

// One thread per pair of an analytic object; sequential compensated scan.
__global__ void k_march_analytic(KArgs a) {
  const int total = a.C->total_pairs;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const uint2 pr = a.pairs[q];
    const int obj = a.inst_object[pr.y];
    const ObjDesc od = a.obj[obj];
    if (od.field == NEDF_FIELD_MLP) continue;
    const W2L g = load_w2l(a.w2l, int(pr.y));
    float o[3], d[3], ol[3], dl[3];
    make_ray(a.rays, pr.x, o, d);
    to_local(g, o, d, ol, dl);
    float ta, tb;
    if (a.clip) {
      if (!sphere_chord(ol, dl, od.bound, ta, tb)) continue;
    } else {
      ta = a.t_near * g.inv_s;
      tb = a.t_far * g.inv_s;
    }
    const int N = a.n_samples;
    const float delta = (tb - ta) / float(N);
    const float px = fmaf(ta, dl[0], ol[0]), py = fmaf(ta, dl[1], ol[1]), pz = fmaf(ta, dl[2], ol[2]);
    float tau = 0.f, tau_c = 0.f, sw = 0.f, sw_c = 0.f, swt = 0.f, swt_c = 0.f;
    for (int i = 0; i < N; ++i) {
      const float tr = (float(i) + 0.5f) * delta;
      const float sig = analytic_sigma(od, fmaf(tr, dl[0], px), fmaf(tr, dl[1], py), fmaf(tr, dl[2], pz));
      const float v = sig * delta;
      const float w = expf(-(tau + tau_c)) * one_minus_exp_neg(v);
      neu_add(sw, sw_c, w);
      neu_add(swt, swt_c, w * (ta + tr));
      neu_add(tau, tau_c, v);
    }
    emit(a, pr, sw + sw_c, swt + swt_c, g.s);
  }
}

template <int DT>
__device__ __forceinline__ float sigma_of(const ObjDesc& od, float u, float x, float y, float z) {
  if (od.sigma_mode == NEDF_SIGMA_SDF)
    return od.param[0] * sigmoidf_(u - sdf_shape(int(od.param[2]), x, y, z) / od.param[1]);
  const float s = softplusf_(u);
  if (od.sigma_mode == NEDF_SIGMA_SOFTPLUS_MASKED)
    return (x * x + y * y + z * z <= od.bound * od.bound) ? s : 0.0f;
  return s;
}

// Matrix-core marcher: a workgroup takes items of 4 pairs (one per wave) of
// one object from a global queue; each wave marches its pair in chunks of
// 32 * NB samples through the register-resident density network, then scans
// the chunk's optical depths across the wave.
template <int DT, int WIDTH, int NHID, int L>
__global__ __launch_bounds__(256, 1) void k_march_mlp(KArgs a) {
  using T = eng::Tr<DT>;
  constexpr int NB = T::NB;
  constexpr int KS0 = eng::ks_for_slots<DT>(3 * L + 2);
  constexpr int KSH = WIDTH / T::KPS;
  constexpr int CHUNK = eng::cmax(eng::chunk_bytes<DT>(KS0, 0), eng::chunk_bytes<DT>(KSH, 1));
  constexpr int SPC = 32 * NB;  // samples per wave per chunk
  __shared__ __attribute__((aligned(16))) uint8_t lds[2 * CHUNK];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
  WsCounters* C = a.C;
  const int N = a.n_samples;
  const int n_chunks = (N + SPC - 1) / SPC;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&C->work_counter, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= C->total_items) break;
    int obj = 0;
    while (obj + 1 < a.n_obj && C->item_start[obj + 1] <= item) ++obj;
    const int local = (item - C->item_start[obj]) * eng::WAVES + wave;
    const bool valid = local < C->cnt[obj];
    const uint2 pr = a.pairs[C->off[obj] + (valid ? local : 0)];
    const ObjDesc od = a.obj[obj];
    const uint8_t* blob = od.blob;
    const nedf_blob_header* hb = reinterpret_cast<const nedf_blob_header*>(blob);
    const float head_b = reinterpret_cast<const float*>(blob + hb->off_head_b)[0];
    const W2L g = load_w2l(a.w2l, int(pr.y));
    float o[3], d[3], ol[3], dl[3];
    make_ray(a.rays, pr.x, o, d);
    to_local(g, o, d, ol, dl);
    float ta = 0.f, tb = 0.f;
    bool seg = true;
    if (a.clip) {
      seg = sphere_chord(ol, dl, od.bound, ta, tb);
      if (!seg) { ta = 0.f; tb = 0.f; }
    } else {
      ta = a.t_near * g.inv_s;
      tb = a.t_far * g.inv_s;
    }
    const float delta = (tb - ta) / float(N);
    const float pa[3] = {fmaf(ta, dl[0], ol[0]), fmaf(ta, dl[1], ol[1]), fmaf(ta, dl[2], ol[2])};
    float carry = 0.f, carry_c = 0.f, sw = 0.f, sw_c = 0.f, swt = 0.f, swt_c = 0.f;
    for (int c = 0; c < n_chunks; ++c) {
      typename T::frag Benc[NB][KS0];
      float xs[NB][3];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int i = c * SPC + 32 * nb + (lane & 31);
        const float tr = (float(i) + 0.5f) * delta;
        float p[3] = {fmaf(tr, dl[0], pa[0]), fmaf(tr, dl[1], pa[1]), fmaf(tr, dl[2], pa[2])};
        xs[nb][0] = p[0]; xs[nb][1] = p[1]; xs[nb][2] = p[2];
        eng::encode_input<DT, 3, L, KS0>(p, half, Benc[nb]);
      }
      float partial[NB][1];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) partial[nb][0] = 0.f;
      typename T::frag Blast[NB][KSH];
      eng::trunk<DT, WIDTH, KS0, NHID, 1, CHUNK, false, 0>(hb, blob, Benc, lds, partial, Blast, nullptr);
      // sample of this lane in the wave-wide scan: c * SPC + lane (NB = 2), or lanes 0..31 (NB = 1)
      float v = 0.f;
      int si = 0;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float u = partial[nb][0] + __shfl_xor(partial[nb][0], 32) + head_b;
        const float sig = sigma_of<DT>(od, u, xs[nb][0], xs[nb][1], xs[nb][2]);
        if (NB == 1 || nb == half) {
          si = c * SPC + (NB == 1 ? lane : lane);
          v = sig * delta;
        }
      }
      if (NB == 1 && lane >= 32) v = 0.f;
      if (si >= N || !seg) v = 0.f;
      // inclusive scan of optical depth over the wave (sample order = lane order)
      float incl = v;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const float y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
      }
      const float tau = (carry + carry_c) + (incl - v);
      const float w = expf(-tau) * one_minus_exp_neg(v);
      const float t = ta + (float(si) + 0.5f) * delta;
      float ws = w, wts = w * t;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        ws += __shfl_xor(ws, off);
        wts += __shfl_xor(wts, off);
      }
      neu_add(sw, sw_c, ws);
      neu_add(swt, swt_c, wts);
      neu_add(carry, carry_c, __shfl(incl, 63));
    }
    if (lane == 0 && valid && seg) emit(a, pr, sw + sw_c, swt + swt_c, g.s);
  }
}

__global__ void k_finalize(KArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n_rays) return;
  const uint64_t k = a.keys[i];
  if (k == NEDF_KEY_EMPTY) {
    a.depth[i] = __int_as_float(0x7f800000);
    a.id[i] = -1;
  } else {
    a.depth[i] = __uint_as_float(uint32_t(k >> 32));
    a.id[i] = int32_t(uint32_t(k & 0xffffffffu));
  }
  if (a.opacity) a.opacity[i] = __uint_as_float(a.opac[i]);
}

template <int DT, int WIDTH, int NHID, int L>
hipError_t launch_mlp(const KArgs& k, hipStream_t s) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_march_mlp<DT, WIDTH, NHID, L>), dim3(ncu), dim3(eng::THREADS), 0, s, k);
  return hipGetLastError();
}

}  // namespace

bool march_mlp_supported(int dtype, int width, int n_hidden, int L) {
  if (dtype != NEDF_F32 && dtype != NEDF_BF16) return false;
  return (width == 64 && n_hidden == 3 && L == 6) || (width == 256 && n_hidden == 8 && L == 10);
}

hipError_t launch_march(const MarchLaunch& m, hipStream_t s) {
  KArgs k;
  std::memset(&k, 0, sizeof(k));
  k.rays.kind = m.rays.kind;
  k.rays.width = m.rays.width;
  k.rays.height = m.rays.height;
  for (int i = 0; i < 3; ++i) {
    k.rays.eye[i] = m.rays.eye[i];
    k.rays.fwd[i] = m.rays.fwd[i];
    k.rays.right[i] = m.rays.right[i];
    k.rays.up[i] = m.rays.up[i];
  }
  k.rays.o = m.rays.o;
  k.rays.d = m.rays.d;
  k.n_rays = m.rays.n;
  k.n_obj = m.n_obj;
  k.n_inst = m.n_inst;
  uint32_t mask = 0;
  bool any_analytic = false;
  for (int i = 0; i < m.n_obj; ++i) {
    k.obj[i] = m.obj[i];
    if (m.obj[i].field == NEDF_FIELD_MLP) mask |= 1u << i;
    else any_analytic = true;
  }
  k.mlp_mask = mask;
  k.inst_object = m.inst_object;
  k.w2l = m.inst_w2l;
  k.n_samples = m.n_samples;
  k.clip = m.clip;
  k.t_near = m.t_near;
  k.t_far = m.t_far;
  k.hit_thr = m.hit_thr;
  k.status = reinterpret_cast<int*>(m.ws);
  k.C = reinterpret_cast<WsCounters*>(m.ws + m.lay.counters);
  k.keys = reinterpret_cast<uint64_t*>(m.ws + m.lay.keys);
  k.opac = reinterpret_cast<uint32_t*>(m.ws + m.lay.opac);
  k.pairs = reinterpret_cast<uint2*>(m.ws + m.lay.pairs);
  k.capacity = m.lay.capacity;
  k.depth = m.depth;
  k.id = m.id;
  k.opacity = m.opacity;
  const int64_t n = m.rays.n;
  const int blk = 256;
  const unsigned grid_rays = unsigned((n + blk - 1) / blk);
  const unsigned grid_init = grid_rays > 1 ? grid_rays : 1;
  prof_mark("march.cull", s, true);
  hipLaunchKernelGGL(k_init, dim3(grid_init), dim3(blk), 0, s, k);
  hipLaunchKernelGGL(k_cull<0>, dim3(grid_init), dim3(blk), 0, s, k);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(64), 0, s, k);
  hipLaunchKernelGGL(k_cull<1>, dim3(grid_init), dim3(blk), 0, s, k);
  prof_mark("march.cull", s, false);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (any_analytic) {
    prof_mark("march.analytic", s, true);
    hipLaunchKernelGGL(k_march_analytic, dim3(1024), dim3(blk), 0, s, k);
    prof_mark("march.analytic", s, false);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (mask) {
    const int W = m.mlp_width, H = m.mlp_hidden, L = m.mlp_L;
    prof_mark("march.mlp", s, true);
    if (m.dtype == NEDF_BF16) {
      if (W == 256 && H == 8 && L == 10) e = launch_mlp<1, 256, 8, 10>(k, s);
      else e = launch_mlp<1, 64, 3, 6>(k, s);
    } else {
      if (W == 256 && H == 8 && L == 10) e = launch_mlp<0, 256, 8, 10>(k, s);
      else e = launch_mlp<0, 64, 3, 6>(k, s);
    }
    prof_mark("march.mlp", s, false);
    if (e != hipSuccess) return e;
  }
  prof_mark("march.finalize", s, true);
  hipLaunchKernelGGL(k_finalize, dim3(grid_init), dim3(blk), 0, s, k);
  prof_mark("march.finalize", s, false);
  return hipGetLastError();
}

}  // namespace nedf
