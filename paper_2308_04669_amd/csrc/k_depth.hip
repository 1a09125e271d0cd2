// Depth stage kernels: culling/binning into per-object pair lists, the plain
// volume-rendering marcher (Eq. 5) on analytic and MLP fields, the NeDF
// intersection network (Eq. 1, 2, 7) with routing of uncertain pairs to the
// marcher, and the packed-key composition (Alg. 1, step 1).
#include <cstring>

#include "pipeline.h"
#include "runtime.h"

namespace nedf {
namespace {

__global__ void k_init(KArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < a.n_rays) {
    a.keys[i] = NEDF_KEY_EMPTY;
    a.opac[i] = 0u;
  }
  if (i == 0) *a.status = 0;
  // every counter word, whatever the grid size
  constexpr int64_t words = int64_t(sizeof(WsCounters) / 4);
  for (int64_t w = i; w < words; w += int64_t(gridDim.x) * blockDim.x)
    reinterpret_cast<int32_t*>(a.C)[w] = w == int64_t(offsetof(WsCounters, dmin_bits) / 4) ? 0x7F800000 : 0;
}

// Exact per-ray test; dm gets the lowest depth the pair can report,
// s (t_perp - l) clamped at 0 (the network's depth is s (t_perp - l mu) with
// mu clamped to [-1, 1], the marcher's lies inside the chord).
__device__ __forceinline__ bool pair_test(const KArgs& a, const float o[3], const float d[3], int inst,
                                          int obj, float& dm) {
  dm = 0.0f;
  if (!a.clip) return true;
  const W2L g = load_w2l(a.w2l, inst);
  float ol[3], dl[3], ta, tb;
  to_local(g, o, d, ol, dl);
  const float bound = a.obj[obj].bound;
  // single-precision t_perp differs from the intersection network's
  // compensated one by a few units in the last place of the terms that form
  // o_l (R^T o / s and c, each at most |o|_1 / s and |c|_1 in size); the
  // bound is lowered by 2^-20 times their sum plus one, well beyond that, so
  // that it never exceeds a depth the network can report
  const float tperp = -(ol[0] * dl[0] + ol[1] * dl[1] + ol[2] * dl[2]);
  const float slack = 9.5367431640625e-7f * ((fabsf(o[0]) + fabsf(o[1]) + fabsf(o[2])) * g.inv_s +
                                             fabsf(g.c[0]) + fabsf(g.c[1]) + fabsf(g.c[2]) + 1.0f);
  dm = fmaxf(g.s * (tperp - bound - slack), 0.0f);
  return sphere_chord(ol, dl, bound, ta, tb);
}

// Culling and binning (Alg. 1, "models in the view frustum"): list A gets
// one (ray, instance) pair for every ray that meets an instance's bounding
// sphere ahead of its origin.  A workgroup takes 256 rays: a 16 x 16 pixel
// tile for camera rays, 256 consecutive rays for ray arrays.  For a tile it
// first keeps only the instances whose bounding sphere can meet the tile's
// frustum (a conservative test; the exact per-ray test decides), in index
// order.  Pass 0 counts pairs per object, pass 1 reserves one range per
// object for the workgroup and writes the pairs; counts are aggregated per
// wave and per workgroup in LDS, so global atomics are one per (workgroup,
// object).
constexpr int CULL_TILE = 16;
constexpr int CULL_BATCH = 1024;  // candidate instances held in LDS at a time

struct TileFrustum {
  float eye[3], rh[3], uh[3], fw[3];  // camera basis (unit vectors)
  float nx0, nx1, ny0, ny1;           // tile bounds as x/z and y/z slopes
};

__device__ __forceinline__ bool tile_meets_sphere(const TileFrustum& f, const float c[3], float r) {
  const float q[3] = {c[0] - f.eye[0], c[1] - f.eye[1], c[2] - f.eye[2]};
  const float X = q[0] * f.rh[0] + q[1] * f.rh[1] + q[2] * f.rh[2];
  const float Y = q[0] * f.uh[0] + q[1] * f.uh[1] + q[2] * f.uh[2];
  const float Z = q[0] * f.fw[0] + q[1] * f.fw[1] + q[2] * f.fw[2];
  // margin for float rounding of the instance record and of the basis
  const float rr = r + 1e-4f * (fabsf(X) + fabsf(Y) + fabsf(Z) + r) + 1e-6f;
  if (Z < -rr) return false;
  if (X - f.nx0 * Z < -rr * sqrtf(1.0f + f.nx0 * f.nx0)) return false;
  if (f.nx1 * Z - X < -rr * sqrtf(1.0f + f.nx1 * f.nx1)) return false;
  if (Y - f.ny0 * Z < -rr * sqrtf(1.0f + f.ny0 * f.ny0)) return false;
  if (f.ny1 * Z - Y < -rr * sqrtf(1.0f + f.ny1 * f.ny1)) return false;
  return true;
}

// World-space bounding sphere of instance k: centre -s R c, radius s l.
__device__ __forceinline__ void instance_sphere(const KArgs& a, int k, int obj, float c[3], float& r) {
  const W2L g = load_w2l(a.w2l, k);
#pragma unroll
  for (int i = 0; i < 3; ++i)
    c[i] = -g.s * (g.rt[i] * g.c[0] + g.rt[3 + i] * g.c[1] + g.rt[6 + i] * g.c[2]);
  r = g.s * a.obj[obj].bound;
}

// Ray bundle of an array-ray workgroup: origins within rho of O, directions
// within angle theta of the unit axis (cos_theta).  A sphere (c, r) can be
// met by one of its rays only if the forward cone from O with half-angle
// theta meets the sphere grown by rho (shifting a ray's origin to O moves
// each of its points by at most rho).
struct RayBundle {
  float O[3], ax[3];
  float rho, theta;
  bool any, prune;
};

__device__ __forceinline__ bool bundle_meets_sphere(const RayBundle& b, const float c[3], float r) {
  const float v[3] = {c[0] - b.O[0], c[1] - b.O[1], c[2] - b.O[2]};
  const float L = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const float R = r + b.rho + 1e-4f * (L + r) + 1e-6f;
  if (L <= R) return true;
  const float cphi = fminf(fmaxf((v[0] * b.ax[0] + v[1] * b.ax[1] + v[2] * b.ax[2]) / L, -1.0f), 1.0f);
  return acosf(cphi) <= b.theta + asinf(R / L) + 1e-4f;
}

template <int PASS, bool CAMERA>
__global__ __launch_bounds__(256) void k_cull(KArgs a) {
  __shared__ int s_cand[CULL_BATCH];
  __shared__ int s_wsum[4];
  __shared__ int s_cnt[NEDF_MAX_OBJECTS], s_base[NEDF_MAX_OBJECTS];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int64_t ray;
  bool live;
  TileFrustum f;
  if constexpr (CAMERA) {
    const int W = a.rays.width, H = a.rays.height;
    const int px = blockIdx.x * CULL_TILE + (t % CULL_TILE), py = blockIdx.y * CULL_TILE + (t / CULL_TILE);
    live = px < W && py < H;
    ray = int64_t(py) * W + px;
    // pixel-centre extremes of the tile as slopes in the camera basis
    const float ax = sqrtf(a.rays.right[0] * a.rays.right[0] + a.rays.right[1] * a.rays.right[1] +
                           a.rays.right[2] * a.rays.right[2]);
    const float ay = sqrtf(a.rays.up[0] * a.rays.up[0] + a.rays.up[1] * a.rays.up[1] + a.rays.up[2] * a.rays.up[2]);
    for (int i = 0; i < 3; ++i) {
      f.eye[i] = a.rays.eye[i];
      f.rh[i] = a.rays.right[i] / ax;
      f.uh[i] = a.rays.up[i] / ay;
      f.fw[i] = a.rays.fwd[i];
    }
    const int i0 = blockIdx.x * CULL_TILE, i1 = min(W, i0 + CULL_TILE) - 1;
    const int j0 = blockIdx.y * CULL_TILE, j1 = min(H, j0 + CULL_TILE) - 1;
    f.nx0 = ax * (2.0f * (float(i0) + 0.5f) / float(W) - 1.0f);
    f.nx1 = ax * (2.0f * (float(i1) + 0.5f) / float(W) - 1.0f);
    f.ny1 = ay * (1.0f - 2.0f * (float(j0) + 0.5f) / float(H));
    f.ny0 = ay * (1.0f - 2.0f * (float(j1) + 0.5f) / float(H));
  } else if (a.ray_grid_w > 0) {
    // image-shaped ray array: 16 x 16 tiles give tight bundles
    const int W = a.ray_grid_w;
    const int px = blockIdx.x * CULL_TILE + (t % CULL_TILE), py = blockIdx.y * CULL_TILE + (t / CULL_TILE);
    ray = int64_t(py) * W + px;
    live = px < W && ray < a.n_rays;
  } else {
    ray = int64_t(blockIdx.x) * blockDim.x + t;
    live = ray < a.n_rays;
  }
  float o[3] = {0, 0, 0}, d[3] = {0, 0, 1};
  if (live) make_ray(a.rays, ray, o, d);
  RayBundle bd;
  if constexpr (!CAMERA) {
    // bundle of the workgroup's rays with a finite direction
    __shared__ float s_red[4][8];
    const bool ok = live && isfinite(d[0]) && isfinite(d[1]) && isfinite(d[2]) && isfinite(o[0]) &&
                    isfinite(o[1]) && isfinite(o[2]);
    float acc[7] = {ok ? o[0] : 0.f, ok ? o[1] : 0.f, ok ? o[2] : 0.f, ok ? d[0] : 0.f, ok ? d[1] : 0.f,
                    ok ? d[2] : 0.f, ok ? 1.f : 0.f};
    for (int i = 0; i < 7; ++i)
      for (int off = 32; off > 0; off >>= 1) acc[i] += __shfl_xor(acc[i], off);
    if (lane == 0)
      for (int i = 0; i < 7; ++i) s_red[wave][i] = acc[i];
    __syncthreads();
    float tot[7];
    for (int i = 0; i < 7; ++i) tot[i] = s_red[0][i] + s_red[1][i] + s_red[2][i] + s_red[3][i];
    bd.any = tot[6] > 0.f;
    const float n = fmaxf(tot[6], 1.f);
    const float dl = sqrtf(tot[3] * tot[3] + tot[4] * tot[4] + tot[5] * tot[5]);
    for (int i = 0; i < 3; ++i) {
      bd.O[i] = tot[i] / n;
      bd.ax[i] = dl > 0.f ? tot[3 + i] / dl : 0.f;
    }
    float rho = 0.f, ct = 1.f;
    if (ok) {
      const float e[3] = {o[0] - bd.O[0], o[1] - bd.O[1], o[2] - bd.O[2]};
      rho = sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
      ct = d[0] * bd.ax[0] + d[1] * bd.ax[1] + d[2] * bd.ax[2];
    }
    for (int off = 32; off > 0; off >>= 1) {
      rho = fmaxf(rho, __shfl_xor(rho, off));
      ct = fminf(ct, __shfl_xor(ct, off));
    }
    __syncthreads();
    if (lane == 0) {
      s_red[wave][0] = rho;
      s_red[wave][1] = ct;
    }
    __syncthreads();
    bd.rho = fmaxf(fmaxf(s_red[0][0], s_red[1][0]), fmaxf(s_red[2][0], s_red[3][0]));
    const float cmin = fminf(fminf(s_red[0][1], s_red[1][1]), fminf(s_red[2][1], s_red[3][1]));
    bd.theta = acosf(fminf(fmaxf(cmin, -1.0f), 1.0f));
    // prune only coherent bundles (a wide one would keep nearly everything)
    bd.prune = bd.any && a.clip && cmin > 0.5f && dl > 0.f;
  }
  PairList* L = &a.C->A;
  if (t < NEDF_MAX_OBJECTS) s_cnt[t] = 0;
  float dlo = INFINITY, dhi = 0.0f;  // range of the pairs' depth bounds (pass 0)
  __syncthreads();
  // traversal 0 counts; in pass 1 traversal 1 writes
  for (int trav = 0; trav <= PASS; ++trav) {
    for (int base = 0; base < a.n_inst; base += CULL_BATCH) {
      const int nb = min(CULL_BATCH, a.n_inst - base);
      int nc = 0;
      bool compact = CAMERA;
      if constexpr (!CAMERA) compact = bd.prune || !bd.any;
      if (compact) {
        // ordered compaction of the instances whose sphere meets the tile
        // (camera rays) or the ray bundle (ray arrays)
        __syncthreads();
        for (int c0 = 0; c0 < nb; c0 += 256) {
          const int k = base + c0 + t;
          bool keep = false;
          if (c0 + t < nb) {
            const int obj = a.inst_object[k];
            if (obj >= 0 && obj < a.n_obj) {
              if constexpr (CAMERA) {
                if (!a.clip) {
                  keep = true;
                } else {
                  float c[3], r;
                  instance_sphere(a, k, obj, c, r);
                  keep = tile_meets_sphere(f, c, r);
                }
              } else if (bd.any) {
                float c[3], r;
                instance_sphere(a, k, obj, c, r);
                keep = bundle_meets_sphere(bd, c, r);
              }
            }
          }
          const uint64_t m = __ballot(keep);
          if (lane == 0) s_wsum[wave] = __popcll(m);
          __syncthreads();
          int off = nc;
          for (int w = 0; w < wave; ++w) off += s_wsum[w];
          const int tot = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
          if (keep) s_cand[off + __popcll(m & ((1ull << lane) - 1ull))] = k;
          nc += tot;
          __syncthreads();
        }
      } else {
        nc = nb;
      }
      for (int ci = 0; ci < nc; ++ci) {
        const int k = compact ? s_cand[ci] : base + ci;
        const int obj = a.inst_object[k];
        float dm = 0.0f;
        const bool pass = live && obj >= 0 && obj < a.n_obj && pair_test(a, o, d, k, obj, dm);
        const uint64_t m = __ballot(pass);
        if (m == 0) continue;
        const int cnt = __popcll(m);
        const int leader = __ffsll((unsigned long long)m) - 1;
        if (trav == 0) {
          if (lane == leader) atomicAdd(&s_cnt[obj], cnt);
          if (PASS == 0 && pass) {
            dlo = fminf(dlo, dm);
            dhi = fmaxf(dhi, dm);
          }
        } else {
          int off = 0;
          if (lane == leader) off = atomicAdd(&s_cnt[obj], cnt);
          off = __shfl(off, leader);
          if (pass) {
            const int pos = s_base[obj] + off + __popcll(m & ((1ull << lane) - 1ull));
            if (pos < L->cnt[obj]) {
              a.pairs[L->off[obj] + pos] = make_uint2(uint32_t(ray), uint32_t(k));
              a.pair_dm[L->off[obj] + pos] = dm;
            }
          }
        }
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
  if constexpr (PASS == 0) {
    // range of the workgroup's bounds, then one atomic pair per workgroup
    // (atomics on one word from every wave of the chip serialise)
    __shared__ float s_rng[2][4];
    for (int off = 32; off > 0; off >>= 1) {
      dlo = fminf(dlo, __shfl_xor(dlo, off));
      dhi = fmaxf(dhi, __shfl_xor(dhi, off));
    }
    if (lane == 0) {
      s_rng[0][wave] = dlo;
      s_rng[1][wave] = dhi;
    }
    __syncthreads();
    if (t == 0) {
      dlo = fminf(fminf(s_rng[0][0], s_rng[0][1]), fminf(s_rng[0][2], s_rng[0][3]));
      dhi = fmaxf(fmaxf(s_rng[1][0], s_rng[1][1]), fmaxf(s_rng[1][2], s_rng[1][3]));
      if (dlo <= dhi) {
        atomicMin(&a.C->dmin_bits, __float_as_uint(dlo));
        atomicMax(&a.C->dmax_bits, __float_as_uint(dhi));
      }
    }
  }
}

// Segment offsets of list A (clamped to capacity) and work items over the
// objects in item_mask.  List B gets the same segments, empty.
__global__ void k_scan_A(KArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  PairList* L = &a.C->A;
  PairList* B = &a.C->B;
  int64_t off = 0;
  int items = 0;
  bool over = false;
  for (int m = 0; m < a.n_obj; ++m) {
    int64_t c = L->cnt[m];
    if (off + c > a.capacity) {
      c = a.capacity - off > 0 ? a.capacity - off : 0;
      over = true;
    }
    L->cnt[m] = int32_t(c);
    L->off[m] = int32_t(off);
    B->off[m] = int32_t(off);
    B->cnt[m] = 0;
    L->item_start[m] = items;
    if ((a.item_mask >> m) & 1u) items += int32_t((c + a.item_pairs - 1) / a.item_pairs);
    L->fill[m] = 0;
    off += c;
  }
  L->off[a.n_obj] = int32_t(off);
  B->off[a.n_obj] = int32_t(off);
  L->item_start[a.n_obj] = items;
  L->total_items = items;
  L->total_pairs = int32_t(off);
  L->work_counter = 0;
  a.C->stats[4] = int32_t(off);  // pairs after culling (kept when later stages rebin list A)
  if (over) set_status(a.status, NEDF_ERR_CAPACITY);
}

// Work items over an already-filled list (segments fixed): list B after the
// network stage, or list A for a second pass with another item size.
__global__ void k_scan_items(KArgs a, PairList* L) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
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

// Front-to-back network stage.  A pair can report no depth below its bound
// s (t_perp - l) (kept per pair by the culling pass, with the bounds' range):
// the network's depth is s (t_perp - l clamp(mu_hat, -1, 1)) and the
// marcher's lies inside the chord, which starts at or after it.  The pairs
// are split into depth slabs of that bound and the network runs slab by slab,
// nearest first; a pair whose bound lies beyond the pixel's nearest hit so far
// cannot win the min-reduce and is skipped.  The result is the same as
// evaluating every pair, whatever the slab boundaries.

__global__ void k_slab_begin(KArgs a) {
  if (blockIdx.x != 0) return;
  PairList* S = &a.C->S;
  const PairList* A = &a.C->A;
  for (int m = threadIdx.x; m < NEDF_MAX_OBJECTS; m += blockDim.x) {
    S->cnt[m] = 0;
    S->off[m] = A->off[m];
  }
}

// Candidates a lane tests at once in the slab filters.
constexpr int SLAB_U = 8;

// Wave-aggregated append of the kept pairs (SLAB_U per lane) to their
// objects' segments of list S: one atomic per object present reserves the
// slots of all of them.  Called with the whole wave active.
__device__ __forceinline__ void push_slab(const KArgs& a, PairList* S, int lane, const bool (&keep)[SLAB_U],
                                          const int (&m)[SLAB_U], const uint2 (&pr)[SLAB_U]) {
  uint64_t pend[SLAB_U];
#pragma unroll
  for (int u = 0; u < SLAB_U; ++u) pend[u] = __ballot(keep[u]);
  const uint64_t below = (1ull << lane) - 1ull;
  for (;;) {
    int m0 = -1;
#pragma unroll
    for (int u = 0; u < SLAB_U; ++u)
      if (m0 < 0 && pend[u]) m0 = __builtin_amdgcn_readlane(m[u], __ffsll((unsigned long long)pend[u]) - 1);
    if (m0 < 0) break;
    bool mine[SLAB_U];
    int pos[SLAB_U], tot = 0;
#pragma unroll
    for (int u = 0; u < SLAB_U; ++u) {
      mine[u] = keep[u] && m[u] == m0;
      const uint64_t mk = __ballot(mine[u]);
      pos[u] = tot + __popcll(mk & below);
      tot += __popcll(mk);
      pend[u] &= ~mk;
    }
    int base = 0;
    if (lane == 0) base = atomicAdd(&S->cnt[m0], tot);
    const int run = S->off[m0] + __builtin_amdgcn_readfirstlane(base);
    for (int u = 0; u < SLAB_U; ++u)
      if (mine[u]) a.pairsS[run + pos[u]] = pr[u];
  }
}

// Tests the pairs whose bits are set in `hits` (lane's pairs q0 + j) against
// the pixels' current nearest hits and appends the survivors to list S.  The
// wave first compacts the candidate indices in LDS (`cand`, 1024 entries) and
// then takes them 64 * SLAB_U at a time, SLAB_U per lane, so that the bound,
// pair and key reads of all of them are in flight together.  Called with the
// whole wave active.
__device__ __forceinline__ void slab_candidates(const KArgs& a, PairList* S, int* cand, int lane, int q0,
                                                uint32_t hits) {
  const int c = __popc(hits);
  int incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  const int n_cand = __shfl(incl, 63);
  if (n_cand == 0) return;
  int k = incl - c;
  while (hits) {
    cand[k++] = q0 + __ffs(hits) - 1;
    hits &= hits - 1u;
  }
  __builtin_amdgcn_wave_barrier();
  for (int c0 = 0; c0 < n_cand; c0 += 64 * SLAB_U) {
    bool keep[SLAB_U];
    int q[SLAB_U], m[SLAB_U];
    uint2 pr[SLAB_U];
    float dm[SLAB_U];
    // lanes past the last candidate read the round's first one and drop it
    const int q_first = cand[c0];
#pragma unroll
    for (int u = 0; u < SLAB_U; ++u) {
      const int idx = c0 + 64 * u + lane;
      keep[u] = idx < n_cand;
      q[u] = keep[u] ? cand[idx] : q_first;
    }
#pragma unroll
    for (int u = 0; u < SLAB_U; ++u) {
      pr[u] = a.pairs[q[u]];
      dm[u] = a.pair_dm[q[u]];
    }
#pragma unroll
    for (int u = 0; u < SLAB_U; ++u) {
      m[u] = a.inst_object[pr[u].y];
      // margin against last-bit differences between kernels
      keep[u] = keep[u] && !(depth_limit(a, pr[u].x) < dm[u] - (1e-5f * dm[u] + 1e-5f));
    }
    push_slab(a, S, lane, keep, m, pr);
  }
  __builtin_amdgcn_wave_barrier();
}

// List S = the pairs of list A in depth slab 0 (objects in mask) whose bound
// does not lie beyond the pixel's current nearest hit.  Also records every
// pair's slab in one byte (0xFF for objects outside the mask) and, per block
// of SLAB_BLOCK pairs, the set of slabs present, so that the later slabs skip
// blocks without their pairs and read one byte per pair in the others.  A
// wave takes one block: sixteen consecutive pairs per lane.
__global__ __launch_bounds__(256) void k_slab_first(KArgs a, uint32_t mask, int n_slabs) {
  __shared__ int s_cand[4][SLAB_BLOCK];
  __shared__ int s_off[NEDF_MAX_OBJECTS + 1];
  const PairList* A = &a.C->A;
  PairList* S = &a.C->S;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // segment offsets and the slab map, read once (the loop below stores to
  // global memory, so the compiler could not keep them in registers)
  if (threadIdx.x <= a.n_obj) s_off[threadIdx.x] = A->off[threadIdx.x];
  const float lo = __uint_as_float(a.C->dmin_bits), hi = __uint_as_float(a.C->dmax_bits);
  const bool single = n_slabs <= 1 || !(hi > lo);
  const float inv_w = single ? 0.0f : float(n_slabs) / (hi - lo);
  __syncthreads();
  const int total = s_off[a.n_obj];
  const int nblk = (total + SLAB_BLOCK - 1) / SLAB_BLOCK;
  const float4* dv = reinterpret_cast<const float4*>(a.pair_dm);
  uint4* sv = reinterpret_cast<uint4*>(a.pair_slab);
  const int wstride = gridDim.x * 4;
  for (int blk = blockIdx.x * 4 + wave; blk < nblk; blk += wstride) {
    const int q0 = blk * SLAB_BLOCK + 16 * lane;
    uint32_t bits = 0, hits = 0;
    if (q0 < total) {
      uint32_t bytes[4];
      int mo = 0;
      while (mo + 1 < a.n_obj && q0 >= s_off[mo + 1]) ++mo;
      int next_off = mo + 1 < a.n_obj ? s_off[mo + 1] : 0x7FFFFFFF;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float4 v = dv[q0 / 4 + i];
        const float dm[4] = {v.x, v.y, v.z, v.w};
        uint32_t by = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int q = q0 + 4 * i + j;
          while (q >= next_off) {
            ++mo;
            next_off = mo + 1 < a.n_obj ? s_off[mo + 1] : 0x7FFFFFFF;
          }
          int sl = 0xFF;
          if (q < total && ((mask >> mo) & 1u)) {
            if (single) {
              sl = 0;
            } else {
              const int kk = int((dm[j] - lo) * inv_w);
              sl = kk < 0 ? 0 : (kk >= n_slabs ? n_slabs - 1 : kk);
            }
            bits |= 1u << sl;
            if (sl == 0) hits |= 1u << (4 * i + j);
          }
          by |= uint32_t(sl) << (8 * j);
        }
        bytes[i] = by;
      }
      sv[q0 / 16] = make_uint4(bytes[0], bytes[1], bytes[2], bytes[3]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bits |= __shfl_xor(bits, off);
    if (lane == 0) a.slab_mask[blk] = bits;
    slab_candidates(a, S, s_cand[wave], lane, q0, hits);
  }
}

// List S for slab `slab` >= 1: a wave takes one block of SLAB_BLOCK pairs,
// skips it unless its slab set holds `slab`, else scans the slab bytes
// (sixteen per lane, one 16-byte load) and tests the matching pairs.
__global__ __launch_bounds__(256) void k_slab_next(KArgs a, int slab) {
  __shared__ int s_cand[4][SLAB_BLOCK];
  const PairList* A = &a.C->A;
  PairList* S = &a.C->S;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int total = A->off[a.n_obj];
  const int nblk = (total + SLAB_BLOCK - 1) / SLAB_BLOCK;
  const uint4* sv = reinterpret_cast<const uint4*>(a.pair_slab);
  const uint32_t pat = 0x01010101u * uint32_t(slab);
  const int wstride = gridDim.x * 4;
  for (int blk = blockIdx.x * 4 + wave; blk < nblk; blk += wstride) {
    if (!((a.slab_mask[blk] >> slab) & 1u)) continue;
    const int q0 = blk * SLAB_BLOCK + 16 * lane;
    uint32_t hits = 0;  // bit j: pair q0 + j is in this slab
    if (q0 < total) {
      const uint4 b = sv[q0 / 16];
      const uint32_t wd[4] = {b.x ^ pat, b.y ^ pat, b.z ^ pat, b.w ^ pat};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (((wd[i] >> (8 * j)) & 0xFFu) == 0u) hits |= 1u << (4 * i + j);
      // bytes past the last pair are ignored
      const int rem = total - q0;
      if (rem < 16) hits &= (1u << rem) - 1u;
    }
    slab_candidates(a, S, s_cand[wave], lane, q0, hits);
  }
}

// Depth test of the fallback list (exact): a pair whose ray enters the
// instance's bounding sphere beyond the pixel's current nearest hit cannot
// win the min-reduce, since every marcher sample lies inside the chord and
// the marched depth is a weighted mean of sample depths.  Kept pairs are
// compacted into list A's pair array (free after the network stage) at list
// B's segment offsets; list B's counts are replaced by the kept counts.
__global__ void k_zero_fill(KArgs a) {
  if (blockIdx.x == 0 && threadIdx.x < NEDF_MAX_OBJECTS) a.C->B.fill[threadIdx.x] = 0;
}

__global__ void k_fallback_depth_test(KArgs a, uint2* out) {
  PairList* B = &a.C->B;
  const int lane = threadIdx.x & 63;
  for (int m = 0; m < a.n_obj; ++m) {
    const int cnt = B->cnt[m], off = B->off[m];
    const float bound = a.obj[m].bound;
    // uniform trip count per wave so that the ballot below sees whole waves
    const int stride = gridDim.x * blockDim.x;
    for (int q0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63); q0 < cnt; q0 += stride) {
      const int q = q0 + lane;
      bool keep = false;
      uint2 pr = make_uint2(0u, 0u);
      if (q < cnt) {
        pr = a.pairs[off + q];
        const W2L g = load_w2l(a.w2l, int(pr.y));
        float o[3], d[3], ol[3], dl[3], ta = 0.f, tb = 0.f;
        make_ray(a.rays, pr.x, o, d);
        to_local(g, o, d, ol, dl);
        const bool seg = a.clip ? sphere_chord(ol, dl, bound, ta, tb) : true;
        const float t_in = a.clip ? g.s * ta : a.t_near;
        keep = seg && !(depth_limit(a, pr.x) < t_in);
      }
      const uint64_t mk = __ballot(keep);
      if (mk) {
        const int leader = __ffsll((unsigned long long)mk) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&B->fill[m], __popcll(mk));
        base = __shfl(base, leader);
        if (keep) out[off + base + __popcll(mk & ((1ull << lane) - 1ull))] = pr;
      }
    }
  }
}

__global__ void k_fallback_commit(KArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  PairList* B = &a.C->B;
  int kept = 0;
  for (int m = 0; m < a.n_obj; ++m) {
    B->cnt[m] = B->fill[m];
    kept += B->fill[m];
  }
  a.C->stats[3] = kept;
}

// One thread per pair of an analytic object in `mask`; sequential
// compensated scan.
__global__ void k_march_analytic(KArgs a, uint32_t mask) {
  const PairList* L = a.L;
  for (int m = 0; m < a.n_obj; ++m) {
    const ObjDesc od = a.obj[m];
    if (od.field == NEDF_FIELD_MLP || !((mask >> m) & 1u)) continue;
    const int cnt = L->cnt[m], off = L->off[m];
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
      const uint2 pr = a.pairs[off + q];
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
      const float A = sw + sw_c;
      if (A >= a.hit_thr && A > 0.0f) emit_key(a, pr.x, pr.y, g.s * ((swt + swt_c) / A));
      atomicMax(&a.opac[pr.x], __float_as_uint(fmaxf(A, 0.0f)));
    }
  }
}

// Matrix-core marcher: a workgroup takes items of 4 pairs (one per wave) of
// one object from list a.L; each wave marches its pair in chunks of 32 NB
// samples through the register-resident density network (NB blocks of 32
// share every weight read from LDS), then scans each block's optical depths
// across the wave in sample order, so that the sums are the same for any NB.
template <int DT, int WIDTH, int NHID, int L, int SBX, int OCC, int NB, int NW>
__global__ __launch_bounds__(64 * NW, OCC) void k_march_mlp(KArgs a) {
  using T = eng::Tr<DT>;
  constexpr int KS0 = eng::ks_for_slots<DT>(3 * L + 2);
  constexpr int KSH = WIDTH / T::KPS;
  constexpr int CHUNK = eng::cmax(eng::chunk_bytes<DT>(KS0, 0), eng::chunk_bytes<DT>(KSH, 1));
  constexpr int SPC = 32 * NB;  // samples per wave per chunk
  __shared__ __attribute__((aligned(16))) uint8_t lds[eng::NBUF * eng::slot_bytes(CHUNK, SBX)];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
  PairList* PL = a.L;
  const int N = a.n_samples;
  const int n_chunks = (N + SPC - 1) / SPC;
  const int total = PL->total_items;
  // one item of lookahead: the next item is claimed during the current
  // item's last pass so that its weights stream in behind this one's
  if (threadIdx.x == 0) s_item = atomicAdd(&PL->work_counter, 1);
  __syncthreads();
  int item = s_item;
  int slot = 0;
  bool primed = false;
  while (item < total) {
    const int obj = item_object(PL, a.n_obj, item);
    const int local = (item - PL->item_start[obj]) * NW + wave;
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
    int next = total;
    for (int c = 0; c < n_chunks; ++c) {
      const bool last = c + 1 == n_chunks;
      if (last) {
        __syncthreads();  // every wave has read s_item
        if (threadIdx.x == 0) s_item = atomicAdd(&PL->work_counter, 1);
        __syncthreads();
        next = s_item;
      }
      const uint8_t* next_blob = !last ? blob : (next < total ? a.obj[item_object(PL, a.n_obj, next)].blob : nullptr);
      typename T::frag Benc[NB][KS0];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float tr = (float(c * SPC + 32 * nb + (lane & 31)) + 0.5f) * delta;
        float p[3] = {fmaf(tr, dl[0], pa[0]), fmaf(tr, dl[1], pa[1]), fmaf(tr, dl[2], pa[2])};
        eng::encode_input<DT, 3, L, KS0>(p, half, Benc[nb]);
      }
      float partial[NB][1];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) partial[nb][0] = 0.f;
      typename T::frag Blast[NB][KSH];
      eng::trunk<DT, WIDTH, KS0, NHID, 1, CHUNK, false, 0, WIDTH / 32, SBX, NB, NW>(hb, blob, Benc, lds, partial,
                                                                               Blast, nullptr, &slot, next_blob,
                                                                               primed);
      primed = next_blob != nullptr;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int si = c * SPC + 32 * nb + (lane & 31);
        const float tr = (float(si) + 0.5f) * delta;
        const float p[3] = {fmaf(tr, dl[0], pa[0]), fmaf(tr, dl[1], pa[1]), fmaf(tr, dl[2], pa[2])};
        const float u = partial[nb][0] + __shfl_xor(partial[nb][0], 32) + head_b;
        float v = mlp_sigma(od, u, p[0], p[1], p[2]) * delta;
        if (lane >= 32 || si >= N || !seg) v = 0.f;
        // inclusive scan of optical depth over the wave (sample order = lane order)
        float incl = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const float y = __shfl_up(incl, off);
          if (lane >= off) incl += y;
        }
        const float tau = (carry + carry_c) + (incl - v);
        const float w = expf(-tau) * one_minus_exp_neg(v);
        float ws = w, wts = w * (ta + tr);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          ws += __shfl_xor(ws, off);
          wts += __shfl_xor(wts, off);
        }
        // a block wholly past the last sample adds exact zeros
        neu_add(sw, sw_c, ws);
        neu_add(swt, swt_c, wts);
        neu_add(carry, carry_c, __shfl(incl, 63));
      }
    }
    if (lane == 0 && valid && seg) {
      const float A = sw + sw_c;
      if (A >= a.hit_thr && A > 0.0f) emit_key(a, pr.x, pr.y, g.s * ((swt + swt_c) / A));
      atomicMax(&a.opac[pr.x], __float_as_uint(fmaxf(A, 0.0f)));
    }
    item = next;
  }
}

// NeDF stage: a workgroup takes items of 128 NB pairs (32 NB per wave) of
// one object; each lane pair evaluates the intersection network on its pairs'
// line coordinates (NB blocks of 32 pairs share every weight read from LDS).
// Confident hits go to the key buffer, uncertain pairs (and origins inside
// the bounding sphere) to list B for the marcher.
template <int DT, int WIDTH, int NHID, int L, int SBX, int OCC, int NB, int NW>
__global__ __launch_bounds__(64 * NW, OCC) void k_nedf(KArgs a) {
  using T = eng::Tr<DT>;
  constexpr int PPW = 32 * NB;  // pairs per wave and item
  constexpr int KS0 = eng::ks_for_slots<DT>(6 * L + 3);
  constexpr int KSH = WIDTH / T::KPS;
  constexpr int CHUNK = eng::cmax(eng::chunk_bytes<DT>(KS0, 0), eng::chunk_bytes<DT>(KSH, 2));
  __shared__ __attribute__((aligned(16))) uint8_t lds[eng::NBUF * eng::slot_bytes(CHUNK, SBX)];
  // per-lane pair state parked across the network (keeps registers free)
  constexpr int NT = 64 * NW;
  __shared__ __attribute__((aligned(16))) uint8_t s_stash[16 * NB * NT];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5;
  const uint32_t stash = eng::lds_offset(s_stash) + 16u * threadIdx.x;
  PairList* PL = a.L;  // the current depth slab
  PairList* FB = &a.C->B;
  const int total = PL->total_items;
  if (threadIdx.x == 0) s_item = atomicAdd(&PL->work_counter, 1);
  __syncthreads();
  int item = s_item;
  int slot = 0;
  bool primed = false;
  // routing counts, per wave, flushed once at the end
  int n_hit = 0, n_fb = 0, n_miss = 0;
  while (item < total) {
    // claim the next item now so that its weights stream in behind this pass
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(&PL->work_counter, 1);
    __syncthreads();
    const int next = s_item;
    const int obj = item_object(PL, a.n_obj, item);
    const int first = (item - PL->item_start[obj]) * (PPW * NW) + wave * PPW + (lane & 31);
    const ObjDesc& od = a.obj[obj];
    const uint8_t* blob = od.nedf_blob;
    const uint8_t* next_blob = next < total ? a.obj[item_object(PL, a.n_obj, next)].nedf_blob : nullptr;
    const nedf_blob_header* hb = reinterpret_cast<const nedf_blob_header*>(blob);
    const float* hbias_p = reinterpret_cast<const float*>(blob + uniform_load_u64(&hb->off_head_b));
    const float hbias[2] = {uniform_load_f32(hbias_p), uniform_load_f32(hbias_p + 1)};
    const float l = od.bound;
    typename T::frag Benc[NB][KS0];
    const float in_scale = DT == 2 ? uniform_load_f32(blob + uniform_load_u64(&hb->off_scales)) : 1.0f;
    // lane-half-dependent encoding constants are recomputed per pass rather
    // than hoisted out of the loop (where they would stay live, and spill,
    // across the network)
    int half_v = half;
    asm volatile("" : "+v"(half_v));
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int local = first + 32 * nb;
      const bool valid = local < PL->cnt[obj];
      const uint2 pr = a.pairs[PL->off[obj] + (valid ? local : 0)];
      const W2L g = load_w2l(a.w2l, int(pr.y));
      float o[3], d[3], dlo[3], ol[3], pl[6], pllo[6], tperp;
      make_ray(a.rays, pr.x, o, d, dlo);
      local_line(g, o, d, dlo, pl, pllo, tperp, ol);
      const bool inside = ol[0] * ol[0] + ol[1] * ol[1] + ol[2] * ol[2] < l * l;
      eng::encode_input<DT, 6, L, KS0>(pl, pllo, half_v, Benc[nb], in_scale);
      // ray and instance ids (< 2^31, flags in bit 31), t_perp and s
      eng::lds_write16(stash + uint32_t(nb) * (16u * NT),
                       eng::u32x4{pr.x | (valid ? 0x80000000u : 0u), pr.y | (inside ? 0x80000000u : 0u),
                                  __float_as_uint(tperp), __float_as_uint(g.s)});
    }
    float partial[NB][2];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) partial[nb][0] = partial[nb][1] = 0.f;
    typename T::frag Blast[NB][KSH];
    eng::trunk<DT, WIDTH, KS0, NHID, 2, CHUNK, false, 0, WIDTH / 32, SBX, NB, NW>(hb, blob, Benc, lds, partial, Blast,
                                                                             nullptr, &slot, next_blob, primed);
    primed = next_blob != nullptr;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      eng::u32x4 st = eng::lds_read16<0>(stash + uint32_t(nb) * (16u * NT)), d1 = st, d2 = st, d3 = st;
      eng::lds_wait4<0>(st, d1, d2, d3);
      const uint2 prs = make_uint2(st.x & 0x7FFFFFFFu, st.y & 0x7FFFFFFFu);
      const bool valid_s = (st.x >> 31) != 0, inside_s = (st.y >> 31) != 0;
      const float mu_hat = partial[nb][0] + __shfl_xor(partial[nb][0], 32) + hbias[0];
      const float z = partial[nb][1] + __shfl_xor(partial[nb][1], 32) + hbias[1];
      const float p = sigmoidf_(z);
      const float D = __uint_as_float(st.w) * (__uint_as_float(st.z) - l * fminf(fmaxf(mu_hat, -1.0f), 1.0f));
      const bool mine = valid_s && half == 0;
      const bool to_fb = mine && (inside_s || (p >= a.p_lo && p <= a.p_hi));
      const bool hit = mine && !to_fb && p > a.p_hi && D > 0.0f;
      if (hit) emit_key(a, prs.x, prs.y, D);
      // wave-aggregated push into the object's segment of list B
      const uint64_t m = __ballot(to_fb);
      if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&FB->cnt[obj], __popcll(m));
        base = __shfl(base, leader);
        if (to_fb) a.pairsB[FB->off[obj] + base + __popcll(m & ((1ull << lane) - 1ull))] = prs;
      }
      const uint64_t mh = __ballot(hit), mv = __ballot(mine);
      n_hit += __popcll(mh);
      n_fb += __popcll(m);
      n_miss += __popcll(mv) - __popcll(mh) - __popcll(m);
    }
    item = next;
  }
  if (lane == 0 && (n_hit | n_fb | n_miss)) {
    atomicAdd(&a.C->stats[0], n_hit);
    atomicAdd(&a.C->stats[1], n_fb);
    atomicAdd(&a.C->stats[2], n_miss);
  }
}

__global__ void k_finalize(KArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n_rays) return;
  const uint64_t k = a.keys[i];
  if (k == NEDF_KEY_EMPTY) {
    a.depth[i] = __int_as_float(0x7f800000);
    if (a.id) a.id[i] = -1;
  } else {
    a.depth[i] = __uint_as_float(uint32_t(k >> 32));
    if (a.id) a.id[i] = int32_t(uint32_t(k & 0xffffffffu));
  }
  if (a.opacity) a.opacity[i] = __uint_as_float(a.opac[i]);
}

// Buffer reuse (Sec. "CUDA implementation"): the depth keys of several
// disjoint instance sets, each computed on its own, merged by their minimum
// into the workspace's keys, which then hold what one pass over the union
// would have left there (the minimum is order-free and every pair's key
// depends on its ray and instance alone).  Keys naming an instance at or
// beyond n_inst are dropped and flag NEDF_ERR_SHAPE in the status word
// (cleared by the caller beforehand).  Also clears the counters as k_init.
__global__ void k_merge_keys(KArgs a, KeySets ks) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < a.n_rays) {
    uint64_t m = NEDF_KEY_EMPTY;
    bool bad = false;
    for (int j = 0; j < ks.n; ++j) {
      const uint64_t k = ks.p[j][i];
      if (k == NEDF_KEY_EMPTY) continue;
      if (uint32_t(k & 0xffffffffu) >= uint32_t(a.n_inst)) {
        bad = true;
        continue;
      }
      m = k < m ? k : m;
    }
    a.keys[i] = m;
    a.opac[i] = 0u;
    if (bad) set_status(a.status, NEDF_ERR_SHAPE);
  }
  constexpr int64_t words = int64_t(sizeof(WsCounters) / 4);
  for (int64_t w = i; w < words; w += int64_t(gridDim.x) * blockDim.x)
    reinterpret_cast<int32_t*>(a.C)[w] = w == int64_t(offsetof(WsCounters, dmin_bits) / 4) ? 0x7F800000 : 0;
}

int cu_count() {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 256;
  }
  return ncu;
}

// Launch shape of the 256-wide BF16/FP8 kernels from the tuning table: value
// 100 * (32-row blocks per wave - 1) + 10 * occupancy + superchunk (blocks
// sharing each weight read, workgroups per CU, chunks per copy); other shapes
// use one block, one workgroup per CU and the default superchunk.  The grid
// is persistent: one workgroup per CU and occupancy level.
// Tuning value of the matrix-core kernels: 1000 * (workgroup waves / 4 - 1) +
// 100 * (row blocks per wave - 1) + 10 * workgroups per CU + chunks per
// superchunk.
int tune_waves(int v) { return v >= 1000 ? 8 : 4; }
int nedf_rows(int v) { return v % 1000 >= 100 ? 2 : 1; }

template <int DT, int WIDTH, int NHID, int L>
void launch_march_mlp(const KArgs& k, hipStream_t s) {
  const dim3 b4(256), b8(512), g1(cu_count()), g2(2 * cu_count());
  if constexpr (DT == 1 && WIDTH == 256) {
    switch (tune_value(NEDF_TUNE_MARCH, DT)) {
      case 11: hipLaunchKernelGGL((k_march_mlp<DT, WIDTH, NHID, L, 1, 1, 1, 4>), g1, b4, 0, s, k); return;
      case 21: hipLaunchKernelGGL((k_march_mlp<DT, WIDTH, NHID, L, 1, 2, 1, 4>), g2, b4, 0, s, k); return;
      case 111: hipLaunchKernelGGL((k_march_mlp<DT, WIDTH, NHID, L, 1, 1, 2, 4>), g1, b4, 0, s, k); return;
      case 112: hipLaunchKernelGGL((k_march_mlp<DT, WIDTH, NHID, L, 2, 1, 2, 4>), g1, b4, 0, s, k); return;
      case 1011: hipLaunchKernelGGL((k_march_mlp<DT, WIDTH, NHID, L, 1, 1, 1, 8>), g1, b8, 0, s, k); return;
      case 1012: hipLaunchKernelGGL((k_march_mlp<DT, WIDTH, NHID, L, 2, 1, 1, 8>), g1, b8, 0, s, k); return;
      default: break;
    }
  }
  hipLaunchKernelGGL((k_march_mlp<DT, WIDTH, NHID, L, eng::sb_default<DT>(), 1, 1, 4>), g1, b4, 0, s, k);
}

template <int DT>
void launch_nedf_net(const KArgs& k, hipStream_t s, int v) {
  const dim3 b4(256), b8(512), g1(cu_count()), g2(2 * cu_count());
  if constexpr (DT == 2) {
    switch (v) {
      case 11: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 1, 1, 1, 4>), g1, b4, 0, s, k); return;
      case 12: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 2, 1, 1, 4>), g1, b4, 0, s, k); return;
      case 21: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 1, 2, 1, 4>), g2, b4, 0, s, k); return;
      case 22: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 2, 2, 1, 4>), g2, b4, 0, s, k); return;
      case 1011: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 1, 1, 1, 8>), g1, b8, 0, s, k); return;
      case 1012: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 2, 1, 1, 8>), g1, b8, 0, s, k); return;
      case 1014: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 4, 1, 1, 8>), g1, b8, 0, s, k); return;
      default: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 4, 1, 1, 4>), g1, b4, 0, s, k); return;
    }
  } else if constexpr (DT == 1) {
    switch (v) {
      case 11: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 1, 1, 1, 4>), g1, b4, 0, s, k); return;
      case 21: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 1, 2, 1, 4>), g2, b4, 0, s, k); return;
      case 111: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 1, 1, 2, 4>), g1, b4, 0, s, k); return;
      case 112: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 2, 1, 2, 4>), g1, b4, 0, s, k); return;
      case 1011: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 1, 1, 1, 8>), g1, b8, 0, s, k); return;
      case 1012: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 2, 1, 1, 8>), g1, b8, 0, s, k); return;
      default: hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 2, 1, 1, 4>), g1, b4, 0, s, k); return;
    }
  } else if constexpr (DT == 3) {
    // MX: superchunks of four blocks; eight waves (items of 256 pairs) or four
    if (v >= 1000) hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 4, 1, 1, 8>), g1, b8, 0, s, k);
    else hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 4, 1, 1, 4>), g1, b4, 0, s, k);
  } else {
    hipLaunchKernelGGL((k_nedf<DT, 256, 8, 8, 1, 1, 1, 4>), g1, b4, 0, s, k);
  }
}

unsigned grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return unsigned(g > 0 ? g : 1);
}

}  // namespace

int march_waves(int dtype, int width) {
  if (dtype != NEDF_BF16 || width != 256) return 4;
  return tune_waves(tune_value(NEDF_TUNE_MARCH, dtype));
}

bool march_mlp_supported(int dtype, int width, int n_hidden, int L) {
  if (dtype != NEDF_F32 && dtype != NEDF_BF16) return false;
  return (width == 64 && n_hidden == 3 && L == 6) || (width == 256 && n_hidden == 8 && L == 10);
}

bool nedf_net_supported(int dtype, int width, int n_hidden, int L) {
  if (dtype != NEDF_F32 && dtype != NEDF_BF16 && dtype != NEDF_FP8 && dtype != NEDF_FP8_MX) return false;
  return width == 256 && n_hidden == 8 && L == 8;
}

bool nedf_cls_supported(int dtype, const nedf_mlp_shape& s) {
  if (dtype != NEDF_F32 && dtype != NEDF_BF16) return false;
  return s.in_kind == NEDF_IN_POINTS16 && s.width == 256 && s.enc_L == 10 && s.n_hidden >= 1 && s.n_hidden <= 64 &&
         s.n_out == 1 + NEDF_CLS_COARSE + NEDF_CLS_FINE;
}

bool shade_supported(int dtype, const nedf_mlp_shape& s) {
  if (dtype != NEDF_F32 && dtype != NEDF_BF16) return false;
  return s.width == 256 && s.n_hidden == 8 && s.enc_L == 10 && s.rgb_width == 128 && s.dir_L == 4;
}

bool refine_supported(int dtype, const nedf_mlp_shape& s) {
  if (dtype != NEDF_F32 && dtype != NEDF_BF16) return false;
  return s.width == 256 && s.n_hidden == 8 && s.enc_L == 10;
}

void stage_init_cull(const KArgs& k0, hipStream_t s, uint32_t item_mask, int item_pairs) {
  KArgs k = k0;
  k.item_mask = item_mask;
  k.item_pairs = item_pairs;
  k.L = &k.C->A;
  const unsigned g = grid_for(k.n_rays);
  prof_mark("depth.cull", s, true);
  hipLaunchKernelGGL(k_init, dim3(g), dim3(256), 0, s, k);
  if (k.rays.kind == 0) {
    const dim3 tg((k.rays.width + CULL_TILE - 1) / CULL_TILE, (k.rays.height + CULL_TILE - 1) / CULL_TILE);
    hipLaunchKernelGGL((k_cull<0, true>), tg, dim3(256), 0, s, k);
    hipLaunchKernelGGL(k_scan_A, dim3(1), dim3(64), 0, s, k);
    hipLaunchKernelGGL((k_cull<1, true>), tg, dim3(256), 0, s, k);
  } else {
    dim3 ag(g);
    if (k.ray_grid_w > 0) {
      const int64_t h = (k.n_rays + k.ray_grid_w - 1) / k.ray_grid_w;
      ag = dim3((k.ray_grid_w + CULL_TILE - 1) / CULL_TILE, unsigned((h + CULL_TILE - 1) / CULL_TILE));
    }
    hipLaunchKernelGGL((k_cull<0, false>), ag, dim3(256), 0, s, k);
    hipLaunchKernelGGL(k_scan_A, dim3(1), dim3(64), 0, s, k);
    hipLaunchKernelGGL((k_cull<1, false>), ag, dim3(256), 0, s, k);
  }
  prof_mark("depth.cull", s, false);
}

void stage_march(const KArgs& k0, hipStream_t s, bool list_b, uint32_t analytic_mask, int dtype, int W, int H,
                 int Lenc) {
  (void)H;
  (void)Lenc;
  KArgs k = k0;
  k.L = list_b ? &k.C->B : &k.C->A;
  if (list_b) {
    // depth-test the fallback pairs against the network's hits, compacting
    // them into list A's array, which the marcher then reads
    k.pairs = k.pairsB;
    hipLaunchKernelGGL(k_zero_fill, dim3(1), dim3(64), 0, s, k);
    hipLaunchKernelGGL(k_fallback_depth_test, dim3(2048), dim3(256), 0, s, k, k0.pairs);
    hipLaunchKernelGGL(k_fallback_commit, dim3(1), dim3(64), 0, s, k);
    k.pairs = k0.pairs;
  }
  if (list_b) {
    k.item_mask = 0;
    for (int m = 0; m < k.n_obj; ++m)
      if (k.obj[m].field == NEDF_FIELD_MLP) k.item_mask |= 1u << m;
    k.item_pairs = march_waves(dtype, W);
    hipLaunchKernelGGL(k_scan_items, dim3(1), dim3(64), 0, s, k, k.L);
  }
  if (analytic_mask) {
    prof_mark(list_b ? "fallback.analytic" : "march.analytic", s, true);
    hipLaunchKernelGGL(k_march_analytic, dim3(512), dim3(256), 0, s, k, analytic_mask);
    prof_mark(list_b ? "fallback.analytic" : "march.analytic", s, false);
  }
  if (W > 0) {
    prof_mark(list_b ? "fallback.mlp" : "march.mlp", s, true);
    if (dtype == NEDF_BF16) {
      if (W == 256) launch_march_mlp<1, 256, 8, 10>(k, s);
      else launch_march_mlp<1, 64, 3, 6>(k, s);
    } else {
      if (W == 256) launch_march_mlp<0, 256, 8, 10>(k, s);
      else launch_march_mlp<0, 64, 3, 6>(k, s);
    }
    prof_mark(list_b ? "fallback.mlp" : "march.mlp", s, false);
  }
}

void stage_nedf(const KArgs& k0, hipStream_t s, int dtype, uint32_t nedf_mask, int n_slabs, bool classifier) {
  KArgs k = k0;
  prof_mark("infer.nedf", s, true);
  k.L = &k.C->S;
  k.pairs = k.pairsS;
  k.item_mask = nedf_mask;
  // launch shape from the tuning table, fixed for all slabs of the stage
  const int v = dtype == NEDF_F32 ? 11 : dtype == NEDF_FP8_MX ? 1014 : tune_value(NEDF_TUNE_NEDF, dtype);
  k.item_pairs = classifier ? 32 * 4 : 32 * tune_waves(v) * nedf_rows(v);
  for (int slab = 0; slab < n_slabs; ++slab) {
    hipLaunchKernelGGL(k_slab_begin, dim3(1), dim3(64), 0, s, k);
    if (slab == 0) hipLaunchKernelGGL(k_slab_first, dim3(2048), dim3(256), 0, s, k0, nedf_mask, n_slabs);
    else hipLaunchKernelGGL(k_slab_next, dim3(2048), dim3(256), 0, s, k0, slab);
    hipLaunchKernelGGL(k_scan_items, dim3(1), dim3(64), 0, s, k, k.L);
    prof_mark("net", s, true);
    if (classifier) launch_nedf_cls(k, s, dtype);
    else if (dtype == NEDF_FP8) launch_nedf_net<2>(k, s, v);
    else if (dtype == NEDF_FP8_MX) launch_nedf_net<3>(k, s, v);
    else if (dtype == NEDF_BF16) launch_nedf_net<1>(k, s, v);
    else launch_nedf_net<0>(k, s, v);
    prof_mark("net", s, false);
  }
  prof_mark("infer.nedf", s, false);
}

void stage_merge_keys(const KArgs& k, hipStream_t s, const KeySets& ks) {
  prof_mark("compose.merge", s, true);
  hipLaunchKernelGGL(k_merge_keys, dim3(grid_for(k.n_rays)), dim3(256), 0, s, k, ks);
  prof_mark("compose.merge", s, false);
}

void stage_finalize(const KArgs& k, hipStream_t s) {
  prof_mark("depth.finalize", s, true);
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(k.n_rays)), dim3(256), 0, s, k);
  prof_mark("depth.finalize", s, false);
}

}  // namespace nedf
