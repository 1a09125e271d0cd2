// Device-side types and helpers shared by the HIP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blob_layout.h"

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

#define NEDF_WS_STATUS 0          // int32 status word at workspace offset 0
#define NEDF_KEY_EMPTY 0x7F800000FFFFFFFFull  // (+inf bits << 32) | 0xFFFFFFFF

// Loads of wave-uniform values through the scalar cache.  The address is made
// provably uniform (readfirstlane) and read through the constant address
// space, so the load is counted with the LDS/scalar operations and waiting
// for it never waits for outstanding vector-memory (global->LDS) copies.
__device__ __forceinline__ const void* uniform_ptr(const void* p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
  return reinterpret_cast<const void*>((uint64_t(hi) << 32) | lo);
}
__device__ __forceinline__ uint64_t uniform_load_u64(const void* p) {
  typedef __attribute__((address_space(4))) const uint64_t cu64;
  return *(cu64*)uniform_ptr(p);
}
__device__ __forceinline__ uint32_t uniform_load_u32(const void* p) {
  typedef __attribute__((address_space(4))) const uint32_t cu32;
  return *(cu32*)uniform_ptr(p);
}
__device__ __forceinline__ float uniform_load_f32(const void* p) {
  typedef __attribute__((address_space(4))) const float cf32;
  return *(cf32*)uniform_ptr(p);
}

// World->local record (see nedf_compose_transforms): o_l = R^T o / s + c.
struct W2L {
  float rt[9];
  float c[3];
  float s, inv_s, pad0, pad1;
};

// Ray source: camera basis (float) or explicit arrays.
struct RaySrc {
  int kind;            // 0 camera, 1 arrays
  int width, height;
  float eye[3], fwd[3], right[3], up[3];  // right/up pre-scaled by the image-plane extents
  const float* o;
  const float* d;
};

// ---- compensated single-precision arithmetic --------------------------------
// Error-free transformations: a + b = s + e exactly (Knuth's two-sum) and
// a * b = p + e exactly (one fused multiply-add).  Contraction is off so that
// every operation stays as written.
struct f2 {
  float hi, lo;
};
__device__ __forceinline__ f2 two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
// |a| >= |b| (or a == 0): a + b = s + e exactly
__device__ __forceinline__ f2 fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ f2 two_prod(float a, float b) {
#pragma clang fp contract(off)
  const float p = a * b;
  return {p, fmaf(a, b, -p)};
}
// a0 v0 + a1 v1 + a2 v2 (+ a . vlo, first order) as hi + lo: the products
// exact, their sum with its rounding errors kept (error about 2^-44 of the
// sum of |terms|).
__device__ __forceinline__ f2 dot3_c(float a0, float a1, float a2, const float v[3], const float vlo[3]) {
#pragma clang fp contract(off)
  const f2 p0 = two_prod(a0, v[0]), p1 = two_prod(a1, v[1]), p2 = two_prod(a2, v[2]);
  const f2 s = two_sum(p0.hi, p1.hi);
  const f2 t = two_sum(s.hi, p2.hi);
  const float lo = ((p0.lo + p1.lo) + p2.lo) + (s.lo + t.lo) + ((a0 * vlo[0] + a1 * vlo[1]) + a2 * vlo[2]);
  return fast_two_sum(t.hi, lo);
}
// a1 b2 - a2 b1 for hi + lo operands, first order in the lo parts.
__device__ __forceinline__ f2 cross_c(f2 a1, f2 b2, f2 a2, f2 b1) {
#pragma clang fp contract(off)
  const f2 p = two_prod(a1.hi, b2.hi), q = two_prod(a2.hi, b1.hi);
  const f2 s = two_sum(p.hi, -q.hi);
  const float lo = s.lo + (p.lo - q.lo) + ((a1.hi * b2.lo + a1.lo * b2.hi) - (a2.hi * b1.lo + a2.lo * b1.hi));
  return fast_two_sum(s.hi, lo);
}

// Ray number `ray`: single-precision origin o and direction d, and the
// direction's residual dlo (d + dlo is the direction to about 2^-44; zero for
// ray arrays, which are exact as given).  A camera ray (Alg. 1: one ray
// through each pixel centre) is formed from the stored single-precision
// basis in compensated arithmetic: the pixel's image-plane coordinates
// u = (2i + 1 - W) / W and v = (H - 2j - 1) / H as hi + lo, the unnormalised
// direction fwd + u right + v up as hi + lo, and its reciprocal length by a
// single-precision square root refined with one Newton step on the residual,
// so that d is the faithfully rounded unit direction.
__device__ __forceinline__ void make_ray(const RaySrc& rs, int64_t ray, float o[3], float d[3], float dlo[3]) {
#pragma clang fp contract(off)
  if (rs.kind == 0) {
    const int i = int(ray % rs.width), j = int(ray / rs.width);
    const float W = float(rs.width), H = float(rs.height);
    const float nu = float(2 * i + 1 - rs.width), nv = float(rs.height - 2 * j - 1);  // exact integers
    const float uh = nu / W, vh = nv / H;
    const float ul = fmaf(-uh, W, nu) / W, vl = fmaf(-vh, H, nv) / H;  // exact remainders, divided
    f2 x[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const f2 p1 = two_prod(uh, rs.right[c]), p2 = two_prod(vh, rs.up[c]);
      const f2 s1 = two_sum(rs.fwd[c], p1.hi);
      const f2 s2 = two_sum(s1.hi, p2.hi);
      const float lo = (s1.lo + s2.lo) + (p1.lo + p2.lo) + (ul * rs.right[c] + vl * rs.up[c]);
      x[c] = fast_two_sum(s2.hi, lo);
    }
    // |x|^2 as hi + lo
    const f2 q0 = two_prod(x[0].hi, x[0].hi), q1 = two_prod(x[1].hi, x[1].hi), q2 = two_prod(x[2].hi, x[2].hi);
    const f2 a = two_sum(q0.hi, q1.hi);
    const f2 b = two_sum(a.hi, q2.hi);
    const float n2lo = ((q0.lo + q1.lo) + q2.lo) + (a.lo + b.lo) +
                       2.0f * ((x[0].hi * x[0].lo + x[1].hi * x[1].lo) + x[2].hi * x[2].lo);
    const f2 n2 = fast_two_sum(b.hi, n2lo);
    // r ~ 1/|x|; e = 1 - |x|^2 r^2 evaluated to the residual; 1/|x| = r (1 + e/2)
    const float r = 1.0f / sqrtf(n2.hi);
    const f2 rr = two_prod(r, r);
    const float t = fmaf(n2.hi, rr.hi, -1.0f);  // exact product, one rounding, |t| small
    const float e = -((t + n2.hi * rr.lo) + n2.lo * rr.hi);
    const float rlo = 0.5f * r * e;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const f2 p = two_prod(x[c].hi, r);
      const f2 dd = fast_two_sum(p.hi, p.lo + (x[c].hi * rlo + x[c].lo * r));
      d[c] = dd.hi;
      dlo[c] = dd.lo;
    }
    o[0] = rs.eye[0]; o[1] = rs.eye[1]; o[2] = rs.eye[2];
  } else {
    o[0] = rs.o[3 * ray + 0]; o[1] = rs.o[3 * ray + 1]; o[2] = rs.o[3 * ray + 2];
    d[0] = rs.d[3 * ray + 0]; d[1] = rs.d[3 * ray + 1]; d[2] = rs.d[3 * ray + 2];
    dlo[0] = dlo[1] = dlo[2] = 0.0f;
  }
}
__device__ __forceinline__ void make_ray(const RaySrc& rs, int64_t ray, float o[3], float d[3]) {
  float dlo[3];
  make_ray(rs, ray, o, d, dlo);
}

__device__ __forceinline__ void to_local(const W2L& g, const float o[3], const float d[3], float ol[3],
                                         float dl[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float a = g.rt[3 * r + 0] * o[0] + g.rt[3 * r + 1] * o[1] + g.rt[3 * r + 2] * o[2];
    ol[r] = fmaf(a, g.inv_s, g.c[r]);
    dl[r] = g.rt[3 * r + 0] * d[0] + g.rt[3 * r + 1] * d[1] + g.rt[3 * r + 2] * d[2];
  }
}

__device__ __forceinline__ W2L load_w2l(const float* w2l, int inst) {
  W2L g;
  const float4* p = reinterpret_cast<const float4*>(w2l + 16 * size_t(inst));
  float4 a = p[0], b = p[1], c = p[2], e = p[3];
  g.rt[0] = a.x; g.rt[1] = a.y; g.rt[2] = a.z; g.rt[3] = a.w;
  g.rt[4] = b.x; g.rt[5] = b.y; g.rt[6] = b.z; g.rt[7] = b.w;
  g.rt[8] = c.x; g.c[0] = c.y; g.c[1] = c.z; g.c[2] = c.w;
  g.s = e.x; g.inv_s = e.y; g.pad0 = e.z; g.pad1 = e.w;
  return g;
}

// The local ray's line (Eq. 1-2) from the single-precision record and a
// world ray (d + dlo), in compensated arithmetic: direction d_l = R^T d,
// moment o_l x d_l and t_perp = -o_l . d_l.  |o_l| can be tens of bounding
// radii while the moment of a candidate line is below one, so plain single
// precision would lose that ratio of digits to cancellation, and the
// encoding multiplies coordinate errors by up to 2^(L-1) pi.  Here each line
// coordinate comes as hi + lo (pl, pllo), its exact value in the record's and
// the ray's numbers to about 2^-44 relative to |o_l|; ol gets the rounded
// local origin.
__device__ __forceinline__ void local_line(const W2L& g, const float o[3], const float d[3], const float dlo[3],
                                           float pl[6], float pllo[6], float& tperp, float ol_out[3]) {
#pragma clang fp contract(off)
  const float zero[3] = {0.0f, 0.0f, 0.0f};
  f2 ol[3], dl[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float a0 = g.rt[3 * r + 0], a1 = g.rt[3 * r + 1], a2 = g.rt[3 * r + 2];
    const f2 a = dot3_c(a0, a1, a2, o, zero);
    const f2 q = two_prod(a.hi, g.inv_s);
    const float qlo = fmaf(a.lo, g.inv_s, q.lo);
    const f2 t = two_sum(q.hi, g.c[r]);
    ol[r] = fast_two_sum(t.hi, t.lo + qlo);
    dl[r] = dot3_c(a0, a1, a2, d, dlo);
    ol_out[r] = ol[r].hi;
    pl[r] = dl[r].hi;
    pllo[r] = dl[r].lo;
  }
  const f2 m0 = cross_c(ol[1], dl[2], ol[2], dl[1]);
  const f2 m1 = cross_c(ol[2], dl[0], ol[0], dl[2]);
  const f2 m2 = cross_c(ol[0], dl[1], ol[1], dl[0]);
  pl[3] = m0.hi; pllo[3] = m0.lo;
  pl[4] = m1.hi; pllo[4] = m1.lo;
  pl[5] = m2.hi; pllo[5] = m2.lo;
  const f2 p0 = two_prod(ol[0].hi, dl[0].hi), p1 = two_prod(ol[1].hi, dl[1].hi), p2 = two_prod(ol[2].hi, dl[2].hi);
  const f2 s = two_sum(p0.hi, p1.hi);
  const f2 t = two_sum(s.hi, p2.hi);
  const float lo = ((p0.lo + p1.lo) + p2.lo) + (s.lo + t.lo) +
                   ((ol[0].hi * dl[0].lo + ol[0].lo * dl[0].hi) + (ol[1].hi * dl[1].lo + ol[1].lo * dl[1].hi) +
                    (ol[2].hi * dl[2].lo + ol[2].lo * dl[2].hi));
  tperp = -(t.hi + lo);
}

// The points of the classifier-form network (16 points on the line around
// its tangency point): the tangency point p_perp = o_l + t_perp d_l
// (t_perp = -o_l . d_l) divided by l, and d_l, each as hi + lo from the same
// compensated record transform as local_line; point k is then
// q + c_k d_l with c_k = (2k + 1) / 16 - 1.
__device__ __forceinline__ void local_points_frame(const W2L& g, const float o[3], const float d[3],
                                                   const float dlo[3], float l, f2 q[3], f2 dv[3], float& tperp,
                                                   float ol_out[3]) {
#pragma clang fp contract(off)
  const float zero[3] = {0.0f, 0.0f, 0.0f};
  f2 ol[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float a0 = g.rt[3 * r + 0], a1 = g.rt[3 * r + 1], a2 = g.rt[3 * r + 2];
    const f2 a = dot3_c(a0, a1, a2, o, zero);
    const f2 qq = two_prod(a.hi, g.inv_s);
    const float qlo = fmaf(a.lo, g.inv_s, qq.lo);
    const f2 t = two_sum(qq.hi, g.c[r]);
    ol[r] = fast_two_sum(t.hi, t.lo + qlo);
    dv[r] = dot3_c(a0, a1, a2, d, dlo);
    ol_out[r] = ol[r].hi;
  }
  const f2 p0 = two_prod(ol[0].hi, dv[0].hi), p1 = two_prod(ol[1].hi, dv[1].hi), p2 = two_prod(ol[2].hi, dv[2].hi);
  const f2 s = two_sum(p0.hi, p1.hi);
  const f2 t = two_sum(s.hi, p2.hi);
  const float lo = ((p0.lo + p1.lo) + p2.lo) + (s.lo + t.lo) +
                   ((ol[0].hi * dv[0].lo + ol[0].lo * dv[0].hi) + (ol[1].hi * dv[1].lo + ol[1].lo * dv[1].hi) +
                    (ol[2].hi * dv[2].lo + ol[2].lo * dv[2].hi));
  const f2 tp = fast_two_sum(-t.hi, -lo);
  tperp = tp.hi;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const f2 pr = two_prod(tp.hi, dv[r].hi);
    const f2 sm = two_sum(ol[r].hi, pr.hi);
    const f2 pp = fast_two_sum(sm.hi, sm.lo + ((pr.lo + ol[r].lo) + (tp.hi * dv[r].lo + tp.lo * dv[r].hi)));
    const float qh = pp.hi / l;
    q[r] = {qh, (fmaf(-qh, l, pp.hi) + pp.lo) / l};
  }
}

// Line coordinates of a ray given in local space (o, d single precision,
// exact as given): the moment o x d with the same compensated cross product,
// as hi + lo.
__device__ __forceinline__ void line_of_local(const float o[3], const float d[3], float pl[6], float pllo[6],
                                              float& tperp) {
#pragma clang fp contract(off)
  const float zero[3] = {0.0f, 0.0f, 0.0f};
  const f2 O[3] = {{o[0], 0.f}, {o[1], 0.f}, {o[2], 0.f}}, D[3] = {{d[0], 0.f}, {d[1], 0.f}, {d[2], 0.f}};
  const f2 m0 = cross_c(O[1], D[2], O[2], D[1]);
  const f2 m1 = cross_c(O[2], D[0], O[0], D[2]);
  const f2 m2 = cross_c(O[0], D[1], O[1], D[0]);
  pl[0] = d[0]; pl[1] = d[1]; pl[2] = d[2];
  pllo[0] = pllo[1] = pllo[2] = 0.0f;
  pl[3] = m0.hi; pllo[3] = m0.lo;
  pl[4] = m1.hi; pllo[4] = m1.lo;
  pl[5] = m2.hi; pllo[5] = m2.lo;
  const f2 t = dot3_c(o[0], o[1], o[2], d, zero);
  tperp = -(t.hi + t.lo);
}

// Chord [a, b] of a unit-direction ray inside |x| <= radius, clipped to t >= 0.
__device__ __forceinline__ bool sphere_chord(const float ol[3], const float dl[3], float radius,
                                             float& a, float& b) {
  const float tp = -(ol[0] * dl[0] + ol[1] * dl[1] + ol[2] * dl[2]);
  const float oo = ol[0] * ol[0] + ol[1] * ol[1] + ol[2] * ol[2];
  const float h2 = radius * radius - (oo - tp * tp);
  if (!(h2 > 0.0f)) return false;
  const float h = sqrtf(h2);
  a = fmaxf(tp - h, 0.0f);
  b = tp + h;
  return b > a;
}

// sin(pi y) (h = 0) or cos(pi y) (h = 1) through the hardware sine
// (argument in revolutions) for y given as y + ylo (|ylo| tiny against one):
// y is first reduced exactly to r in [-1, 1] (y - 2 rint(y / 2) is exact for
// |y| < 2^23); the residual and the cosine's quarter-period shift join after
// the reduction, where the argument 0.5 r + (0.5 ylo + 0.25 h) rounds by at
// most 1.5 2^-25 revolutions, not before it, where it would round at the
// precision of y (2^-17 at y ~ 100).  One instruction serves both lane
// halves (sine and cosine lanes).
__device__ __forceinline__ float sinpi_hw(float y, float ylo, int h) {
  const float r = y - 2.0f * rintf(0.5f * y);
  return __builtin_amdgcn_sinf(fmaf(0.5f, r, fmaf(0.5f, ylo, 0.25f * float(h))));
}
__device__ __forceinline__ float sinpi_hw(float y, int h = 0) { return sinpi_hw(y, 0.0f, h); }

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

// log(1 + x) for 0 <= x <= 1: Taylor series below 1/16, else logf.
__device__ __forceinline__ float log1p_pos(float x) {
  if (x < 0.0625f) {
    // x - x^2/2 + x^3/3 - ... + x^7/7 (next term < 1e-9 relative)
    float p = 1.0f / 7.0f;
    p = fmaf(p, x, -1.0f / 6.0f);
    p = fmaf(p, x, 1.0f / 5.0f);
    p = fmaf(p, x, -1.0f / 4.0f);
    p = fmaf(p, x, 1.0f / 3.0f);
    p = fmaf(p, x, -0.5f);
    p = fmaf(p, x, 1.0f);
    return p * x;
  }
  return logf(1.0f + x);
}

// 1 - exp(-v) for v >= 0: Taylor series below 1/4, else 1 - expf(-v).
__device__ __forceinline__ float one_minus_exp_neg(float v) {
  if (v < 0.25f) {
    // v - v^2/2 + v^3/6 - ... - v^8/8! (next term < 1e-9 relative)
    float p = -1.0f / 40320.0f;
    p = fmaf(p, v, 1.0f / 5040.0f);
    p = fmaf(p, v, -1.0f / 720.0f);
    p = fmaf(p, v, 1.0f / 120.0f);
    p = fmaf(p, v, -1.0f / 24.0f);
    p = fmaf(p, v, 1.0f / 6.0f);
    p = fmaf(p, v, -0.5f);
    p = fmaf(p, v, 1.0f);
    return p * v;
  }
  return 1.0f - expf(-v);
}

__device__ __forceinline__ float softplusf_(float u) {
  return fmaxf(u, 0.0f) + log1p_pos(expf(-fabsf(u)));
}

// Packed (depth, id) key: ordering of non-negative float bits is the float
// ordering, so a 64-bit min keeps the smallest depth and, on equal depth, the
// lowest id.
__device__ __forceinline__ uint64_t pack_key(float depth, int id) {
  return (uint64_t(__float_as_uint(depth)) << 32) | uint64_t(uint32_t(id));
}

__device__ __forceinline__ void set_status(int* ws_status, int code) { atomicMax(ws_status, code); }

// Analytic signed distances of the SDF-biased shapes (must match the
// generator's shape list: sphere, rounded box, torus, ellipsoid).
__device__ __forceinline__ float sdf_shape(int shape, float x, float y, float z) {
  if (shape == 0) return sqrtf(x * x + y * y + z * z) - 0.6f;
  if (shape == 1) {
    const float qx = fabsf(x) - 0.4f, qy = fabsf(y) - 0.4f, qz = fabsf(z) - 0.4f;
    const float mx = fmaxf(qx, 0.f), my = fmaxf(qy, 0.f), mz = fmaxf(qz, 0.f);
    return sqrtf(mx * mx + my * my + mz * mz) + fminf(fmaxf(qx, fmaxf(qy, qz)), 0.f) - 0.05f;
  }
  if (shape == 2) {
    const float qx = sqrtf(x * x + z * z) - 0.5f;
    return sqrtf(qx * qx + y * y) - 0.2f;
  }
  const float ax = x / 0.7f, ay = y / 0.45f, az = z / 0.35f;
  const float bx = x / 0.49f, by = y / 0.2025f, bz = z / 0.1225f;
  const float k0 = sqrtf(ax * ax + ay * ay + az * az), k1 = sqrtf(bx * bx + by * by + bz * bz);
  return k1 > 0.f ? k0 * (k0 - 1.0f) / k1 : -0.35f;
}
