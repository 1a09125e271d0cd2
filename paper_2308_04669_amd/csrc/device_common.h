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

__device__ __forceinline__ void make_ray(const RaySrc& rs, int64_t ray, float o[3], float d[3]) {
  if (rs.kind == 0) {
    const int i = int(ray % rs.width), j = int(ray / rs.width);
    const float u = 2.0f * (float(i) + 0.5f) / float(rs.width) - 1.0f;
    const float v = 1.0f - 2.0f * (float(j) + 0.5f) / float(rs.height);
    float x = fmaf(u, rs.right[0], fmaf(v, rs.up[0], rs.fwd[0]));
    float y = fmaf(u, rs.right[1], fmaf(v, rs.up[1], rs.fwd[1]));
    float z = fmaf(u, rs.right[2], fmaf(v, rs.up[2], rs.fwd[2]));
    const float inv = 1.0f / sqrtf(x * x + y * y + z * z);
    d[0] = x * inv; d[1] = y * inv; d[2] = z * inv;
    o[0] = rs.eye[0]; o[1] = rs.eye[1]; o[2] = rs.eye[2];
  } else {
    o[0] = rs.o[3 * ray + 0]; o[1] = rs.o[3 * ray + 1]; o[2] = rs.o[3 * ray + 2];
    d[0] = rs.d[3 * ray + 0]; d[1] = rs.d[3 * ray + 1]; d[2] = rs.d[3 * ray + 2];
  }
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

// sin(pi * y) through the hardware sine (argument in revolutions) after an
// exact reduction of y to [-1, 1].
__device__ __forceinline__ float sinpi_hw(float y) {
  const float r = y - 2.0f * rintf(0.5f * y);  // exact for |y| < 2^23
  return __builtin_amdgcn_sinf(0.5f * r);
}

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
