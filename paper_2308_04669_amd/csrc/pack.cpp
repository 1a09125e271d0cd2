// Host-side packing of float32 network weights into the blob layout read by
// the matrix-core kernels (see blob_layout.h for the register layout).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "blob_layout.h"
#include "nedf.h"
#include "runtime.h"

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// float -> OCP E4M3FN code: nearest finite value, ties to the even code,
// saturating at +-448 (codes 0x00..0x7E for the magnitude).
uint8_t e4m3_rne(float f) {
  static double val[127];
  static bool init = false;
  if (!init) {
    for (int c = 0; c < 127; ++c) {
      const int e = c >> 3, m = c & 7;
      val[c] = e == 0 ? std::ldexp(m / 8.0, -6) : std::ldexp(1.0 + m / 8.0, e - 7);
    }
    init = true;
  }
  const double a = std::fabs(double(f));
  int best = 0;
  if (a >= 448.0) {
    best = 126;
  } else {
    int lo = 0;
    while (lo + 1 < 127 && val[lo + 1] <= a) ++lo;
    best = lo;
    if (lo + 1 < 127) {
      const double dl = a - val[lo], dh = val[lo + 1] - a;
      if (dh < dl || (dh == dl && ((lo + 1) & 1) == 0)) best = lo + 1;
    }
  }
  return uint8_t(best | (std::signbit(f) && best ? 0x80 : 0));
}

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

struct Plan {
  nedf_blob_header h;
  bool ok = false;
  std::string why;
};

int in_components(int in_kind) { return in_kind == NEDF_IN_PLUECKER ? 6 : 3; }

Plan plan_blob(const nedf_mlp_shape* s, int32_t dtype) {
  Plan p;
  std::memset(&p.h, 0, sizeof(p.h));
  if (!s) { p.why = "shape is NULL"; return p; }
  if (dtype != NEDF_F32 && dtype != NEDF_BF16 && dtype != NEDF_FP8 && dtype != NEDF_FP8_MX) {
    p.why = "dtype not supported by the packer";
    return p;
  }
  if (s->in_kind != NEDF_IN_XYZ && s->in_kind != NEDF_IN_PLUECKER) { p.why = "bad in_kind"; return p; }
  if (s->width != 64 && s->width != 256) { p.why = "width must be 64 or 256"; return p; }
  if (s->n_hidden < 2 || s->n_hidden > NEDF_MAX_LAYERS) { p.why = "n_hidden must be 2..16"; return p; }
  if (s->n_out < 1 || s->n_out > 2) { p.why = "n_out must be 1 or 2"; return p; }
  if (s->enc_L < 0 || s->enc_L > 12) { p.why = "enc_L must be 0..12"; return p; }
  if (s->rgb_width != 0 && s->rgb_width != 128) { p.why = "rgb_width must be 0 or 128"; return p; }
  if (s->rgb_width && (s->dir_L < 0 || s->dir_L > 8)) { p.why = "dir_L must be 0..8"; return p; }
  if (s->rgb_width && s->in_kind != NEDF_IN_XYZ) { p.why = "colour branch needs an xyz input"; return p; }
  nedf_blob_header& h = p.h;
  const bool bf = dtype == NEDF_BF16;
  const bool mx = dtype == NEDF_FP8_MX;
  const bool f8 = dtype == NEDF_FP8 || mx;
  if (f8 && s->rgb_width) { p.why = "FP8 packing covers networks without a colour branch"; return p; }
  if (mx && s->in_kind != NEDF_IN_PLUECKER) { p.why = "MX FP8 packing covers the intersection network"; return p; }
  const int n = in_components(s->in_kind);
  h.magic = NEDF_BLOB_MAGIC;
  h.version = NEDF_BLOB_VERSION;
  h.dtype = uint32_t(dtype);
  h.in_kind = uint32_t(s->in_kind);
  h.enc_L = uint32_t(s->enc_L);
  h.width = uint32_t(s->width);
  h.n_hidden = uint32_t(s->n_hidden);
  h.n_out = uint32_t(s->n_out);
  h.rgb_width = uint32_t(s->rgb_width);
  h.dir_L = uint32_t(s->dir_L);
  h.n_in = uint32_t(n * (1 + 2 * s->enc_L));
  h.n_dir = s->rgb_width ? uint32_t(3 * (1 + 2 * s->dir_L)) : 0u;
  const int slots = nedf_enc_slots(n, s->enc_L);
  auto round4 = [](int x) { return (x + 3) / 4 * 4; };
  h.ks_in = f8 ? uint32_t((slots + 31) / 32) : bf ? uint32_t((slots + 7) / 8) : uint32_t(round4(slots));
  h.ks_hidden = f8 ? uint32_t(s->width / 64) : bf ? uint32_t(s->width / 16) : uint32_t(s->width / 2);
  if (s->rgb_width) {
    const int dslots = nedf_enc_slots(3, s->dir_L);
    h.ks_rgb = h.ks_hidden + (bf ? uint32_t((dslots + 7) / 8) : uint32_t(round4(dslots)));
  }
  h.frag_bytes = f8 ? 2048u : bf ? 1024u : 256u;
  const size_t fbn = size_t(s->width / 32);
  size_t off = align256(sizeof(nedf_blob_header));
  for (int i = 0; i < s->n_hidden; ++i) {
    const size_t ks = i == 0 ? h.ks_in : h.ks_hidden;
    const size_t heads = i == s->n_hidden - 1 ? size_t(s->n_out) : 0;
    h.chunk_bytes[i] = uint32_t(ks * h.frag_bytes + (mx ? 1024 : 0) + 128 * (1 + heads));
    h.off_layer[i] = off;
    off = align256(off + fbn * h.chunk_bytes[i]);
  }
  h.off_head_b = off;
  off = align256(off + 16);
  if (s->rgb_width) {
    const size_t rfb = size_t(s->rgb_width / 32);
    h.rgb_chunk_bytes = uint32_t(h.ks_rgb * h.frag_bytes + 128 * (1 + 3));
    h.off_rgb = off;
    off = align256(off + rfb * h.rgb_chunk_bytes);
    h.off_rgbh_b = off;
    off = align256(off + 16);
  }
  h.off_scales = off;
  off = align256(off + (1 + 2 * NEDF_MAX_LAYERS) * 4);
  h.total_bytes = off;
  p.ok = true;
  return p;
}

int n_comp(const nedf_blob_header& h) { return h.in_kind == NEDF_IN_PLUECKER ? 6 : 3; }

// Actual input feature (or -1) of logical K index k.
//   part: 0 = encoded network input, 1 = previous hidden layer,
//         2 = colour layer (hidden features, then the direction encoding)
int logical_to_feature(const nedf_blob_header& h, int part, int k) {
  const bool bf = h.dtype == NEDF_BF16;
  const bool f8 = h.dtype == NEDF_FP8 || h.dtype == NEDF_FP8_MX;
  int ks, hh, j;
  if (f8) { ks = k / 64; hh = (k % 64) / 32; j = k % 32; }
  else if (bf) { ks = k / 16; hh = (k % 16) / 8; j = k % 8; }
  else { ks = k / 2; hh = k % 2; j = 0; }
  if (f8) {
    if (part == 0) {
      const int a = 32 * ks + j;
      if (a >= nedf_enc_slots(n_comp(h), int(h.enc_L))) return -1;
      return nedf_enc_feature(n_comp(h), int(h.enc_L), a, hh);
    }
    return nedf_acc_feature(2 * ks + j / 16, hh, j % 16);
  }
  const int n = h.in_kind == NEDF_IN_PLUECKER ? 6 : 3;
  if (part == 0) {
    const int a = bf ? 8 * ks + j : ks;
    if (a >= nedf_enc_slots(n, int(h.enc_L))) return -1;
    return nedf_enc_feature(n, int(h.enc_L), a, hh);
  }
  if (part == 2 && ks >= int(h.ks_hidden)) {
    const int kd = ks - int(h.ks_hidden);
    const int a = bf ? 8 * kd + j : kd;
    if (a >= nedf_enc_slots(3, int(h.dir_L))) return -1;
    const int f = nedf_enc_feature(3, int(h.dir_L), a, hh);
    return f < 0 ? -1 : int(h.width) + f;
  }
  const int fb = bf ? ks / 2 : ks / 16;
  const int r = bf ? (ks % 2) * 8 + j : ks % 16;
  return nedf_acc_feature(fb, hh, r);
}

// Write the fragments of one Linear layer W [rows][cols] (row-major).
void pack_fragments(const nedf_blob_header& h, int part, const float* W, int rows, int cols,
                    int ks_count, size_t chunk_bytes, uint8_t* dst, float w_scale = 1.0f) {
  const bool bf = h.dtype == NEDF_BF16;
  if (h.dtype == NEDF_FP8_MX) {
    // MX: per output row and K-step two blocks of 32 weights (bytes 16 b ..
    // 16 b + 15 of both lane halves), each with its own scale 2^e, the
    // smallest with amax / 2^e <= 448; lane l keeps the byte of block l / 32 at
    // [ks_count x 2 KB] + 16 l + ks
    for (int fb = 0; fb < rows / 32; ++fb)
      for (int ks = 0; ks < ks_count; ++ks) {
        uint8_t* frag = dst + size_t(fb) * chunk_bytes + size_t(ks) * 2048;
        uint8_t* scl = dst + size_t(fb) * chunk_bytes + size_t(ks_count) * 2048;
        for (int rr = 0; rr < 32; ++rr) {
          const int row = 32 * fb + rr;
          for (int b = 0; b < 2; ++b) {
            float vals[2][16];
            double amax = 0.0;
            for (int hh = 0; hh < 2; ++hh)
              for (int i = 0; i < 16; ++i) {
                const int k = 64 * ks + 32 * hh + 16 * b + i;
                const int f = logical_to_feature(h, part, k);
                const float v = (f >= 0 && f < cols) ? W[size_t(row) * cols + f] : 0.0f;
                vals[hh][i] = v;
                amax = std::max(amax, std::fabs(double(v)));
              }
            int byte = 0;
            double X = 1.0;
            if (amax > 0.0 && std::isfinite(amax)) {
              int ex = 0;
              std::frexp(amax, &ex);  // amax = m 2^ex, 0.5 <= m < 1: floor(log2 amax) = ex - 1
              int e0 = ex - 1 - 8;
              if (amax / std::ldexp(1.0, e0) > 448.0) ++e0;
              const int e = std::min(std::max(e0, -127), 127);
              byte = e + 127;
              X = std::ldexp(1.0, e);
            }
            for (int hh = 0; hh < 2; ++hh) {
              const int l = rr + 32 * hh;
              for (int i = 0; i < 16; ++i)
                frag[((16 * b + i) / 16) * 1024 + l * 16 + ((16 * b + i) % 16)] = e4m3_rne(float(vals[hh][i] / X));
              if (hh == b) scl[l * 16 + ks] = uint8_t(byte);
            }
          }
        }
      }
    return;
  }
  if (h.dtype == NEDF_FP8) {
    // FP8: lane l of K-step ks holds 32 bytes k = 64 ks + 32 (l / 32) + j;
    // bytes 0..15 in the first 1 KB half of the fragment, 16..31 in the second
    for (int fb = 0; fb < rows / 32; ++fb)
      for (int ks = 0; ks < ks_count; ++ks) {
        uint8_t* frag = dst + size_t(fb) * chunk_bytes + size_t(ks) * 2048;
        for (int l = 0; l < 64; ++l) {
          const int row = 32 * fb + (l % 32);
          for (int jj = 0; jj < 32; ++jj) {
            const int k = 64 * ks + 32 * (l / 32) + jj;
            const int f = logical_to_feature(h, part, k);
            const float v = (f >= 0 && f < cols) ? W[size_t(row) * cols + f] / w_scale : 0.0f;
            frag[(jj / 16) * 1024 + l * 16 + (jj % 16)] = e4m3_rne(v);
          }
        }
      }
    return;
  }
  const int fbn = rows / 32;
  for (int fb = 0; fb < fbn; ++fb)
    for (int ks = 0; ks < ks_count; ++ks) {
      uint8_t* frag = dst + size_t(fb) * chunk_bytes + size_t(ks) * h.frag_bytes;
      for (int l = 0; l < 64; ++l) {
        const int row = 32 * fb + (l % 32);
        if (bf) {
          uint16_t* out = reinterpret_cast<uint16_t*>(frag) + l * 8;
          for (int jj = 0; jj < 8; ++jj) {
            const int k = 16 * ks + 8 * (l / 32) + jj;
            const int f = logical_to_feature(h, part, k);
            out[jj] = (f >= 0 && f < cols) ? bf16_rne(W[size_t(row) * cols + f]) : uint16_t(0);
          }
        } else {
          // F32: four consecutive K-steps share one 16-byte lane word
          float* out = reinterpret_cast<float*>(dst + size_t(fb) * chunk_bytes + size_t(ks / 4) * 1024 +
                                                size_t(l) * 16 + size_t(ks % 4) * 4);
          const int k = 2 * ks + (l / 32);
          const int f = logical_to_feature(h, part, k);
          *out = (f >= 0 && f < cols) ? W[size_t(row) * cols + f] : 0.0f;
        }
      }
    }
}

// Bias of every output block, placed after the block's fragments (divided by
// the layer's to-real multiplier for FP8, whose accumulators are in scaled units).
void pack_bias(const float* b, int rows, int ks_count, int frag_bytes, size_t chunk_bytes, uint8_t* dst,
               float to_real = 1.0f, int extra = 0) {
  for (int fb = 0; fb < rows / 32; ++fb) {
    float* out = reinterpret_cast<float*>(dst + size_t(fb) * chunk_bytes + size_t(ks_count) * frag_bytes + extra);
    for (int hh = 0; hh < 2; ++hh)
      for (int r = 0; r < 16; ++r) out[hh * 16 + r] = b[nedf_acc_feature(fb, hh, r)] / to_real;
  }
}

// Narrow head W [n_out][in_width]: row o's weights of input block fb follow
// that block's bias, [h][16] in accumulator order.
void pack_head(const float* W, int n_out, int in_width, int ks_count, int frag_bytes, size_t chunk_bytes,
               uint8_t* dst, int extra = 0) {
  for (int fb = 0; fb < in_width / 32; ++fb)
    for (int o = 0; o < n_out; ++o) {
      float* out = reinterpret_cast<float*>(dst + size_t(fb) * chunk_bytes + size_t(ks_count) * frag_bytes + extra +
                                            128 * (1 + o));
      for (int hh = 0; hh < 2; ++hh)
        for (int r = 0; r < 16; ++r) out[hh * 16 + r] = W[size_t(o) * in_width + nedf_acc_feature(fb, hh, r)];
    }
}

// ---- classifier-form intersection network ------------------------------------
struct ClsPlan {
  nedf_cls_header h;
  nedf_blob_header hb;  // dtype-only header for the shared fragment packer
  bool ok = false;
  std::string why;
};

ClsPlan plan_cls(const nedf_mlp_shape* s, int32_t dtype) {
  ClsPlan p;
  std::memset(&p.h, 0, sizeof(p.h));
  std::memset(&p.hb, 0, sizeof(p.hb));
  if (dtype != NEDF_F32 && dtype != NEDF_BF16) { p.why = "classifier networks pack as F32 or BF16"; return p; }
  if (s->width != 256) { p.why = "classifier width must be 256"; return p; }
  if (s->enc_L != 10) { p.why = "classifier encoding must have 10 levels"; return p; }
  if (s->n_hidden < 1 || s->n_hidden > 64) { p.why = "residual blocks must be 1..64"; return p; }
  if (s->n_out != 1 + NEDF_CLS_COARSE + NEDF_CLS_FINE) { p.why = "classifier n_out must be 193"; return p; }
  if (s->rgb_width) { p.why = "classifier networks have no colour branch"; return p; }
  const bool bf = dtype == NEDF_BF16;
  nedf_cls_header& h = p.h;
  h.magic = NEDF_CLS_MAGIC;
  h.version = 1;
  h.dtype = uint32_t(dtype);
  h.in_kind = NEDF_IN_POINTS16;
  h.enc_L = uint32_t(s->enc_L);
  h.width = uint32_t(s->width);
  h.n_blocks = uint32_t(s->n_hidden);
  h.n_points = NEDF_CLS_POINTS;
  const int slots = nedf_enc_slots(3, s->enc_L);  // 32
  h.ks_point = bf ? uint32_t(slots / 8) : uint32_t(slots);
  h.ks_chunk = bf ? 4u : 16u;
  h.n_head_chunks = NEDF_CLS_POINTS * h.ks_point / h.ks_chunk;
  const uint32_t frag = bf ? 1024u : 256u;
  h.head_chunk_bytes = 8u * h.ks_chunk * frag;
  const uint32_t ksh = bf ? uint32_t(s->width / 16) : uint32_t(s->width / 2);
  h.hidden_chunk_bytes = ksh * frag + 128u;
  h.tail_chunk_bytes = h.hidden_chunk_bytes;
  size_t off = align256(sizeof(nedf_cls_header));
  h.off_head = off;
  off = align256(off + size_t(h.n_head_chunks) * h.head_chunk_bytes);
  h.off_head_bias = off;
  off = align256(off + 1024);
  h.off_hidden = off;
  h.hidden_layer_bytes = align256(size_t(8) * h.hidden_chunk_bytes);
  off += size_t(2 * s->n_hidden) * h.hidden_layer_bytes;
  h.off_tail = off;
  off = align256(off + size_t(NEDF_CLS_TAIL_BLOCKS) * h.tail_chunk_bytes);
  h.total_bytes = off;
  p.hb.dtype = uint32_t(dtype);
  p.hb.frag_bytes = frag;
  p.hb.ks_hidden = ksh;
  p.ok = true;
  return p;
}

// Head fragments: column 63 p + e of W is feature e of point p's encoding.
void pack_cls_head(const nedf_cls_header& h, const float* W, int cols, uint8_t* dst) {
  const bool bf = h.dtype == NEDF_BF16;
  const int per_point = 3 * (1 + 2 * int(h.enc_L));
  const int cpp = int(h.ks_point / h.ks_chunk);  // chunks per point
  const int slots = nedf_enc_slots(3, int(h.enc_L));
  for (uint32_t c = 0; c < h.n_head_chunks; ++c) {
    const int pt = int(c) / cpp;
    const int ks0 = (int(c) % cpp) * int(h.ks_chunk);
    uint8_t* chunk = dst + size_t(c) * h.head_chunk_bytes;
    for (int fb = 0; fb < 8; ++fb)
      for (int r = 0; r < 4; ++r) {
        uint8_t* rd = chunk + size_t(fb * 4 + r) * 1024;
        for (int l = 0; l < 64; ++l) {
          const int row = 32 * fb + (l % 32), hh = l / 32;
          if (bf) {
            uint16_t* out = reinterpret_cast<uint16_t*>(rd + l * 16);
            for (int j = 0; j < 8; ++j) {
              const int a = 8 * (ks0 + r) + j;
              const int f = a < slots ? nedf_enc_feature(3, int(h.enc_L), a, hh) : -1;
              const int col = f < 0 ? -1 : per_point * pt + f;
              out[j] = (col >= 0 && col < cols) ? bf16_rne(W[size_t(row) * cols + col]) : uint16_t(0);
            }
          } else {
            float* out = reinterpret_cast<float*>(rd + l * 16);
            for (int i = 0; i < 4; ++i) {
              const int a = ks0 + 4 * r + i;
              const int f = a < slots ? nedf_enc_feature(3, int(h.enc_L), a, hh) : -1;
              const int col = f < 0 ? -1 : per_point * pt + f;
              out[i] = (col >= 0 && col < cols) ? W[size_t(row) * cols + col] : 0.0f;
            }
          }
        }
      }
  }
}

int32_t pack_cls(const nedf_mlp_shape* shape, int32_t dtype, const float* const* W, const float* const* b,
                 void* out, size_t out_bytes) {
  ClsPlan p = plan_cls(shape, dtype);
  if (!p.ok) return nedf::fail(NEDF_ERR_SHAPE, "nedf_pack_mlp: " + p.why);
  const nedf_cls_header& h = p.h;
  if (out_bytes < h.total_bytes) return nedf::fail(NEDF_ERR_WORKSPACE, "nedf_pack_mlp: output buffer too small");
  const int nl = 2 * shape->n_hidden + 2;
  for (int i = 0; i < nl; ++i)
    if (!W[i] || !b[i]) return nedf::fail(NEDF_ERR_NULL, "nedf_pack_mlp: NULL layer pointer");
  uint8_t* base = static_cast<uint8_t*>(out);
  std::memset(base, 0, h.total_bytes);
  std::memcpy(base, &h, sizeof(h));
  const int Wd = shape->width;
  const int in_cols = NEDF_CLS_POINTS * 3 * (1 + 2 * shape->enc_L);
  pack_cls_head(h, W[0], in_cols, base + h.off_head);
  float* hb = reinterpret_cast<float*>(base + h.off_head_bias);
  for (int fb = 0; fb < 8; ++fb)
    for (int hh = 0; hh < 2; ++hh)
      for (int r = 0; r < 16; ++r) hb[(fb * 2 + hh) * 16 + r] = b[0][nedf_acc_feature(fb, hh, r)];
  const int ksh = int(p.hb.ks_hidden), fragb = int(p.hb.frag_bytes);
  for (int i = 0; i < 2 * shape->n_hidden; ++i) {
    uint8_t* dst = base + h.off_hidden + size_t(i) * h.hidden_layer_bytes;
    pack_fragments(p.hb, 1, W[1 + i], Wd, Wd, ksh, h.hidden_chunk_bytes, dst);
    pack_bias(b[1 + i], Wd, ksh, fragb, h.hidden_chunk_bytes, dst);
  }
  // tail rows in kernel order: coarse, fine, hit logit, zeros
  const int rows = 32 * NEDF_CLS_TAIL_BLOCKS;
  std::vector<float> Wt(size_t(rows) * Wd, 0.0f), bt(rows, 0.0f);
  const float* Ws = W[nl - 1];
  const float* bs = b[nl - 1];
  for (int r = 0; r < rows; ++r) {
    int src = -1;
    if (r < NEDF_CLS_COARSE + NEDF_CLS_FINE) src = 1 + r;
    else if (r == NEDF_CLS_HIT_ROW) src = 0;
    if (src < 0) continue;
    std::memcpy(&Wt[size_t(r) * Wd], Ws + size_t(src) * Wd, sizeof(float) * Wd);
    bt[r] = bs[src];
  }
  uint8_t* dst = base + h.off_tail;
  pack_fragments(p.hb, 1, Wt.data(), rows, Wd, ksh, h.tail_chunk_bytes, dst);
  pack_bias(bt.data(), rows, ksh, fragb, h.tail_chunk_bytes, dst);
  return NEDF_OK;
}

}  // namespace

extern "C" size_t nedf_mlp_packed_bytes(const nedf_mlp_shape* shape, int32_t dtype) {
  if (shape && shape->in_kind == NEDF_IN_POINTS16) {
    ClsPlan c = plan_cls(shape, dtype);
    if (!c.ok) {
      nedf::set_error(c.why);
      return 0;
    }
    return size_t(c.h.total_bytes);
  }
  Plan p = plan_blob(shape, dtype);
  if (!p.ok) {
    nedf::set_error(p.why);
    return 0;
  }
  return size_t(p.h.total_bytes);
}

extern "C" int32_t nedf_pack_mlp(const nedf_mlp_shape* shape, int32_t dtype, const float* const* W,
                                 const float* const* b, const float* fp8_scales, void* out,
                                 size_t out_bytes) {
  if (!shape || !W || !b || !out) return nedf::fail(NEDF_ERR_NULL, "nedf_pack_mlp: NULL argument");
  if (shape->in_kind == NEDF_IN_POINTS16) return pack_cls(shape, dtype, W, b, out, out_bytes);
  if (dtype == NEDF_FP8 && !fp8_scales) return nedf::fail(NEDF_ERR_NULL, "nedf_pack_mlp: FP8 needs per-layer scales");
  Plan p = plan_blob(shape, dtype);
  if (!p.ok) return nedf::fail(dtype == NEDF_F32 || dtype == NEDF_BF16 ? NEDF_ERR_SHAPE : NEDF_ERR_DTYPE,
                               "nedf_pack_mlp: " + p.why);
  const nedf_blob_header& h = p.h;
  if (out_bytes < h.total_bytes) return nedf::fail(NEDF_ERR_WORKSPACE, "nedf_pack_mlp: output buffer too small");
  const int n_layers = shape->n_hidden + 1 + (shape->rgb_width ? 2 : 0);
  for (int i = 0; i < n_layers; ++i)
    if (!W[i] || !b[i]) return nedf::fail(NEDF_ERR_NULL, "nedf_pack_mlp: NULL layer pointer");
  uint8_t* base = static_cast<uint8_t*>(out);
  std::memset(base, 0, h.total_bytes);
  std::memcpy(base, &h, sizeof(h));
  const int Wd = shape->width;
  const int fragb = int(h.frag_bytes);
  const bool f8 = dtype == NEDF_FP8;
  const int extra = dtype == NEDF_FP8_MX ? 1024 : 0;  // MX weight-block scales after the fragments
  float* sc = reinterpret_cast<float*>(base + h.off_scales);
  if (f8) {
    // scales: [0] 1 / a_0, then per layer {a_L w_L (to real), 1 / a_{L+1}}
    for (int i = 0; i < shape->n_hidden; ++i)
      if (!(fp8_scales[2 * i] > 0.0f) || !(fp8_scales[2 * i + 1] > 0.0f))
        return nedf::fail(NEDF_ERR_SHAPE, "nedf_pack_mlp: FP8 scales must be positive");
    sc[0] = 1.0f / fp8_scales[1];
    for (int i = 0; i < shape->n_hidden; ++i) {
      sc[1 + 2 * i] = fp8_scales[2 * i] * fp8_scales[2 * i + 1];
      sc[2 + 2 * i] = i + 1 < shape->n_hidden ? 1.0f / fp8_scales[2 * (i + 1) + 1] : 1.0f;
    }
  }
  for (int i = 0; i < shape->n_hidden; ++i) {
    const int cols = i == 0 ? int(h.n_in) : Wd;
    const int ks = int(i == 0 ? h.ks_in : h.ks_hidden);
    uint8_t* dst = base + h.off_layer[i];
    pack_fragments(h, i == 0 ? 0 : 1, W[i], Wd, cols, ks, h.chunk_bytes[i], dst, f8 ? fp8_scales[2 * i] : 1.0f);
    pack_bias(b[i], Wd, ks, fragb, h.chunk_bytes[i], dst, f8 ? sc[1 + 2 * i] : 1.0f, extra);
    if (i == shape->n_hidden - 1)
      pack_head(W[shape->n_hidden], shape->n_out, Wd, ks, fragb, h.chunk_bytes[i], dst, extra);
  }
  std::memcpy(base + h.off_head_b, b[shape->n_hidden], sizeof(float) * shape->n_out);
  if (shape->rgb_width) {
    const int rw = shape->rgb_width;
    uint8_t* dst = base + h.off_rgb;
    pack_fragments(h, 2, W[shape->n_hidden + 1], rw, Wd + int(h.n_dir), int(h.ks_rgb), h.rgb_chunk_bytes, dst);
    pack_bias(b[shape->n_hidden + 1], rw, int(h.ks_rgb), fragb, h.rgb_chunk_bytes, dst);
    pack_head(W[shape->n_hidden + 2], 3, rw, int(h.ks_rgb), fragb, h.rgb_chunk_bytes, dst);
    std::memcpy(base + h.off_rgbh_b, b[shape->n_hidden + 2], sizeof(float) * 3);
  }
  return NEDF_OK;
}
