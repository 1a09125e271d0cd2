// Packed-network layout shared by the host packer and the HIP kernels.
//
// Register-resident MLP design.  A wave owns NB blocks of 32 samples.  Every
// layer is computed transposed, out^T[feature][sample] = W[feature][k] *
// act^T[k][sample], on 32x32 matrix-core tiles: weights are the A operand
// (32 output features x K-step), activations the B operand (K-step x 32
// samples), so lane l always holds sample (l % 32).  The accumulator of
// output block fb holds, in lane half h = l / 32 and register r (0..15),
// feature 32 fb + 8 (r / 4) + 4 h + (r % 4).  Those registers are re-used
// directly as the next layer's B operand; the K order this produces differs
// from the natural feature order, so the packer permutes the K columns of
// every layer's weights to match ("logical" k -> actual input feature).
//
// BF16 (v_mfma_f32_32x32x16_bf16): a K-step has 16 values, lane half h holds
//   logical k = 16 ks + 8 h + j (j = 0..7).  Output regs r of block fb become
//   K-step ks = 2 fb + r / 8, j = r % 8.
// F32 (v_mfma_f32_32x32x2_f32): a K-step has 2 values, lane half h holds
//   logical k = 2 ks + h.  Output reg r of block fb becomes K-step 16 fb + r.
//   Four consecutive K-steps of a lane share one 16-byte word (K-step counts
//   are rounded up to multiples of 4 with zero weights).
//
// First-layer inputs (the sinusoidal encoding) are computed in registers in an
// order chosen so that both lane halves do the same work: "argument slot" a
// holds level a / n, component a % n for a < n L, and the lane half selects
// sin (h = 0) or cos (h = 1) as sin(pi (2^level p + h / 2)); the identity
// components follow, two per slot (component 2 i + h), then zero padding.
// BF16 slot a sits at K-step a / 8, j = a % 8; F32 slot a is K-step a.
#pragma once
#include <stdint.h>

#define NEDF_BLOB_MAGIC 0x4644454Eu  // "NEDF"
#define NEDF_BLOB_VERSION 2u
#define NEDF_MAX_LAYERS 16

// A layer is stored as FB = out_width / 32 contiguous "chunks", one per output
// block, each chunk_bytes long:
//   [K-steps x fragment bytes: weights of the 32 output features]
//   [128 B: bias, [lane half h][16] float in accumulator order]
//   [heads x 128 B: narrow-head weights reading this block, [h][16] float]
// The last hidden layer carries the n_out head rows, the colour layer the
// 3 colour-head rows; other layers carry none.  A chunk is what one LDS
// buffer holds while the workgroup multiplies that output block.
// Offsets are bytes from the blob start; sections are 256-byte aligned.
struct nedf_blob_header {
  uint32_t magic, version, dtype, in_kind;
  uint32_t enc_L, width, n_hidden, n_out;
  uint32_t rgb_width, dir_L, n_in, n_dir;        // n_in: encoded input features
  uint32_t ks_in, ks_hidden, ks_rgb, frag_bytes;  // K-steps of first / hidden / colour layer
  uint32_t chunk_bytes[NEDF_MAX_LAYERS];          // per hidden layer
  uint32_t rgb_chunk_bytes, pad0;
  uint64_t off_layer[NEDF_MAX_LAYERS];  // first chunk of each hidden layer
  uint64_t off_head_b;                  // head bias [n_out] float
  uint64_t off_rgb;                     // first chunk of the colour layer
  uint64_t off_rgbh_b;                  // colour head bias [3] float
  uint64_t off_scales;                  // FP8: per hidden layer {w_scale, a_scale} float
  uint64_t total_bytes;
};

// ---- index maps (host and device) ----------------------------------------
// Feature held by accumulator register r of output block fb in lane half h.
static inline
#ifdef __HIPCC__
__host__ __device__
#endif
int nedf_acc_feature(int fb, int h, int r) { return 32 * fb + 8 * (r / 4) + 4 * h + (r % 4); }

// Number of argument slots (K-steps x lane halves / 2) of an encoded input of
// n components and L levels: n L sin/cos slots, then ceil(n / 2) identity slots.
static inline
#ifdef __HIPCC__
__host__ __device__
#endif
int nedf_enc_slots(int n, int L) { return n * L + (n + 1) / 2; }

// Actual encoding feature (natural order: [p, sin L0, cos L0, sin L1, ...],
// each block n wide) of slot a in lane half h, or -1 for padding.
static inline
#ifdef __HIPCC__
__host__ __device__
#endif
int nedf_enc_feature(int n, int L, int a, int h) {
  if (a < n * L) {
    int level = a / n, comp = a % n;
    return n + level * 2 * n + h * n + comp;
  }
  int i = a - n * L;
  int c = 2 * i + h;
  return (i < (n + 1) / 2 && c < n) ? c : -1;
}

// ---- classifier-form intersection network (in_kind NEDF_IN_POINTS16) --------
// Head: the 16 points' encodings are consumed point by point, so the head
// layer is stored as chunks that each cover a few K-steps of all 8 output
// blocks: chunk c, block fb, 16-byte LDS read r sits at (fb * 4 + r) * 1024
// (BF16: read r is K-step r of point c; F32: two chunks per point, read r
// holds K-steps 4 r .. 4 r + 3 of the chunk's 16).  A point's 32 argument
// slots follow the first-layer slot order above with n = 3.  Head bias:
// [block][lane half][16] float in accumulator order.  Residual layers: as
// hidden layers above (8 chunks of fragments + bias each).  Tail: 7 chunks,
// rows reordered to coarse bins 0..63, fine bins 64..191, hit logit 192,
// zero rows 193..223.
#define NEDF_CLS_MAGIC 0x534C434Eu  // "NCLS"
#define NEDF_CLS_POINTS 16
#define NEDF_CLS_COARSE 64
#define NEDF_CLS_FINE 128
#define NEDF_CLS_TAIL_BLOCKS 7
#define NEDF_CLS_HIT_ROW 192

struct nedf_cls_header {
  uint32_t magic, version, dtype, in_kind;
  uint32_t enc_L, width, n_blocks, n_points;
  uint32_t ks_point, ks_chunk, n_head_chunks, head_chunk_bytes;  // head: K-steps per point / per chunk
  uint32_t hidden_chunk_bytes, tail_chunk_bytes, pad0, pad1;
  uint64_t off_head, off_head_bias, off_hidden, hidden_layer_bytes, off_tail, total_bytes;
};
