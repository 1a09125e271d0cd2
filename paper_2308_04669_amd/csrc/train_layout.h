// Device layout of an intersection network's training state: float32 master
// weights and biases, Adam moments, last-step gradients and bfloat16 copies
// of every weight matrix for the matrix-core GEMMs, [N][Kpad] and transposed
// [Kpad][N] (K padded to a multiple of 64 with zeros).  Layer i is [N][K] row-major (PyTorch layout); layers
// 0..n_hidden-1 are the hidden layers, layer n_hidden the head.  A
// classifier-form network (NEDF_IN_POINTS16) has the head, two layers per
// residual block and the tail, whose 193 rows are kept as 256 (rows past
// Nsrc stay zero: their gradients are zero).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "blob_layout.h"
#include "nedf.h"

#define NEDF_TRAIN_MAX_LAYERS 34  // classifier form with 16 residual blocks

struct nedf_train_layer {
  int32_t N, K, Kpad;
  int32_t Nsrc;  // rows of the caller's array (N, or 193 for the classifier tail)
  size_t W, b, mW, vW, gW, mb, vb, gb, W16, W16T;  // byte offsets in the state buffer
};

struct nedf_train_layout {
  int32_t n_layers;
  nedf_train_layer L[NEDF_TRAIN_MAX_LAYERS];
  size_t total;
};

static inline size_t nedf_tl_align(size_t x) { return (x + 255) & ~size_t(255); }

// Offset 0 holds the int64 Adam step counter (the number of updates made).
static inline nedf_train_layout nedf_train_layout_of(const nedf_mlp_shape& s) {
  nedf_train_layout t;
  const bool cls = s.in_kind == NEDF_IN_POINTS16;
  const int n_in = cls ? NEDF_CLS_POINTS * 3 * (1 + 2 * s.enc_L)
                       : (s.in_kind == NEDF_IN_PLUECKER ? 6 : 3) * (1 + 2 * s.enc_L);
  t.n_layers = cls ? 2 * s.n_hidden + 2 : s.n_hidden + 1;
  size_t off = 256;
  for (int i = 0; i < t.n_layers; ++i) {
    nedf_train_layer& l = t.L[i];
    const bool last = i == t.n_layers - 1;
    l.N = cls ? s.width : (last ? s.n_out : s.width);
    l.Nsrc = last ? s.n_out : l.N;
    l.K = i == 0 ? n_in : s.width;
    // the GEMMs take K in pairs of 64-deep stages and weight-gradient
    // tiles of 128 input columns
    l.Kpad = (l.K + 127) / 128 * 128;
    const size_t nw = size_t(l.N) * l.K * 4, nb = size_t(l.N) * 4;
    l.W = off; off = nedf_tl_align(off + nw);
    l.mW = off; off = nedf_tl_align(off + nw);
    l.vW = off; off = nedf_tl_align(off + nw);
    l.gW = off; off = nedf_tl_align(off + nw);
    l.b = off; off = nedf_tl_align(off + nb);
    l.mb = off; off = nedf_tl_align(off + nb);
    l.vb = off; off = nedf_tl_align(off + nb);
    l.gb = off; off = nedf_tl_align(off + nb);
    l.W16 = off; off = nedf_tl_align(off + size_t(l.N) * l.Kpad * 2);
    l.W16T = off; off = nedf_tl_align(off + size_t(l.N) * l.Kpad * 2);
  }
  t.total = off;
  return t;
}
