// Device layout of an intersection network's training state: float32 master
// weights and biases, Adam moments, last-step gradients and bfloat16 copies
// of every weight matrix for the matrix-core GEMMs, [N][Kpad] and transposed
// [Kpad][N] (K padded to a multiple of 64 with zeros).  Layer i is [N][K] row-major (PyTorch layout); layers
// 0..n_hidden-1 are the hidden layers, layer n_hidden the head.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "blob_layout.h"
#include "nedf.h"

struct nedf_train_layer {
  int32_t N, K, Kpad;
  size_t W, b, mW, vW, gW, mb, vb, gb, W16, W16T;  // byte offsets in the state buffer
};

struct nedf_train_layout {
  int32_t n_layers;
  nedf_train_layer L[NEDF_MAX_LAYERS + 1];
  size_t total;
};

static inline size_t nedf_tl_align(size_t x) { return (x + 255) & ~size_t(255); }

// Offset 0 holds the int64 Adam step counter (the number of updates made).
static inline nedf_train_layout nedf_train_layout_of(const nedf_mlp_shape& s) {
  nedf_train_layout t;
  const int n_in = (s.in_kind == NEDF_IN_PLUECKER ? 6 : 3) * (1 + 2 * s.enc_L);
  t.n_layers = s.n_hidden + 1;
  size_t off = 256;
  for (int i = 0; i < t.n_layers; ++i) {
    nedf_train_layer& l = t.L[i];
    l.N = i < s.n_hidden ? s.width : s.n_out;
    l.K = i == 0 ? n_in : s.width;
    l.Kpad = (l.K + 63) / 64 * 64;
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
