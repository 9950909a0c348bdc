// Batched GN-MPPI over many independent chain MPC instances of uneven size
// (device-side descriptors and work tables shared by the batched kernels).
//
// Every step of an iteration is one launch per shape class (the template
// parameters -- lanes per sample, MFMA column tiles, sweep register tiles --
// split the batch into a few classes).  A launch is persistent: its grid is
// sized to the machine and each block walks a flattened list of work items
// (instance, tile), so instances of any size share the launch and no block
// idles on a short instance.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gnm {

// One instance as the batched kernels see it (float32 chain, LS Jacobian with
// the BF16x3 sample contraction, FP64 normal equations; J = S G^{-1} is not
// formed: the GGN system is solved in terms of S and G).
struct BatchInst {
  int M, N, K, n, m;      // masses, horizon, samples, decisions 2N, residuals N (4M + 2)
  int npad, kpad;         // n rounded up to 16; K rounded up to 32
  int nsplit, split_len;  // k-slices of S = dR W^T
  int grows;              // rows of G = W W^T below S in every k-slice (n, or 0)
  int gsplit, gsplit_len; // k-slices of G = W W^T
  int hchunk, hsplit;     // row chunks of [S r0]^T [S r0]
  int64_t ldw, ldr;       // leading dimensions of W (n x K) and R (m x K)
  uint64_t seed;          // Philox key of this instance
  const float* x0;
  const float* q;
  const float* r;
  const float* xref;
  float* U;
  int32_t* status;  // [0] Jacobian (G rank), [1] GGN (positive definite), [2] line search
  double* info;     // alpha*, C*, j* of the last line search
  float* W;
  float* R;
  float* C;       // null: the step needs no per-sample costs
  float* r0;
  float* c0;
  float* dU;      // n
  float* S;       // m x npad
  float* part;    // nsplit x m x npad (S partials)
  float* gpart;   // gsplit x n x npad (G partials)
  float* Ginv;    // n x npad
  __bf16* Wh;     // n x kpad
  __bf16* Wl;     // n x kpad
  double* Gsum;   // n x n
  double* hpart;  // hsplit x P x P, P = n + 1
  double* Hsum;   // P x P
  float* alpha;   // line-search step lengths (shared)
};

// Work item: instance index and tile index within that instance.
struct BatchItem {
  int inst, tile;
};

// A persistent launch: `count` items at `items` (device), grid of `blocks`.
struct BatchLaunch {
  const BatchItem* items;
  int count, blocks;
};

}  // namespace gnm
